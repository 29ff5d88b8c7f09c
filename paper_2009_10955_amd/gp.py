"""Python binding of libgp.so (the C ABI in include/gp.h).

Argument marshalling only: every step of the counting path runs in the HIP
library. PyTorch supplies device memory and streams. If the library is not
built, importing works but every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgp.so")
MAX_K = 8

GP_IN_DEVICE = 1
GP_NO_HUB_BITMAPS = 2
GP_DENSE_HUB_BITMAPS = 4

STATUS = {
    0: "GP_OK", -1: "GP_ERR_ARG", -2: "GP_ERR_CSR_UNSORTED", -3: "GP_ERR_CSR_ASYMMETRIC",
    -4: "GP_ERR_CSR_SELFLOOP", -5: "GP_ERR_CSR_DUPLICATE", -6: "GP_ERR_PATTERN",
    -7: "GP_ERR_NOMEM", -8: "GP_ERR_HIP", -9: "GP_ERR_OVERFLOW", -10: "GP_ERR_BUDGET",
    -11: "GP_ERR_CSR_RANGE", -12: "GP_ERR_UNSUPPORTED", -13: "GP_ERR_TIMEOUT",
    -14: "GP_ERR_INTERNAL",
}


class GpError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        msg = _lib().gp_strerror(status).decode() if _LIB is not None else self.name
        super().__init__(f"{what}: {self.name} ({msg})" if what else f"{self.name} ({msg})")


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("tri_cnt", ctypes.c_uint64), ("hash", ctypes.c_uint64),
                ("load_seconds", ctypes.c_double), ("hub_vertices", ctypes.c_int64),
                ("hub_bitmap_bytes", ctypes.c_int64)]


class LoadOpts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("hub_min_degree", ctypes.c_int64),
                ("hub_budget_bytes", ctypes.c_int64)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("max_states", ctypes.c_int64), ("max_sets", ctypes.c_int32),
                ("force_order", ctypes.c_int32 * MAX_K), ("force_set", ctypes.c_int32),
                ("n_force_restr", ctypes.c_int32),
                ("force_restr", ctypes.c_int32 * (2 * MAX_K * MAX_K)),
                ("cost_cap", ctypes.c_double), ("max_seconds", ctypes.c_double),
                ("iep", ctypes.c_int32)]


class Launch(ctypes.Structure):
    _fields_ = [("group", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("leaf_mode", ctypes.c_int32),
                ("root_stride", ctypes.c_int32), ("root_offset", ctypes.c_int32),
                ("split_ways", ctypes.c_int32), ("split_vertices", ctypes.c_int32),
                ("xcd_tasks", ctypes.c_int32), ("batch_runs", ctypes.c_int32)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("max_configs", ctypes.c_int32), ("sample_stride", ctypes.c_int32),
                ("tune_launch", ctypes.c_int32), ("budget_seconds", ctypes.c_double),
                ("try_iep", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("target_ms", ctypes.c_double),
                ("cost_cap", ctypes.c_double), ("initial_slice", ctypes.c_int64),
                ("group", ctypes.c_int32), ("leaf_mode", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("max_query_ms", ctypes.c_double),
                ("iep", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("iterations", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("busy_seconds", ctypes.c_double), ("joined_midflight", ctypes.c_int64),
                ("max_batch", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("order", ctypes.c_int32 * MAX_K),
                ("n_restr", ctypes.c_int32), ("restr", ctypes.c_int32 * (2 * MAX_K * MAX_K)),
                ("aut", ctypes.c_uint64), ("cost", ctypes.c_double), ("n_sets", ctypes.c_int32),
                ("n_states", ctypes.c_int64), ("n_schedules", ctypes.c_int32),
                ("k_eff", ctypes.c_int32), ("set_index", ctypes.c_int32),
                ("plan_seconds", ctypes.c_double), ("tuned", ctypes.c_int32),
                ("iep", ctypes.c_int32), ("iep_div", ctypes.c_int32),
                ("n_measured", ctypes.c_int32), ("launch", Launch), ("tuned_ms", ctypes.c_double)]




# every symbol include/gp.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
SIGNATURES = {
    "gp_load_graph": (_I32, [_P, _P, _I64, _I64, ctypes.c_uint32, _P, ctypes.POINTER(_P)]),
    "gp_load_opts_default": (None, [ctypes.POINTER(LoadOpts)]),
    "gp_load_graph_opts": (_I32, [_P, _P, _I64, _I64, ctypes.POINTER(LoadOpts), _P, ctypes.POINTER(_P)]),
    "gp_graph_stats": (_I32, [_P, ctypes.POINTER(Stats)]),
    "gp_graph_new_id": (_I32, [_P, _P]),
    "gp_graph_layout": (_I32, [_P, _P, _P]),
    "gp_free_graph": (None, [_P]),
    "gp_plan_opts_default": (None, [ctypes.POINTER(PlanOpts)]),
    "gp_plan_create": (_I32, [_P, _I32, _I32, ctypes.POINTER(Stats), ctypes.POINTER(PlanOpts),
                              ctypes.POINTER(_P)]),
    "gp_plan_get": (_I32, [_P, ctypes.POINTER(PlanInfo)]),
    "gp_plan_get_set": (_I32, [_P, _I32, ctypes.POINTER(_I32), _P]),
    "gp_plan_get_schedule": (_I32, [_P, _I32, _P]),
    "gp_plan_model_cost": (_I32, [_P, _I32, _I32, ctypes.POINTER(Stats),
                                  ctypes.POINTER(ctypes.c_double)]),
    "gp_free_plan": (None, [_P]),
    "gp_tune_opts_default": (None, [ctypes.POINTER(TuneOpts)]),
    "gp_plan_tune": (_I32, [_P, _P, ctypes.POINTER(TuneOpts), _P, ctypes.POINTER(_P)]),
    "gp_plan_with_launch": (_I32, [_P, ctypes.POINTER(Launch), ctypes.POINTER(_P)]),
    "gp_launch_default": (None, [ctypes.POINTER(Launch)]),
    "gp_count": (_I32, [_P, _P, ctypes.POINTER(Launch), _P, ctypes.POINTER(ctypes.c_uint64)]),
    "gp_count_async": (_I32, [_P, _P, ctypes.POINTER(Launch), _P, _P]),
    "gp_count_noalloc": (_I32, [_P, _P, ctypes.POINTER(Launch), _P, _P]),
    "gp_count_per_root": (_I32, [_P, _P, ctypes.POINTER(Launch), _P, _P,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "gp_count_batch": (_I32, [_P, _P, _I32, ctypes.POINTER(Launch), _P, _P]),
    "gp_estimate": (_I32, [_P, _P, ctypes.POINTER(Launch), ctypes.c_double, _P,
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64),
                           ctypes.POINTER(_I64)]),
    "gp_list": (_I32, [_P, _P, ctypes.POINTER(Launch), _P, _P, ctypes.c_uint64,
                       ctypes.POINTER(ctypes.c_uint64)]),
    "gp_count_traffic": (_I32, [_P, _P, ctypes.POINTER(Launch), _P,
                                ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "gp_check_sum": (_I32, [_P, _I64, ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_uint64),
                            ctypes.POINTER(ctypes.c_uint32)]),
    "gp_batch_create": (_I32, [_P, _P, _I32, ctypes.POINTER(Launch), _P, ctypes.POINTER(_P)]),
    "gp_batch_tune": (_I32, [_P, _P, _I32, _P, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_double)]),
    "gp_batch_run": (_I32, [_P, _P, _P]),
    "gp_batch_set_sample": (_I32, [_P, _I64, _I64, _P]),
    "gp_free_batch": (None, [_P]),
    "gp_server_opts_default": (None, [ctypes.POINTER(ServerOpts)]),
    "gp_server_create": (_I32, [_P, _I32, ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]),
    "gp_server_submit": (_I32, [_P, _I32, _P, _I32, _I32, ctypes.POINTER(ctypes.c_uint64)]),
    "gp_server_poll": (_I32, [_P, ctypes.c_uint64, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                              ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)]),
    "gp_server_wait": (_I32, [_P, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_I32),
                              ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)]),
    "gp_server_stats_get": (_I32, [_P, ctypes.POINTER(ServerStats)]),
    "gp_server_destroy": (None, [_P]),
    "gp_strerror": (ctypes.c_char_p, [_I32]),
    "gp_version": (ctypes.c_char_p, []),
}

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (loads it on first use)."""
    return _lib()


def _check(status: int, what: str) -> None:
    if status != 0:
        raise GpError(status, what)


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _launch(group=0, waves_per_cu=0, chunk=0, leaf_mode=0, root_stride=0, root_offset=0,
            split_ways=0, split_vertices=0, xcd_tasks=0, batch_runs=0) -> Launch:
    return Launch(group, waves_per_cu, chunk, leaf_mode, root_stride, root_offset, split_ways,
                  split_vertices, xcd_tasks, batch_runs)


class Graph:
    """A data graph resident on the current GPU, owned by the library."""

    def __init__(self, row_ptr, col, stream=None, hub_bitmaps: str = "auto", hub_min_degree: int = 0,
                 hub_budget_bytes: int = 0):
        """hub_bitmaps: "auto" (degree >= hub_min_degree, default 64, within
        hub_budget_bytes, default 8 GiB), "none", or "dense" (every vertex)."""
        lib = _lib()
        extra = {"auto": 0, "none": GP_NO_HUB_BITMAPS, "dense": GP_DENSE_HUB_BITMAPS}[hub_bitmaps]
        o = LoadOpts()
        lib.gp_load_opts_default(ctypes.byref(o))
        o.hub_min_degree = int(hub_min_degree)
        o.hub_budget_bytes = int(hub_budget_bytes)
        self._h = ctypes.c_void_p()
        try:
            import torch
            is_tensor = isinstance(row_ptr, torch.Tensor)
        except ImportError:  # pragma: no cover
            is_tensor = False
        if is_tensor:
            assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32
            assert row_ptr.is_cuda and col.is_cuda
            row_ptr = row_ptr.contiguous()
            col = col.contiguous()
            n = row_ptr.numel() - 1
            o.flags = GP_IN_DEVICE | extra
            st = lib.gp_load_graph_opts(row_ptr.data_ptr(), col.data_ptr(), n, col.numel(), ctypes.byref(o),
                                        _stream_handle(stream), ctypes.byref(self._h))
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            n = rp.shape[0] - 1
            o.flags = extra
            st = lib.gp_load_graph_opts(rp.ctypes.data, cl.ctypes.data if cl.size else None, n, cl.size,
                                        ctypes.byref(o), _stream_handle(stream), ctypes.byref(self._h))
        _check(st, "gp_load_graph_opts")

    @classmethod
    def from_csr(cls, g, device: bool = False, stream=None, hub_bitmaps: str = "auto", **opts) -> "Graph":
        """From an object with numpy ``row_ptr`` / ``col``; device=True uploads
        them as torch tensors first and loads from device memory."""
        if device:
            import torch
            rp = torch.from_numpy(np.asarray(g.row_ptr, dtype=np.int64)).cuda()
            cl = torch.from_numpy(np.asarray(g.col, dtype=np.int32)).cuda()
            return cls(rp, cl, stream, hub_bitmaps, **opts)
        return cls(g.row_ptr, g.col, stream, hub_bitmaps, **opts)

    @property
    def handle(self):
        return self._h

    def stats(self) -> Stats:
        s = Stats()
        _check(_lib().gp_graph_stats(self._h, ctypes.byref(s)), "gp_graph_stats")
        return s

    def new_id(self) -> np.ndarray:
        n = self.stats().n
        out = np.empty(n, dtype=np.int32)
        _check(_lib().gp_graph_new_id(self._h, out.ctypes.data), "gp_graph_new_id")
        return out

    def layout(self) -> tuple[np.ndarray, np.ndarray]:
        s = self.stats()
        rp = np.empty(s.n + 1, dtype=np.int64)
        cl = np.empty(max(1, 2 * s.m), dtype=np.int32)
        _check(_lib().gp_graph_layout(self._h, rp.ctypes.data, cl.ctypes.data), "gp_graph_layout")
        return rp, cl[:2 * s.m]

    def close(self) -> None:
        if self._h:
            _lib().gp_free_graph(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A compiled configuration (schedule + restriction set) for one pattern."""

    def __init__(self, k: int, edges: Sequence[tuple[int, int]], stats: Stats | None = None,
                 force_order: Sequence[int] | None = None, force_set: int | None = None,
                 force_restr: Sequence[tuple[int, int]] | None = None, max_states: int = 0,
                 max_sets: int = 0, cost_cap: float = 0.0, iep: int | bool = False):
        lib = _lib()
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
        o = PlanOpts()
        lib.gp_plan_opts_default(ctypes.byref(o))
        o.max_states = max_states
        o.max_sets = max_sets
        o.cost_cap = cost_cap
        # True: as many innermost levels as the schedule allows; 2..4: at most that many
        o.iep = int(iep) if not isinstance(iep, bool) else (1 if iep else 0)
        if force_order is not None:
            for i, v in enumerate(force_order):
                o.force_order[i] = v
        if force_set is not None:
            o.force_set = force_set
        if force_restr is not None:
            o.n_force_restr = len(force_restr)
            for i, (a, b) in enumerate(force_restr):
                o.force_restr[2 * i] = a
                o.force_restr[2 * i + 1] = b
        self._h = ctypes.c_void_p()
        self.k = k
        self.edges = [tuple(x) for x in edges]
        st = lib.gp_plan_create(e.ctypes.data, k, len(edges),
                                ctypes.byref(stats) if stats is not None else None,
                                ctypes.byref(o), ctypes.byref(self._h))
        _check(st, "gp_plan_create")

    @property
    def handle(self):
        return self._h

    def info(self) -> PlanInfo:
        inf = PlanInfo()
        _check(_lib().gp_plan_get(self._h, ctypes.byref(inf)), "gp_plan_get")
        return inf

    @property
    def order(self) -> tuple[int, ...]:
        inf = self.info()
        return tuple(inf.order[i] for i in range(inf.k))

    @property
    def restrictions(self) -> list[tuple[int, int]]:
        inf = self.info()
        return [(inf.restr[2 * i], inf.restr[2 * i + 1]) for i in range(inf.n_restr)]

    def sets(self) -> list[frozenset]:
        out = []
        buf = (ctypes.c_int32 * (2 * MAX_K * MAX_K))()
        nr = ctypes.c_int32()
        for i in range(self.info().n_sets):
            _check(_lib().gp_plan_get_set(self._h, i, ctypes.byref(nr), buf), "gp_plan_get_set")
            out.append(frozenset((buf[2 * j], buf[2 * j + 1]) for j in range(nr.value)))
        return out

    def schedules(self) -> list[tuple[int, ...]]:
        out = []
        buf = (ctypes.c_int32 * MAX_K)()
        for i in range(self.info().n_schedules):
            _check(_lib().gp_plan_get_schedule(self._h, i, buf), "gp_plan_get_schedule")
            out.append(tuple(buf[j] for j in range(self.k)))
        return out

    def model_cost(self, idx_schedule: int, idx_set: int, stats: Stats | None = None) -> float:
        c = ctypes.c_double()
        _check(_lib().gp_plan_model_cost(self._h, idx_schedule, idx_set,
                                         ctypes.byref(stats) if stats is not None else None,
                                         ctypes.byref(c)), "gp_plan_model_cost")
        return c.value

    def tuned(self, graph: "Graph", max_configs: int = 0, sample_stride: int = 0,
              tune_launch: bool = True, budget_seconds: float = 0.0, stream=None,
              try_iep: bool = False) -> "Plan":
        """A new plan whose configuration and launch shape were timed on graph;
        try_iep: IEP configurations compete too (the result may count with IEP)."""
        o = TuneOpts(max_configs, sample_stride, 1 if tune_launch else -1, budget_seconds,
                     1 if try_iep else 0)
        h = ctypes.c_void_p()
        _check(_lib().gp_plan_tune(graph.handle, self._h, ctypes.byref(o), _stream_handle(stream),
                                   ctypes.byref(h)), "gp_plan_tune")
        p = Plan.__new__(Plan)
        p._h = h
        p.k = self.k
        p.edges = list(self.edges)
        return p

    def with_launch(self, **launch) -> "Plan":
        """A copy of this plan whose default launch shape (the one it takes in
        a batch) has the given non-zero fields."""
        q = Plan.__new__(Plan)
        q.k = self.k
        q.edges = list(self.edges)
        q._h = ctypes.c_void_p()
        _check(_lib().gp_plan_with_launch(self._h, ctypes.byref(_launch(**launch)), ctypes.byref(q._h)),
               "gp_plan_with_launch")
        return q

    def launch(self) -> dict:
        l = self.info().launch
        return dict(group=l.group, waves_per_cu=l.waves_per_cu, chunk=l.chunk, leaf_mode=l.leaf_mode,
                    split_ways=l.split_ways, split_vertices=l.split_vertices, xcd_tasks=l.xcd_tasks,
                    batch_runs=l.batch_runs)

    def close(self) -> None:
        if self._h:
            _lib().gp_free_plan(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count(graph: Graph, plan: Plan, stream=None, **launch) -> int:
    """Exact embedding count (blocking)."""
    out = ctypes.c_uint64()
    lp = _launch(**launch)
    _check(_lib().gp_count(graph.handle, plan.handle, ctypes.byref(lp), _stream_handle(stream),
                           ctypes.byref(out)), "gp_count")
    return out.value


def count_async(graph: Graph, plan: Plan, dev_out, stream=None, **launch) -> None:
    """Enqueue a count; dev_out is a CUDA uint64/int64 tensor with >= 2 entries
    that receives {count, overflow flag}."""
    lp = _launch(**launch)
    _check(_lib().gp_count_async(graph.handle, plan.handle, ctypes.byref(lp), _stream_handle(stream),
                                 dev_out.data_ptr()), "gp_count_async")


def count_noalloc(graph: Graph, plan: Plan, dev_out, stream=None, **launch) -> None:
    """As count_async, with no device allocation (the library's static
    workspace; see gp_count_noalloc)."""
    lp = _launch(**launch)
    _check(_lib().gp_count_noalloc(graph.handle, plan.handle, ctypes.byref(lp), _stream_handle(stream),
                                   dev_out.data_ptr()), "gp_count_noalloc")


def count_per_root(graph: Graph, plan: Plan, stream=None, **launch):
    """(total, per-root counts as a CUDA int64 tensor indexed by layout CSR entry)."""
    import torch
    s = graph.stats()
    per = torch.empty(max(1, 2 * s.m), dtype=torch.int64, device="cuda")
    out = ctypes.c_uint64()
    lp = _launch(**launch)
    _check(_lib().gp_count_per_root(graph.handle, plan.handle, ctypes.byref(lp),
                                    _stream_handle(stream), per.data_ptr(), ctypes.byref(out)),
           "gp_count_per_root")
    return out.value, per[:2 * s.m]


def list_embeddings(graph: Graph, plan: Plan, capacity: int | None = None, out=None, stream=None,
                    **launch):
    """(rows, total): the embeddings as a CUDA int32 tensor of shape
    (min(total, capacity), k), row r holding the original vertex id that each
    pattern vertex maps to, and the number of embeddings. capacity None: the
    count is taken first and every embedding is returned. out: an optional
    CUDA int32 tensor of at least capacity * k elements to write into."""
    import torch
    k = plan.k
    if capacity is None:
        capacity = count(graph, plan, stream=stream)
    capacity = int(capacity)
    if capacity < 0:
        raise ValueError("capacity must be >= 0")
    if out is None:
        out = torch.empty((max(1, capacity), k), dtype=torch.int32, device="cuda")
    elif out.dtype != torch.int32 or not out.is_cuda or out.numel() < capacity * k or not out.is_contiguous():
        raise ValueError("out must be a contiguous CUDA int32 tensor of at least capacity * k elements")
    total = ctypes.c_uint64()
    lp = _launch(**launch)
    _check(_lib().gp_list(graph.handle, plan.handle, ctypes.byref(lp), _stream_handle(stream),
                          out.data_ptr() if capacity > 0 else None, capacity, ctypes.byref(total)), "gp_list")
    n = min(total.value, capacity)
    return out.reshape(-1)[:n * k].view(n, k), total.value


def count_traffic(graph: Graph, plan: Plan, stream=None, **launch) -> tuple[int, int]:
    """(count, algorithmic bytes) from the instrumented kernel (blocking)."""
    out = ctypes.c_uint64()
    b = ctypes.c_uint64()
    lp = _launch(**launch)
    _check(_lib().gp_count_traffic(graph.handle, plan.handle, ctypes.byref(lp),
                                   _stream_handle(stream), ctypes.byref(out), ctypes.byref(b)),
           "gp_count_traffic")
    return out.value, b.value


def estimate(graph: Graph, plan: Plan, budget_ms: float = 0.0, stream=None, **launch) -> dict:
    """Full-run time estimate of a count from a strided root sample
    (see gp_estimate): {"ms", "sample_count", "sample_stride"}; ms is inf when
    the sample ran past budget_ms."""
    ms = ctypes.c_double()
    cnt = ctypes.c_uint64()
    stride = ctypes.c_int64()
    lp = _launch(**launch)
    _check(_lib().gp_estimate(graph.handle, plan.handle, ctypes.byref(lp), float(budget_ms),
                              _stream_handle(stream), ctypes.byref(ms), ctypes.byref(cnt),
                              ctypes.byref(stride)), "gp_estimate")
    v = ms.value
    return {"ms": float("inf") if v >= 1e299 else v, "sample_count": cnt.value,
            "sample_stride": stride.value}


def count_batch(graph: Graph, plans: Sequence[Plan], stream=None, **launch) -> list[int]:
    """Counts of several plans counted together (gp_count_batch; blocking)."""
    arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    out = (ctypes.c_uint64 * len(plans))()
    lp = _launch(**launch)
    _check(_lib().gp_count_batch(graph.handle, arr, len(plans), ctypes.byref(lp),
                                 _stream_handle(stream), out), "gp_count_batch")
    return list(out)


def batch_tune(graph: Graph, plans: Sequence[Plan], stream=None) -> tuple[dict, float]:
    """Fastest batched launch shape for these plans (gp_batch_tune): ({group,
    leaf_mode, batch_runs}, its time in ms)."""
    arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    lp = Launch()
    ms = ctypes.c_double()
    _check(_lib().gp_batch_tune(graph.handle, arr, len(plans), _stream_handle(stream), ctypes.byref(lp),
                                ctypes.byref(ms)), "gp_batch_tune")
    return {"group": lp.group, "leaf_mode": lp.leaf_mode, "batch_runs": lp.batch_runs}, ms.value


class Batch:
    """Several plans counted together, the launches captured in one hipGraph."""

    def __init__(self, graph: Graph, plans: Sequence[Plan], stream=None, **launch):
        self.graph = graph
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
        lp = _launch(**launch)
        self._h = ctypes.c_void_p()
        _check(_lib().gp_batch_create(graph.handle, arr, len(plans), ctypes.byref(lp),
                                      _stream_handle(stream), ctypes.byref(self._h)),
               "gp_batch_create")

    def run(self, stream=None) -> list[int]:
        out = (ctypes.c_uint64 * len(self.plans))()
        _check(_lib().gp_batch_run(self._h, _stream_handle(stream), out), "gp_batch_run")
        return list(out)

    def set_sample(self, root_stride: int, root_offset: int, stream=None) -> None:
        """Count every plan's roots[root_offset + r * root_stride] from the next
        run on (see gp_batch_set_sample)."""
        _check(_lib().gp_batch_set_sample(self._h, int(root_stride), int(root_offset),
                                          _stream_handle(stream)), "gp_batch_set_sample")

    def close(self) -> None:
        if self._h:
            _lib().gp_free_batch(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query loop over resident graphs (see gp_server_create)."""

    def __init__(self, graphs: Sequence[Graph], max_active: int = 0, target_ms: float = 0.0,
                 cost_cap: float = 0.0, initial_slice: int = 0, group: int = 0, leaf_mode: int = 0,
                 waves_per_cu: int = 0, max_query_ms: float = 0.0, iep: int | None = None):
        self.graphs = list(graphs)
        o = ServerOpts()
        _lib().gp_server_opts_default(ctypes.byref(o))
        if iep is not None:
            o.iep = int(iep)
        for name, val in (("max_active", max_active), ("target_ms", target_ms),
                          ("cost_cap", cost_cap), ("initial_slice", initial_slice),
                          ("group", group), ("leaf_mode", leaf_mode),
                          ("waves_per_cu", waves_per_cu), ("max_query_ms", max_query_ms)):
            if val:
                setattr(o, name, val)
        arr = (ctypes.c_void_p * len(graphs))(*[g.handle for g in graphs])
        self._h = ctypes.c_void_p()
        _check(_lib().gp_server_create(arr, len(graphs), ctypes.byref(o), ctypes.byref(self._h)),
               "gp_server_create")

    def submit(self, graph: int, k: int, edges) -> int:
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
        t = ctypes.c_uint64()
        _check(_lib().gp_server_submit(self._h, graph, e.ctypes.data, k, e.size // 2, ctypes.byref(t)),
               "gp_server_submit")
        return t.value

    def poll(self, ticket: int):
        """None while running, else (status, count, latency_s)."""
        done = ctypes.c_int32()
        st = ctypes.c_int32()
        c = ctypes.c_uint64()
        lat = ctypes.c_double()
        _check(_lib().gp_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st),
                                     ctypes.byref(c), ctypes.byref(lat)), "gp_server_poll")
        return (st.value, c.value, lat.value) if done.value else None

    def wait(self, ticket: int, timeout_s: float = 0.0):
        st = ctypes.c_int32()
        c = ctypes.c_uint64()
        lat = ctypes.c_double()
        _check(_lib().gp_server_wait(self._h, ticket, timeout_s, ctypes.byref(st), ctypes.byref(c),
                                     ctypes.byref(lat)), "gp_server_wait")
        return st.value, c.value, lat.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib().gp_server_stats_get(self._h, ctypes.byref(s)), "gp_server_stats_get")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self) -> None:
        if self._h:
            _lib().gp_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_sum(values, div: int = 1, stream=None) -> tuple[int, int]:
    """(quotient mod 2^64, flags) of the exact device accumulation of the
    uint64 values divided by div (see gp_check_sum)."""
    v = np.ascontiguousarray(np.asarray(values, dtype=np.uint64).reshape(-1))
    out = ctypes.c_uint64()
    flags = ctypes.c_uint32()
    _check(_lib().gp_check_sum(v.ctypes.data if v.size else None, v.size, int(div), _stream_handle(stream),
                               ctypes.byref(out), ctypes.byref(flags)), "gp_check_sum")
    return out.value, flags.value


def version() -> str:
    return _lib().gp_version().decode()
