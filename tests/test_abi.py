"""The C-ABI library loads and exports every symbol include/gp.h declares
(no device calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2009_10955_amd import gp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "gp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gp_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["gp_load_graph", "gp_plan_create", "gp_count", "gp_count_batch",
                     "gp_count_async", "gp_count_per_root", "gp_strerror", "gp_free_graph",
                     "gp_free_plan", "gp_graph_stats", "gp_plan_get"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gp.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert set(_declared_functions()) == set(gp.SIGNATURES)


def test_host_only_calls():
    lib = gp.library()
    assert lib.gp_strerror(0).decode() == "ok"
    assert "64 bits" in lib.gp_strerror(-9).decode()
    assert "gfx950" in gp.version()


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and field offsets of every struct in gp.h, as laid out by a C
    compiler, equal the ctypes mirrors in the binding."""
    structs = {"gp_stats": gp.Stats, "gp_plan_opts": gp.PlanOpts, "gp_plan_info": gp.PlanInfo,
               "gp_launch": gp.Launch, "gp_tune_opts": gp.TuneOpts,
               "gp_server_opts": gp.ServerOpts, "gp_server_stats": gp.ServerStats,
               "gp_load_opts": gp.LoadOpts}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_argument_errors_need_no_device():
    lib = gp.library()
    h = ctypes.c_void_p()
    assert lib.gp_load_graph(None, None, 4, 0, 0, None, ctypes.byref(h)) == -1
    assert lib.gp_load_graph(None, None, -1, 0, 0, None, ctypes.byref(h)) == -1
    assert lib.gp_count(None, None, None, None, None) == -1
    assert lib.gp_count_batch(None, None, 0, None, None, None) == -1


def test_plan_with_launch_is_host_only_and_validated():
    """A plan's default launch shape can be set on a copy (host only); bad
    fields are refused and leave the output untouched."""
    from paper_2009_10955_amd import inputs as I
    p = gp.Plan(*I.PATTERNS["house"])
    q = p.with_launch(group=8, leaf_mode=3, chunk=4, split_ways=4)
    lq, lp = q.launch(), p.launch()
    assert (lq["group"], lq["leaf_mode"], lq["chunk"], lq["split_ways"]) == (8, 3, 4, 4)
    assert (q.order, q.restrictions) == (p.order, p.restrictions)
    assert lp["waves_per_cu"] == lq["waves_per_cu"]
    lib = gp.library()
    h = ctypes.c_void_p(7)
    for bad in (dict(group=12), dict(leaf_mode=5), dict(waves_per_cu=33), dict(chunk=-1)):
        assert lib.gp_plan_with_launch(p.handle, ctypes.byref(gp._launch(**bad)), ctypes.byref(h)) == -1
        assert h.value == 7
    assert lib.gp_plan_with_launch(None, ctypes.byref(gp._launch()), ctypes.byref(h)) == -1
