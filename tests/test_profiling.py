"""Host logic of the counter summaries that fill bench.py's roofline.traffic:
plan matching and the scaling of FETCH_SIZE / WRITE_SIZE by a copy kernel."""
import csv

from paper_2009_10955_amd import profiling


PLAN = {"order": [0, 1, 2, 3, 4], "restrictions": [[1, 0], [2, 0]],
        "launch": {"group": 64, "chunk": 4, "leaf_mode": 4, "split_ways": 4}}


def test_same_plan_compares_order_restrictions_launch_and_iep():
    assert profiling.same_plan(PLAN, dict(PLAN))
    # summaries written before the flag existed count as plain
    assert profiling.same_plan(PLAN, dict(PLAN, iep=False))
    assert not profiling.same_plan(PLAN, dict(PLAN, iep=True))
    assert not profiling.same_plan(dict(PLAN, iep=True), PLAN)
    assert profiling.same_plan(dict(PLAN, iep=True), dict(PLAN, iep=True))
    assert not profiling.same_plan(PLAN, dict(PLAN, launch=dict(PLAN["launch"], chunk=1)))
    assert not profiling.same_plan(PLAN, dict(PLAN, order=[0, 1, 2, 4, 3]))
    assert not profiling.same_plan(PLAN, None) and not profiling.same_plan(None, PLAN)


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_by_the_copy_kernel(tmp_path):
    mib = 1 << 20
    # the copy moves 1 MiB each way; FETCH_SIZE reads half of it, WRITE_SIZE all;
    # counters come per instance and are summed per dispatch
    _write(tmp_path / "f_counter_collection.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": 256},
        {"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": 256},
        {"Dispatch_Id": 2, "Kernel_Name": "count_kernel<5, 64, 4, 0, false>", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 100},
        {"Dispatch_Id": 3, "Kernel_Name": "count_kernel<5, 64, 4, 0, false>", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 40},
    ])
    _write(tmp_path / "w_counter_collection.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": 1024},
        {"Dispatch_Id": 2, "Kernel_Name": "count_kernel<5, 64, 4, 0, false>", "Counter_Name": "WRITE_SIZE",
         "Counter_Value": 10},
    ])
    _write(tmp_path / "l_counter_collection.csv", [
        {"Dispatch_Id": 2, "Kernel_Name": "count_kernel<5, 64, 4, 0, false>", "Counter_Name": "TCC_HIT_sum",
         "Counter_Value": 90},
        {"Dispatch_Id": 2, "Kernel_Name": "count_kernel<5, 64, 4, 0, false>", "Counter_Name": "TCC_MISS_sum",
         "Counter_Value": 10},
    ])
    s = profiling.traffic_summary(str(tmp_path / "f_*.csv"), str(tmp_path / "w_*.csv"), "count_kernel<5", mib,
                                  "5-cycle", "rmat17", PLAN, str(tmp_path / "l_*.csv"))
    assert s["fetch_scale"] == 2.0 and s["write_scale"] == 1.0
    # the longest dispatch of the kernel: 100 KiB read (x2), 10 KiB written
    assert s["fetch_kib"] == 100 and s["write_kib"] == 10
    assert s["hbm_bytes_per_launch"] == 100 * 1024 * 2 + 10 * 1024
    assert s["l2"]["hit_rate"] == 0.9
    assert s["plan"] == PLAN and s["kernel_source_hash"] == profiling.kernel_source_hash()
