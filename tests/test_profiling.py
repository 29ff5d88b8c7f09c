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


def _write_db(path, rows):
    """A database shaped like rocprofv3's SQLite output: only the
    counters_collection view's columns the summaries read."""
    import sqlite3
    con = sqlite3.connect(path)
    con.execute("CREATE TABLE counters_collection (dispatch_id INTEGER, kernel_name TEXT, "
                "counter_name TEXT, value REAL)")
    con.executemany("INSERT INTO counters_collection VALUES (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_summary_from_sqlite_databases(tmp_path):
    """The same scaling from rocprofv3's SQLite output (*.db globs): values
    of one dispatch summed over the counter's instances, the longest
    dispatch of the kernel kept, the copy kernel calibrating each counter."""
    mib = 1 << 20
    k = "void gpcount::count_kernel<5, 64, 1, 0, 2>(GpPlanDesc, gpcount::CountArgs)"
    _write_db(tmp_path / "f_results.db", [
        (1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 300), (1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 212),
        (2, k, "FETCH_SIZE", 60), (2, k, "FETCH_SIZE", 40), (3, k, "FETCH_SIZE", 70)])
    _write_db(tmp_path / "w_results.db", [
        (1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024), (2, k, "WRITE_SIZE", 8), (2, k, "WRITE_SIZE", 2)])
    _write_db(tmp_path / "l_results.db", [
        (2, k, "TCC_HIT_sum", 30), (2, k, "TCC_MISS_sum", 70)])
    s = profiling.traffic_summary(str(tmp_path / "f_*.db"), str(tmp_path / "w_*.db"), "count_kernel", mib,
                                  "all", "rmat22", PLAN, str(tmp_path / "l_*.db"))
    assert s["copy_fetch_kib"] == 512 and s["fetch_scale"] == 2.0 and s["write_scale"] == 1.0
    assert s["fetch_kib"] == 100 and s["write_kib"] == 10
    assert s["hbm_bytes_per_launch"] == 100 * 1024 * 2 + 10 * 1024
    assert s["l2"]["hit_rate"] == 0.3


def test_stored_traffic_applies_only_to_the_current_kernel_sources(tmp_path):
    """A summary is returned only while the kernel sources hash as they did
    when its counters were taken; a missing or unreadable file gives none."""
    import json
    good = {"workload": "rmat22", "hbm_bytes_per_launch": 1.0,
            "kernel_source_hash": profiling.kernel_source_hash()}
    (tmp_path / "good.json").write_text(json.dumps(good))
    (tmp_path / "old.json").write_text(json.dumps(dict(good, kernel_source_hash="0" * 16)))
    (tmp_path / "bad.json").write_text("{not json")
    assert profiling.load_traffic(str(tmp_path / "good.json")) == good
    assert profiling.load_traffic(str(tmp_path / "old.json")) is None
    assert profiling.load_traffic(str(tmp_path / "bad.json")) is None
    assert profiling.load_traffic(str(tmp_path / "missing.json")) is None
