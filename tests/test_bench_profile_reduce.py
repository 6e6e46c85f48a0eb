"""bench.py's reduction of rocprofv3 output to the per-launch counter record
(CPU only, synthetic CSV files): durations and every counter come from the
same dispatches -- the last `steps` of each scoring kernel -- and the byte
counters are scaled by the plain copy's readings."""
import csv
import json
import os

import bench

LARGE = "void perch::score_kernel<1024, false, false, true, false>(perch::Work, int)"
SMALL = "void perch::score_kernel<512, false, false, true, false>(perch::Work, int)"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _launches():
    """One-object accounting launches (5 per kernel), 2 warm-up and 3 timed
    steps; dispatch ids interleave the two kernels as in a bench run."""
    out, d = [], 1
    for phase, n, ms_large in (("acct", 5, 2.0), ("warm", 2, 10.0), ("timed", 3, 10.0)):
        for k in range(n):
            out.append((d, LARGE, ms_large + (0.5 * k if phase == "timed" else 0.0)))
            out.append((d + 1, SMALL, 1.0))
            d += 2
    return out


def test_reduce_profile_uses_the_timed_dispatches(tmp_path):
    root = str(tmp_path)
    launches = _launches()
    _write(os.path.join(root, "trace", "host", "1_kernel_trace.csv"),
           ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["KERNEL_DISPATCH", d, n, 1000, 1000 + int(ms * 1e6)] for d, n, ms in launches])
    # counters: FETCH 1 KiB per ms of the launch, WRITE 2 KiB, VALU 1e6 per ms
    for counter, per_ms in (("FETCH_SIZE", 1.0), ("WRITE_SIZE", 2.0)):
        _write(os.path.join(root, counter, "host", "1_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
               [[d, n, counter, per_ms * ms] for d, n, ms in launches])
        # the copy reads half the true bytes on FETCH_SIZE, all of them on WRITE_SIZE
        copy = 524288.0 if counter == "FETCH_SIZE" else 1048576.0
        _write(os.path.join(root, f"copy_{counter}", "host", "1_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
               [[1, "at::native::copy_kernel", counter, copy]])
    _write(os.path.join(root, "sq", "host", "1_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           [[d, n, "SQ_INSTS_VALU", 1e6 * ms] for d, n, ms in launches])
    out = os.path.join(root, "rec.json")
    bench.reduce_profile(root, 3, out, 2, 0)
    rec = json.load(open(out))
    large = rec["kernels"]["score_lds_large"]
    timed = [d for d, n, ms in launches if n == LARGE][-3:]
    assert large["dispatches"] == timed
    assert abs(large["avg_ms"] - 10.5) < 1e-9             # 10, 10.5, 11 ms
    # FETCH_SIZE x2 (calibration), in bytes
    assert abs(large["fetch_size_bytes_per_launch"] - 10.5 * 1024 * 2.0) < 1e-6
    assert abs(large["write_size_bytes_per_launch"] - 21.0 * 1024) < 1e-6
    assert abs(large["sq_insts_valu_per_launch"] - 10.5e6) < 1e-3
    assert abs(rec["calibration"]["FETCH_SIZE"]["scale"] - 2.0) < 1e-12
    small = rec["kernels"]["score_lds_small"]
    assert abs(small["avg_ms"] - 1.0) < 1e-9 and len(small["dispatches"]) == 3
    assert rec["kernel_source_sha"] == bench.kernel_source_sha()
    assert rec["variant"] == {"volume": "aabb", "jo": "exact", "search": "table"}


def test_counters_apply_only_to_their_workload():
    """The committed record was taken on the default 640x480 five-object
    workload; another configuration or scene option reports no counters."""
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", "score_kernel_cfg2_counters.json")))
    if rec.get("kernel_source_sha") != bench.kernel_source_sha():
        return                                    # stale record: None everywhere, checked by the bench itself
    assert bench.measured_counters("score_lds_large") is not None
    assert bench.measured_counters("score_lds_large", 3) is None
    assert bench.measured_traffic("score_lds_large", 2, bench.counter_variant("cyl", None, None)) is None
    assert bench.measured_traffic("score_lds_small", 2, bench.counter_variant(None, "nn", None)) is None


def test_trace_gaps_from_marker_ranges(tmp_path, capsys):
    """Plain passes and graph launches are delimited by the library's roctx
    ranges; busy time is the union of kernel intervals, gaps what lies
    between them."""
    root = str(tmp_path)
    ms = 1_000_000
    marks = [["perch_set_scene", 0, ms], ["perch_set_scene", ms, 2 * ms]]
    kern = []
    # one plain pass over the two scenes (each call returns once its kernels are done): kernels 10-20,
    # 21-30 (1 ms gap), 30-40 (touching), 41-50 (1 ms gap)
    marks += [["perch_best_poses", 10 * ms, 20 * ms + ms // 2], ["perch_best_poses", 21 * ms, 50 * ms + ms // 2]]
    kern += [[10 * ms, 20 * ms], [21 * ms, 30 * ms], [30 * ms, 40 * ms], [41 * ms, 50 * ms]]
    # one graph launch: overlapping kernels 60-70 and 65-80, then a later call at 100
    marks += [["perch_batch_launch", 60 * ms, 61 * ms], ["perch_score_batch", 100 * ms, 101 * ms]]
    kern += [[60 * ms, 70 * ms], [65 * ms, 80 * ms], [100 * ms, 110 * ms]]
    _write(os.path.join(root, "t", "x_marker_api_trace.csv"), ["Function", "Start_Timestamp", "End_Timestamp"],
           [[f, a, b] for f, a, b in marks])
    _write(os.path.join(root, "t", "x_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["k", a, b] for a, b in kern])
    bench.trace_gaps(root)
    out = json.loads(capsys.readouterr().out)
    assert out["scenes"] == 2
    (p,) = out["plain_passes"]
    assert p["wall_ms"] == 40.0 and p["gaps"] == 2 and p["gaps_ms"] == 2.0 and abs(p["busy_frac"] - 38 / 40) < 1e-9
    (g,) = out["graph_launches"]
    assert g["wall_ms"] == 20.0 and g["gaps"] == 0 and g["busy_frac"] == 1.0
