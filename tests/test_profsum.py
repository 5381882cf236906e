"""Host logic of the rocprofv3 summaries (paper_2503_12886_amd/profsum.py) on
small synthetic CSV files: short kernel names, the window average over a
range of one kernel's launches, the per-launch HBM bytes scaled by a copy
of known size, and the per-kernel counter table."""
import csv
import os

import pytest

from paper_2503_12886_amd import profsum


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_short_names():
    assert profsum.short_name("void gbr::composite_bwd_kernel<16, 64>(gbr::PassArgs, float const*)") == \
        "composite_bwd_kernel"
    assert profsum.short_name("gbr::(anonymous namespace)::timer_stamp_kernel(unsigned long long*, int)") == \
        "timer_stamp_kernel"


def test_window_average_follows_launch_order(tmp_path):
    # launches of one kernel listed out of order; the window counts them by start time
    rows = []
    for k, (start, dur) in enumerate([(500, 50), (100, 10), (300, 30), (200, 20), (400, 40)]):
        rows.append([k, "void gbr::composite_bwd_kernel<16, 64>(gbr::PassArgs, float const*)", start, start + dur])
        rows.append([100 + k, "void gbr::other_kernel(int)", start + 1, start + 2])
    _write(tmp_path / "run_kernel_trace.csv", ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           rows)
    line = profsum.window(str(tmp_path), "composite_bwd", 1, 3)   # durations 20, 30, 40 ns
    assert "launches 1..3 of 5" in line and "avg 0.03 us" in line
    with pytest.raises(LookupError):
        profsum.window(str(tmp_path), "composite_bwd", 4, 3)


def test_traffic_scales_by_the_copy(tmp_path):
    fetch, write = tmp_path / "f", tmp_path / "w"
    os.makedirs(fetch)
    os.makedirs(write)
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void gbr::composite_bwd_kernel<16, 64>(gbr::PassArgs, float const*)"
    # two counter instances per dispatch are summed; FETCH counts half the copy's bytes
    _write(fetch / "run_counter_collection.csv", hdr, [
        [1, k, "FETCH_SIZE", 10.0], [1, k, "FETCH_SIZE", 10.0],
        [2, k, "FETCH_SIZE", 30.0], [2, k, "FETCH_SIZE", 10.0],
        [3, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0]])
    _write(write / "run_counter_collection.csv", hdr, [
        [1, k, "WRITE_SIZE", 4.0], [2, k, "WRITE_SIZE", 8.0],
        [3, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0]])
    res = profsum.traffic(str(fetch), str(write), "composite_bwd", 1024 * 1024, "copyBuffer")
    assert res["fetch_factor"] == pytest.approx(2.0) and res["write_factor"] == pytest.approx(1.0)
    assert res["fetch_bytes_per_launch"] == pytest.approx(30.0 * 1024 * 2.0)   # mean of 20 and 40 KiB, x2
    assert res["write_bytes_per_launch"] == pytest.approx(6.0 * 1024)
    win = profsum.traffic(str(fetch), str(write), "composite_bwd", 1024 * 1024, "copyBuffer", (1, 1))
    assert win["fetch_bytes_per_launch"] == pytest.approx(40.0 * 1024 * 2.0)
    assert win["write_bytes_per_launch"] == pytest.approx(8.0 * 1024)


def test_counters_table_sums_instances_and_windows(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void gbr::composite_fwd_kernel<16, 64>(gbr::PassArgs, float*)"
    o = "void gbr::loss_kernel(float const*)"
    rows = []
    for d, v in enumerate([1.0, 2.0, 4.0, 8.0]):      # four launches of the forward, two instances each
        rows += [[d, k, "SQ_WAVES", v], [d, k, "SQ_WAVES", v], [d, k, "SQ_INSTS_VALU", 10 * v]]
    rows += [[10, o, "SQ_WAVES", 5.0], [10, o, "SQ_INSTS_VALU", 7.0]]
    _write(tmp_path / "run_counter_collection.csv", hdr, rows)
    out = profsum.counters(str(tmp_path)).splitlines()
    assert out[0] == "| kernel | dispatches | SQ_INSTS_VALU | SQ_WAVES |"
    assert "| composite_fwd_kernel | 4 | 37.5 | 7.5 |" in out     # means of 10..80 and of 2..16
    assert "| loss_kernel | 1 | 7 | 5 |" in out
    win = profsum.counters(str(tmp_path), kernels=["composite_fwd"], windows={"composite_fwd": (1, 2)}).splitlines()
    assert len(win) == 3 and "| composite_fwd_kernel | 2 | 30 | 6 |" in win   # launches 1 and 2 only
