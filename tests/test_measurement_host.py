"""Host-side measurement logic (no GPU): the rocprofv3 summary arithmetic in
paper_2102_12978_amd.profiling, the committed profile records, and the
benchmark's single-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2102_12978_amd import profiling as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COUNTER_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id",
                "Thread_Id", "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size",
                "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
                "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp",
                "End_Timestamp"]


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COUNTER_COLS)
        w.writeheader()
        for i, (name, grid, counter, value) in enumerate(rows):
            w.writerow({c: 0 for c in COUNTER_COLS} | {
                "Dispatch_Id": i + 1, "Grid_Size": grid, "Kernel_Name": name,
                "Counter_Name": counter, "Counter_Value": value})


A = "void ns::(anonymous namespace)::step2_kernel<2, false, false>(ns::Problem, long long)"
B = "void ns::(anonymous namespace)::step2_kernel<2, true, false>(ns::Problem, long long)"


@pytest.fixture
def csvs(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    # kernel A at two launch shapes: only grid 256 is the one asked for
    _counters(f, [(A, 256, "FETCH_SIZE", 1000.0), (A, 256, "FETCH_SIZE", 1200.0),
                  (A, 512, "FETCH_SIZE", 9999.0), (B, 64, "FETCH_SIZE", 100.0)])
    _counters(w, [(A, 256, "WRITE_SIZE", 2000.0), (A, 512, "WRITE_SIZE", 7777.0),
                  (B, 64, "WRITE_SIZE", 50.0)])
    # a 1 MiB copy whose FETCH_SIZE reads half the bytes, WRITE_SIZE all of them
    _counters(cf, [("copy", 4096, "FETCH_SIZE", 512.0), ("fill", 16, "FETCH_SIZE", 1.0)])
    _counters(cw, [("copy", 4096, "WRITE_SIZE", 1024.0)])
    return str(f), str(w), str(cf), str(cw)


def test_short_name_strips_namespaces_and_arguments():
    assert PR.short_name(A) == "step2_kernel<2, false, false>"
    assert PR.short_name("void k(int)") == "k"


def test_traffic_scales_by_the_copy_and_filters_the_grid(csvs):
    f, w, cf, cw = csvs
    import argparse
    a = argparse.Namespace(kernel="step2_kernel<2, false, false>", grid=256, fetch=f, write=w,
                           copy_fetch=cf, copy_write=cw, copy_bytes=1 << 20, cells=100,
                           cmd="x")
    t = PR.traffic(a)
    assert t["dispatches"] == {"fetch": 2, "write": 1}
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["read_bytes_per_launch"] == round(1100.0 * 1024 * 2)
    assert t["write_bytes_per_launch"] == round(2000.0 * 1024)
    assert t["bytes_per_cell"] == round((1100.0 * 2048 + 2000.0 * 1024) / 100, 2)
    a.grid = None                      # every launch shape of the name
    assert PR.traffic(a)["dispatches"]["fetch"] == 3


def test_traffic_sum_adds_the_launches_of_a_group(csvs):
    f, w, cf, cw = csvs
    import io
    from contextlib import redirect_stdout
    buf = io.StringIO()
    with redirect_stdout(buf):
        PR.main(["sum", "--name", "pass", "--row", "step2_kernel<2, false, false>@256",
                 "--row", "step2_kernel<2, true, false>", "--fetch", f, "--write", w,
                 "--copy-fetch", cf, "--copy-write", cw, "--copy-bytes", str(1 << 20),
                 "--cells", "10", "--cmd", "x"])
    t = json.loads(buf.getvalue())
    rd = 1100.0 * 2048 + 100.0 * 2048
    wr = 2000.0 * 1024 + 50.0 * 1024
    assert t["read_bytes_per_launch"] == round(rd)
    assert t["write_bytes_per_launch"] == round(wr)
    assert t["bytes_per_launch"] == round(rd) + round(wr)
    assert [l["kernel"] for l in t["launches"]] == ["step2_kernel<2, false, false>",
                                                    "step2_kernel<2, true, false>"]


def test_missing_kernel_is_an_error_not_a_zero(csvs):
    f, w, cf, cw = csvs
    with pytest.raises(SystemExit):
        PR.counter_per_dispatch(f, "no_such_kernel", "FETCH_SIZE")
    with pytest.raises(SystemExit):
        PR.counter_per_dispatch(f, "step2_kernel<2, false, false>", "FETCH_SIZE", grid=7)


def test_pass_spans_group_consecutive_dispatches(tmp_path):
    cols = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id",
            "Kernel_Id", "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp"]
    path = tmp_path / "trace.csv"
    rows = []
    # two passes of four overlapping launches, another kernel in between
    for base, d0 in ((1_000_000, 1), (5_000_000, 6)):
        for q in range(4):
            rows.append({"Dispatch_Id": d0 + q, "Kernel_Name": "step2_kernel<2, x>",
                         "Start_Timestamp": base + 100 * q,
                         "End_Timestamp": base + 2_000_000 - 100 * q})
    rows.append({"Dispatch_Id": 5, "Kernel_Name": "other", "Start_Timestamp": 0,
                 "End_Timestamp": 10})
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: 0 for c in cols} | r)
    n, mean, lo, hi = PR.pass_spans(str(path), "step2_kernel", 4)
    assert n == 2 and mean == pytest.approx(2.0) and lo == hi == pytest.approx(2.0)


def test_committed_profiles_run_committed_files_only():
    """Each summary under profiles/ names the command that made it; none of
    them runs or reads anything outside the committed tree."""
    pdir = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(pdir))
    assert names, "no profile summaries"
    for n in names:
        text = open(os.path.join(pdir, n)).read()
        assert "rocprofv3" in text, n
        assert "_work" not in text and "/root/reference" not in text, n


@pytest.mark.parametrize("kind", ["step2", "step3"])
def test_step_traffic_records_are_tied_to_the_kernel_source_and_tile(kind):
    import bench
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles"))
             if n.startswith(f"{kind}_pass_768x768x255_rows") and n.endswith("_traffic.json")]
    assert names
    for n in names:
        t = json.load(open(os.path.join(ROOT, "profiles", n)))
        assert t["kernel"] == f"{kind}_pass" and len(t["launches"]) == 4
        assert t["bytes_per_launch"] == t["read_bytes_per_launch"] + t["write_bytes_per_launch"]
        assert len(t["kernel_sha256_16"]) == 16
        rows, zc = t["tile"]["rows"], t["tile"]["zchunk"]
        assert n == f"{kind}_pass_768x768x255_rows{rows}_z{zc}_traffic.json"
        # every launch of the summary is the pass kernel at that tile height
        assert all(l["kernel"].startswith(f"{kind}_kernel<{rows},") for l in t["launches"])
        # the bench line takes this record for its own tile shape only, and
        # only while the kernel source is the one profiled
        got = bench.measured_traffic(f"{kind}_pass", (rows, zc))
        if t["kernel_sha256_16"] == bench.kernel_hash(f"{kind}_pass"):
            assert got == t["bytes_per_launch"]
        else:
            assert got is None
    assert bench.measured_traffic(f"{kind}_pass", (3, 7)) is None
    assert bench.measured_traffic(f"{kind}_pass", None) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
