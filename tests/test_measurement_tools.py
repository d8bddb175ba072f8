"""Host-side measurement tooling: bench.py's one-GPU contract, the shrinking-heuristic grid of
the paper's evaluation (Table 3), and the rocprofv3 summaries (kernel-trace statistics,
per-dispatch counter totals over hardware instances, counter calibration into bytes)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_heuristic_grid_is_the_papers():
    from paper_1406_5161_amd import datagen as g
    from paper_1406_5161_amd.heuristics import GRID
    names = [x[0] for x in GRID]
    assert names[0] == "none" and len(GRID) == 13
    for mode in ("single", "multi"):
        for k in (2, 500, 1000):
            assert "%s random:%d" % (mode, k) in names
        for pct in (5, 10, 50):
            assert "%s numsamples:%d%%" % (mode, pct) in names
    by = {x[0]: x[1:] for x in GRID}
    assert by["none"][0] == g.SHRINK_NONE
    assert by["multi random:500"] == (g.SHRINK_MULTI, g.KIND_FIXED, 500.0)
    assert by["single numsamples:10%"] == (g.SHRINK_SINGLE, g.KIND_FRACTION, 0.10)


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


@pytest.fixture()
def fake_profiles(tmp_path):
    """Kernel-trace and counter CSVs in rocprofv3's column layout: two dispatches of a loop
    kernel with two counter instances each, and a 1 MiB calibration copy."""
    tr = tmp_path / "trace"
    tr.mkdir()
    _write_csv(tr / "x_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [["loop_kernel", 0, 1000], ["other", 1000, 1500], ["loop_kernel", 2000, 5000]])
    fe = tmp_path / "fetch"
    fe.mkdir()
    _write_csv(fe / "x_counter_collection.csv", ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
               [["loop_kernel", 1, "FETCH_SIZE", 10.0], ["loop_kernel", 1, "FETCH_SIZE", 30.0],
                ["loop_kernel", 3, "FETCH_SIZE", 50.0], ["loop_kernel", 3, "FETCH_SIZE", 70.0]])
    wr = tmp_path / "write"
    wr.mkdir()
    _write_csv(wr / "x_counter_collection.csv", ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
               [["loop_kernel", 1, "WRITE_SIZE", 4.0], ["loop_kernel", 3, "WRITE_SIZE", 8.0]])
    cf = tmp_path / "calib_fetch"
    cf.mkdir()
    _write_csv(cf / "x_counter_collection.csv", ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
               [["copyBuffer", 1, "FETCH_SIZE", 512.0]])
    cw = tmp_path / "calib_write"
    cw.mkdir()
    _write_csv(cw / "x_counter_collection.csv", ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
               [["copyBuffer", 1, "WRITE_SIZE", 1024.0]])
    return tmp_path


def _profsum(*args):
    r = subprocess.run([sys.executable, "-m", "paper_1406_5161_amd.profsum", *map(str, args)], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_profsum_trace_statistics(fake_profiles):
    out = _profsum("trace", fake_profiles / "trace", "--kernel", "loop_kernel")
    line = [l for l in out.splitlines() if l.startswith("loop_kernel")][0].split()
    assert line[1] == "2"                                  # calls
    assert float(line[3]) == pytest.approx(2.0)            # average duration, us (1 and 3 us)
    assert "dispatches of *loop_kernel* (us): 1.0 3.0" in out


def test_profsum_counter_totals_over_instances(fake_profiles):
    out = _profsum("pmc", fake_profiles / "fetch", "--kernel", "loop_kernel", "--totals")
    assert "FETCH_SIZE total per dispatch (2 instances): 40 120" in out


def test_profsum_traffic_calibration(fake_profiles, tmp_path):
    dst = tmp_path / "traffic.json"
    _profsum("traffic", "--fetch", fake_profiles / "fetch", "--write", fake_profiles / "write",
             "--calib-fetch", fake_profiles / "calib_fetch", "--calib-write", fake_profiles / "calib_write",
             "--calib-bytes", 1 << 20, "--kernel", "loop_kernel", "--workload", "w", "--out", dst)
    t = json.load(open(dst))
    # calibration: 1 MiB copy reads 512 KiB of FETCH_SIZE (x2) and 1024 KiB of WRITE_SIZE (x1)
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    # per dispatch, instances added: FETCH 40 and 120 KiB (average 80), WRITE 4 and 8 (average 6)
    assert t["fetch_kib_per_dispatch"] == pytest.approx(80.0)
    assert t["hbm_bytes_per_launch"] == pytest.approx(80 * 1024 * 2.0 + 6 * 1024)
    assert t["workload"] == "w"


def test_source_hash_ignores_comments_only(tmp_path):
    """The counter summaries are keyed by a hash of the loop kernel's code: editing a comment
    keeps it, changing a statement does not."""
    sys.path.insert(0, ROOT)
    from paper_1406_5161_amd.profsum import source_hash
    a = tmp_path / "a.hip"
    a.write_text("// header\nint f(int x) {\n    return x + 1;   // add one\n}\n/* block\n   comment */\n")
    h0 = source_hash([str(a)])
    a.write_text("// a different header\n\nint f(int x) {\n    return x + 1;\n}\n")
    assert source_hash([str(a)]) == h0
    a.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert source_hash([str(a)]) != h0
