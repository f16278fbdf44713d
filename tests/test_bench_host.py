"""Host logic of bench.py (no GPU): the bench contract's guard for several
GPUs, the counter summary read from a rocprofv3 database, and the rule that
a traffic figure is reported only for the workload and kernel sources it
was measured on."""
import importlib.util
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _fake_db(path, rows):
    """A database with the `counters_collection` columns summarize_pmc reads."""
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT)
    assert r.returncode != 0
    assert "GPU" in (r.stdout + r.stderr)


def test_counter_summary_from_database(bench, tmp_path):
    gib_kib = 1024.0 * 1024.0  # 1 GiB in KiB
    fetch = tmp_path / "fetch"
    write = tmp_path / "write"
    fetch.mkdir()
    write.mkdir()
    # the calibration copy reads 1 GiB and writes 1 GiB; FETCH_SIZE reads half
    _fake_db(str(fetch / "run_results.db"), [
        ("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib / 2),
        ("gcol::inc_detect_kernel(gcol::KeySource, gcol::IncBufs)", "FETCH_SIZE", 1000.0),
        ("gcol::inc_detect_kernel(gcol::KeySource, gcol::IncBufs)", "FETCH_SIZE", 3000.0),
    ])
    _fake_db(str(write / "run_results.db"), [
        ("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib_kib),
        ("gcol::inc_detect_kernel(gcol::KeySource, gcol::IncBufs)", "WRITE_SIZE", 10.0),
        ("gcol::inc_detect_kernel(gcol::KeySource, gcol::IncBufs)", "WRITE_SIZE", 30.0),
    ])
    out = tmp_path / "traffic.json"
    bench.summarize_pmc(str(fetch), str(write), "d1", str(out))
    t = json.loads(out.read_text())
    assert t["workload"] == "d1"
    assert abs(t["copy_calibration"]["fetch_scale"] - 2.0) < 1e-9
    assert abs(t["copy_calibration"]["write_scale"] - 1.0) < 1e-9
    k = t["kernels"]["inc_detect_kernel"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes_per_launch"] == int(2000.0 * 1024 * 2.0)   # mean 2000 KiB, scaled x2
    assert k["write_bytes_per_launch"] == int(20.0 * 1024)
    assert k["hbm_bytes_per_launch"] == k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def test_traffic_only_for_its_workload_and_sources(bench, tmp_path, monkeypatch):
    from paper_2107_00075_amd.build import source_hash
    good = {"source_hash": source_hash(), "workload": "d1",
            "kernels": {"inc_detect_kernel": {"hbm_bytes_per_launch": 1234}}}
    path = tmp_path / "pmc_traffic.json"
    path.write_text(json.dumps(good))
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(path))
    assert bench.load_traffic("inc_detect_kernel", "d1") == 1234
    assert bench.load_traffic("inc_detect_kernel", "d2pd2") is None      # another workload's figure
    assert bench.load_traffic("inc_color_kernel", "d1") is None          # not measured
    path.write_text(json.dumps(dict(good, source_hash="0" * 16)))
    assert bench.load_traffic("inc_detect_kernel", "d1") is None          # kernels changed since


def test_counter_rate_sums_every_kernel_or_reports_none(bench, monkeypatch):
    """The whole coloring's counter rate: counter bytes per launch times
    launches, summed over the timed round kernels, over their summed time;
    None as soon as one kernel has no counter figure."""
    per_launch = {"inc_detect_kernel": 600, "inc_tail_kernel": 5000}
    monkeypatch.setattr(bench, "load_traffic", lambda k, w: per_launch.get(k))
    kern = {"inc_detect_kernel": (300, 2000, 4), "inc_tail_kernel": (900, 1000, 1)}  # (alg bytes, ns, launches)
    r = bench.counter_rate(kern, "d1")
    assert r["bytes"] == 600 * 4 + 5000 * 1
    assert r["kernel_ms"] == round(3000 / 1e6, 3)
    assert r["gb_per_s"] == round((600 * 4 + 5000) / 3000, 1)
    assert r["frac_of_peak"] == round((600 * 4 + 5000) / 3000 / bench.HBM_PEAK_GBS, 4)
    kern["inc_color_kernel"] = (10, 10, 1)
    assert bench.counter_rate(kern, "d1") is None


def test_call_rate_counts_every_dispatch_of_a_step(bench, tmp_path):
    """The whole-call rate: counter bytes per launch times the counter run's
    dispatches (one step), over one step's kernel time from a kernel-trace
    database; the runtime's copies and torch's kernels are left out, and a
    kernel the trace lacks gives None."""
    import sqlite3
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start integer, end integer)")
    rows = [("void gcol::inc_tail_kernel(gcol::KeySource)", 0, 4000)] * 2 + \
           [("void gcol::bin_kernel<3>(int)", 0, 100)] * 2 + \
           [("__amd_rocclr_copyBuffer", 0, 999999)] * 2
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    trace = bench._trace_rows(str(tmp_path))
    assert trace["inc_tail_kernel"] == (2, 8000) and trace["bin_kernel<PD2>"] == (2, 200)
    traffic = {"kernels": {
        "inc_tail_kernel": {"hbm_bytes_per_launch": 3000, "dispatches": 1},
        "bin_kernel<PD2>": {"hbm_bytes_per_launch": 50, "dispatches": 1},
        "__amd_rocclr_copyBuffer": {"hbm_bytes_per_launch": 10 ** 9, "dispatches": 5},
        "at::native::vectorized_elementwise_kernel<4>": {"hbm_bytes_per_launch": 10 ** 9, "dispatches": 1}}}
    r = bench.call_rate(trace, traffic, steps=2)
    assert r["bytes_per_step"] == 3050
    assert r["kernel_ms_per_step"] == round((8000 + 200) / 2 / 1e6, 3)
    assert r["gb_per_s"] == round(3050 / ((8000 + 200) / 2), 1)
    assert r["kernels"] == 2
    traffic["kernels"]["inc_color_kernel"] = {"hbm_bytes_per_launch": 1, "dispatches": 1}
    assert bench.call_rate(trace, traffic, steps=2) is None
