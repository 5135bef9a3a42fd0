"""Host-side checks of the measurement bookkeeping: the rocprofv3 summaries
(counter scaling by a device copy, the timed-step windows of a kernel trace,
the VALU issue time) and bench.py's roofline record and traffic lookup, on
small synthetic rocprofv3 CSV files."""
import csv
import json
import math
import os

import pytest

import bench
from paper_2005_10445_amd import profiling as prof


def _write_counters(d, rows):
    """rows: (dispatch id, kernel name, counter, value)"""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, k, c, v in rows:
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def _write_trace(d, dispatches):
    """dispatches: (kernel name, start ns, end ns) in any order"""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "t_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for k, s, e in dispatches:
            w.writerow({"Kernel_Name": k, "Start_Timestamp": s, "End_Timestamp": e})


def test_traffic_scales_by_the_copy_reference(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    kern = "void acq::k_correlate<0>(CorrArgs)"
    # the copy of 1 MiB reads 512 KiB and writes 1024 KiB by the counters
    _write_counters(tmp_path / "cf", [(1, copy, "FETCH_SIZE", 512.0)])
    _write_counters(tmp_path / "cw", [(1, copy, "WRITE_SIZE", 1024.0)])
    # three dispatches of the kernel; --last 2 keeps the last two
    _write_counters(tmp_path / "kf", [(1, kern, "FETCH_SIZE", 100.0), (2, kern, "FETCH_SIZE", 10.0),
                                      (3, kern, "FETCH_SIZE", 30.0)])
    _write_counters(tmp_path / "kw", [(1, kern, "WRITE_SIZE", 8.0), (2, kern, "WRITE_SIZE", 2.0),
                                      (3, kern, "WRITE_SIZE", 4.0)])
    t = prof.traffic(str(tmp_path / "kf"), str(tmp_path / "kw"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                     "k_correlate", 1 << 20, "cmd", last=2)
    assert t["fetch_scale_bytes_per_kib"] == 2048.0 and t["write_scale_bytes_per_kib"] == 1024.0
    assert t["bytes_read_per_launch"] == 20.0 * 2048.0           # mean of 10 and 30 counted KiB
    assert t["bytes_written_per_launch"] == 3.0 * 1024.0
    assert t["bytes_per_launch"] == t["bytes_read_per_launch"] + t["bytes_written_per_launch"]
    assert t["dispatches"] == "last 2"
    every = prof.traffic(str(tmp_path / "kf"), str(tmp_path / "kw"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                         "k_correlate", 1 << 20, "cmd")
    assert every["bytes_read_per_launch"] == pytest.approx((140.0 / 3) * 2048.0)


def test_last_dispatches_opens_the_window_at_the_anchor(tmp_path):
    # plan-time tuning: a Stockham candidate and the chosen kernel, then the timed
    # steps (fill, chosen kernel, refine) three times
    d = []
    t = 0
    for _ in range(4):
        d.append(("k_correlate<Stockham, 0, 0>", t, t + 70)); t += 100
    for _ in range(2):
        d.append(("k_correlate<Fft14, 0, 0>", t, t + 30)); t += 100
    for step in range(3):
        d.append(("k_fill", t, t + 1)); t += 10
        d.append(("k_correlate<Fft14, 0, 0>", t, t + 24 + step)); t += 100
        d.append(("k_refine", t, t + 2)); t += 10
    _write_trace(tmp_path, d)
    w = prof.last_dispatches(str(tmp_path), 2)
    assert w["k_correlate<Fft14, 0, 0>"] == [25, 26]
    assert "k_correlate<Stockham, 0, 0>" not in w
    assert w["k_refine"] == [2, 2] and w["k_fill"] == [1]   # the window opens at the anchor's dispatch
    with pytest.raises(KeyError):
        prof.last_dispatches(str(tmp_path), 2, anchor="k_absent")


def test_timed_dispatches_skip_the_warmup(tmp_path):
    d = []
    t = 0
    for step in range(5):                    # 2 warm-up + 3 timed steps, 2 launches of k_a per step
        for j in range(2):
            d.append(("k_a", t, t + 10 * step + j)); t += 100
        d.append(("k_b", t, t + 5)); t += 100
    d.append(("k_plan", t, t + 1000))         # launched once: left out
    _write_trace(tmp_path, d)
    w = prof.timed_dispatches(str(tmp_path), 2, 5)
    assert w["k_a"] == [20, 21, 30, 31, 40, 41]
    assert w["k_b"] == [5, 5, 5]
    assert "k_plan" not in w


def test_issue_time(tmp_path):
    kern = "void acq::k_correlate<0>(CorrArgs)"
    n = 1024 * 2.4e9 / 4 * 1e-3              # wave instructions that take 1 ms to issue
    _write_counters(tmp_path, [(1, kern, "SQ_INSTS_VALU", 5.0), (2, kern, "SQ_INSTS_VALU", n)])
    s = prof.issue_summary(str(tmp_path), "k_correlate", "cmd", last=1)
    assert "1.000 ms per dispatch" in s and "(the last 1)" in s


def test_roofline_record():
    r = bench.roofline(78.65, 2.0, 157.3e9, 16e6)
    assert r["bound"] == "alu" and r["peak"] == bench.PEAK_FP32_TFLOPS
    assert r["frac"] == pytest.approx(0.5) and r["frac_unpacked_peak"] == pytest.approx(1.0)
    assert r["hbm_gbs"] == pytest.approx(8.0) and r["hbm_frac"] == pytest.approx(8.0 / bench.PEAK_HBM_GBS)
    assert bench.roofline(50.0, 2.0, 1e11, None)["hbm_gbs"] is None


def test_correlate_flops():
    # one product of a 2^15-point transform with V valid lags
    M, V = 1 << 15, 16385
    assert bench.correlate_flops(1, 1, 1, M, V) == 5.0 * M * 15 + 6.0 * M + 4.0 * V
    assert bench.correlate_flops(64, 11, 63, M, V) == pytest.approx(1.206e11, rel=1e-3)


def test_traffic_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    good = {"kernel_source_hash": prof.kernel_source_hash(prof.KERNEL_SOURCES),
            "kernel_sources": list(prof.KERNEL_SOURCES), "bytes_per_launch": 123.0}
    stale = dict(good, kernel_source_hash="0" * 16)
    (tmp_path / "good.json").write_text(json.dumps(good))
    (tmp_path / "stale.json").write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"a": str(tmp_path / "good.json"), "b": str(tmp_path / "stale.json"),
                                                 "c": str(tmp_path / "missing.json")})
    assert bench.traffic_per_launch("a") == 123.0
    assert bench.traffic_per_launch("b") is None
    assert bench.traffic_per_launch("c") is None
    assert bench.traffic_per_launch("other") is None


def test_committed_traffic_files_name_their_sources():
    for path in bench.TRAFFIC_FILES.values():
        with open(path) as f:
            t = json.load(f)
        assert set(t["kernel_sources"]) in (set(prof.KERNEL_SOURCES), set(prof.FSK_SOURCES)), path
        assert t["bytes_per_launch"] > 0 and math.isfinite(t["bytes_per_launch"])


def test_lds_summary(tmp_path):
    kern = "void acq::(anonymous namespace)::k_correlate<acq::Fft14, 0, 0>(acq::CorrArgs)"
    other = "void acq::(anonymous namespace)::k_refine(acq::RefineArgs)"
    rows = []
    for i, (k, inst, bank, act) in enumerate([(kern, 100.0, 10.0, 400.0), (kern, 300.0, 30.0, 400.0),
                                              (other, 5.0, 0.0, 20.0)]):
        rows += [(i + 1, k, "SQ_INSTS_LDS", inst), (i + 1, k, "SQ_LDS_BANK_CONFLICT", bank),
                 (i + 1, k, "SQ_ACTIVE_INST_LDS", act)]
    _write_counters(tmp_path, rows)
    s = prof.lds_summary(str(tmp_path), "cmd")
    lines = [l for l in s.splitlines() if l.startswith("k_")]
    assert lines[0].split()[0] == "k_correlate<Fft14," and lines[1].split()[0] == "k_refine"
    f = lines[0].split()
    # 2 dispatches; means 200 instructions, 20 conflict cycles, 400 issue cycles, share 0.05
    assert f[-7] == "2" and float(f[-6]) == 200.0 and float(f[-5]) == 20.0 and float(f[-1]) == 0.05
