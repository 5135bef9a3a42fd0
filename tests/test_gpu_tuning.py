"""Segment-length autotuning (acq_tune_fft_len) on the GPU: every candidate M
is timed and listed, the plans made at each M return the same detections as
the FP64 oracle (results do not depend on M), and a configuration whose
per-phase transform would exceed 2^14 points at 2M lists M alone."""
import numpy as np
import pytest

import oracle
import siggen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FS = 8e6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_plain_workload_segment_lengths(dev):
    """The plain workload's shape (1 tag of 1024 chips at 4 samples per chip,
    one bin, 2^17 samples, one transmission at -10 dB): candidates 2^13 .. 2^16."""
    from paper_2005_10445_amd import Plan, tune_fft_len
    w = siggen.workload("plain_fp32")
    T, C, spc, N = w["num_tags"], w["num_chips"], w["spc"], w["block_len"]
    chips = siggen.make_codes(w["seeds"][0], T, C)
    freqs = np.zeros(1)
    x, txs = siggen.make_block(w["seeds"][0], N, chips, spc, FS, freqs, w["n_tx"], snr_db=w["snr_db"])
    xd = torch.from_numpy(x).to(dev)
    best, table = tune_fft_len(xd, reps=2, chips=chips, spc=spc, fs_hz=FS, max_block_len=N)
    print("[tuning]", best, table, flush=True)
    assert [e["fft_len"] for e in table] == [1 << 13, 1 << 14, 1 << 15, 1 << 16]
    assert best in (1 << 13, 1 << 14, 1 << 15, 1 << 16)
    assert best == min(table, key=lambda e: e["ms"])["fft_len"]
    assert all(e["ms"] > 0 for e in table)
    ref = [r for r in oracle.acquire(x, chips, spc, freqs, FS) if r["detected"]]
    assert len(ref) == 1
    for e in table:
        with Plan(chips, spc, FS, max_block_len=N, fft_len=e["fft_len"]) as p:
            p.set_tuning(e["engine"], e["tag_tile"])
            got = p.detect(xd)
        assert [(d.tag, d.bin, d.lag) for d in got] == [(r["tag"], r["bin"], r["lag"]) for r in ref], e
        assert abs(got[0].toa - ref[0]["toa"]) <= 1e-3
        assert abs(got[0].peak_power - ref[0]["peak_power"]) <= 1e-9 * ref[0]["peak_power"]


def test_two_samples_per_chip_lists_one_length(dev):
    """8192-chip codes at 2 samples per chip: M = 2^15 is the only length whose
    per-phase transform (M / 2) fits one workgroup."""
    from paper_2005_10445_amd import tune_fft_len
    T, C, spc, N = 4, 8192, 2, 70000
    chips = siggen.make_codes(930, T, C)
    freqs, _ = oracle.snap_bins(FS, C * spc, 3, 0.0, 1000.0)
    x, _ = siggen.make_block(931, N, chips, spc, FS, freqs, 2, snr_db=(-10.0, -5.0))
    best, table = tune_fft_len(torch.from_numpy(x).to(dev), reps=1, chips=chips, spc=spc, fs_hz=FS,
                               num_bins=3, bin_step_hz=1000.0, max_block_len=N)
    assert best == 1 << 15 and [e["fft_len"] for e in table] == [1 << 15]
