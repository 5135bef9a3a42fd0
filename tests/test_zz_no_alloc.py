"""acq_detect_noalloc through the C ABI: the search whose per-search buffers
live in the library's static device array gives acq_detect's results, on
calls in a row with a shorter block second (the array keeps the previous
call's contents), at a small shape and at the 64-tag x 11-bin x 2^20-sample
tag-bank shape in the launch configuration the bench times; a block needing
more than the array holds is rejected and the next call still works."""
import ctypes

import numpy as np
import pytest

import oracle
import siggen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _noalloc(plan, x, capacity):
    """Call acq_detect_noalloc with device outputs; returns (status, count, records)."""
    from paper_2005_10445_amd import _capi
    rec = _capi.AcqDetection
    out = torch.full((max(capacity, 1) * ctypes.sizeof(rec),), 0x5A, dtype=torch.uint8, device=x.device)
    cnt = torch.full((1,), -7, dtype=torch.int32, device=x.device)
    rc = plan._lib.acq_detect_noalloc(plan._h, ctypes.c_void_p(x.data_ptr()), x.numel(),
                                      ctypes.c_void_p(out.data_ptr()), capacity, ctypes.c_void_p(cnt.data_ptr()))
    torch.cuda.synchronize()
    if rc != 0:
        return rc, None, None
    n = int(cnt.item())
    raw = out.cpu().numpy().tobytes()
    recs = (rec * max(capacity, 1)).from_buffer_copy(raw)
    return rc, n, [recs[i] for i in range(min(n, capacity))]


def _cmp(got, want):
    g = [(r.block, r.tag, r.bin, r.lag, r.toa_samples, r.peak_power, r.z, r.energy, r.flags, r.crossings)
         for r in got]
    w = [(d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power, d.z, d.energy, d.flags, d.crossings) for d in want]
    assert g == w


def test_noalloc_equals_detect_small(dev):
    from paper_2005_10445_amd import Plan
    fs, T, C, spc, K, M = 8e6, 6, 600, 2, 5, 2048
    L = C * spc
    chips = siggen.make_codes(500, T, C)
    freqs, _ = oracle.snap_bins(fs, L, K, 0.0, 20e3)
    xs = [siggen.make_block(510 + i, n, chips, spc, fs, freqs, 3, snr_db=(-6.0, 0.0))[0]
          for i, n in enumerate((20000, 9001))]
    with Plan(chips, spc, fs, num_bins=K, bin_step_hz=20e3, fft_len=M, max_block_len=20000) as p:
        for x in xs:                          # the longer block first, then a shorter one
            xd = torch.from_numpy(x).to(dev)
            rc, n, got = _noalloc(p, xd, T)
            assert rc == 0
            want = p.detect(xd)
            assert n == len(want) and want
            _cmp(got, want)
        # truncation: count is the total, only `capacity` records are written
        xd = torch.from_numpy(xs[0]).to(dev)
        want = p.detect(xd)
        rc, n, got = _noalloc(p, xd, 1)
        assert rc == 0 and n == len(want)
        _cmp(got, want[:1])
        # a block shorter than a template: no detections
        rc, n, got = _noalloc(p, xd[:L - 1].contiguous(), T)
        assert rc == 0 and n == 0


def test_noalloc_equals_detect_tagbank(dev):
    """The tag-bank shape with the bench's tuned launch (tile 32, grid form)."""
    from paper_2005_10445_amd import Plan
    w = siggen.workload("tagbank_fp32")
    T, C, spc, K, N = w["num_tags"], w["num_chips"], w["spc"], w["num_bins"], w["block_len"]
    chips = siggen.make_codes(w["seeds"][0], T, C)
    with Plan(chips, spc, w["fs_hz"], num_bins=K, bin_step_hz=w["bin_step_hz"], max_block_len=N,
              fft_len=w["fft_len"], tag_tile=32) as p:
        blocks = [siggen.make_block(w["seeds"][0], N, chips, spc, w["fs_hz"], p.freqs_hz, w["n_tx"],
                                    snr_db=w["snr_db"])[0],
                  siggen.make_block(w["seeds"][1], 600000, chips, spc, w["fs_hz"], p.freqs_hz, 6,
                                    snr_db=w["snr_db"])[0]]
        for x in blocks:
            xd = torch.from_numpy(x).to(dev)
            rc, n, got = _noalloc(p, xd, T)
            assert rc == 0
            want = p.detect(xd)
            assert n == len(want) and len(want) >= 5
            _cmp(got, want)


def test_noalloc_rejects_blocks_beyond_the_array(dev):
    from paper_2005_10445_amd import Plan, _capi
    fs, T, C, spc = 8e6, 1, 8192, 2
    chips = siggen.make_codes(520, T, C)
    N = 5_000_000                              # 306 segments of 2^15 points: 80 MB of spectra
    with Plan(chips, spc, fs, fft_len=1 << 15, max_block_len=N) as p:
        big = torch.zeros(N, dtype=torch.complex64, device=dev)
        rc, _, _ = _noalloc(p, big, T)
        assert rc == _capi.ACQ_ERR_WORKSPACE_TOO_SMALL
        assert b"static scratch" in p._lib.acq_last_error()
        x, txs = siggen.make_block(521, 200000, chips, spc, fs, np.zeros(1), 1, snr_db=(-10.0, -10.0))
        xd = torch.from_numpy(x).to(dev)
        rc, n, got = _noalloc(p, xd, T)
        assert rc == 0
        want = p.detect(xd)
        assert n == len(want) == 1
        _cmp(got, want)
