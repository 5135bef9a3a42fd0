"""The boundary's memory and launch contracts on the GPU (through the C ABI):
a caller-owned workspace, asynchronous searches with device-resident results,
a caller-captured hipGraph of acq_detect, non-finite input checks, the batch
block_of output, and the threshold-crossing counts against the FP64 oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import siggen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FS = 8e6
T, C, SPC, K, STEP, M = 6, 600, 2, 5, 20e3, 2048
L = C * SPC


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _setup(seed=0, lens=(15037, 9001, 20000)):
    chips = siggen.make_codes(300 + seed, T, C)
    freqs, _ = oracle.snap_bins(FS, L, K, 0.0, STEP)
    blocks = [siggen.make_block(310 + seed, n, chips, SPC, FS, freqs, 3, snr_db=(-6.0, 0.0), sub=b)
              for b, n in enumerate(lens)]
    return chips, freqs, blocks


def _plan(chips, **kw):
    from paper_2005_10445_amd import Plan
    kw.setdefault("max_block_len", 20000)
    return Plan(chips, SPC, FS, num_bins=K, bin_step_hz=STEP, fft_len=M, **kw)


def _hip_runtime():
    """The HIP runtime this process already loaded (through torch), for plain copies."""
    path = None
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64.so" in line:
                path = line.split()[-1]
                break
    assert path, "HIP runtime not loaded"
    hip = ctypes.CDLL(path)
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    return hip


def _key(d):
    return (d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power, d.z, d.energy, d.flags, d.crossings)


def test_caller_workspace_equals_library_workspace(dev):
    from paper_2005_10445_amd import workspace_size
    chips, freqs, blocks = _setup()
    xs = [torch.from_numpy(x).to(dev) for x, _ in blocks]
    kw = dict(max_batch_blocks=4)
    need = workspace_size(chips=chips, spc=SPC, fs_hz=FS, num_bins=K, bin_step_hz=STEP, fft_len=M,
                          max_block_len=20000, **kw)
    ws = torch.full((need + 4096,), 0xAB, dtype=torch.uint8, device=dev)    # stale contents
    with _plan(chips, **kw) as own, _plan(chips, workspace=ws, **kw) as mine:
        assert mine.geometry["workspace_bytes"] == need
        for x in xs:
            assert [_key(d) for d in mine.detect(x)] == [_key(d) for d in own.detect(x)]
        assert [_key(d) for d in mine.detect_batch(xs)] == [_key(d) for d in own.detect_batch(xs)]
    # the plan wrote inside the caller's buffer and nowhere past the size it asked for
    assert bool((ws[:need] != 0xAB).any()) and bool((ws[need:] == 0xAB).all())


def test_async_search_and_collect(dev):
    chips, freqs, blocks = _setup(1)
    xs = [torch.from_numpy(x).to(dev) for x, _ in blocks]
    with _plan(chips, max_batch_blocks=4) as sync, _plan(chips, max_batch_blocks=4, asynchronous=True) as asy:
        for x in xs:
            asy.enqueue(x)
            assert [_key(d) for d in asy.collect()] == [_key(d) for d in sync.detect(x)]
        ref = [_key(d) for d in sync.detect_batch(xs)]
        assert [_key(d) for d in asy.detect_batch(xs)] == ref
        # two asynchronous batches in a row: the second waits only for the first's upload
        L_ = asy._lib
        n = len(xs)
        ptrs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        lens = (ctypes.c_int64 * n)(*[x.numel() for x in xs])
        for _ in range(2):
            assert L_.acq_detect_batch(asy._h, ptrs, lens, n, None, 0, None, None) == 0
        assert [_key(d) for d in asy.collect()] == ref
        # the device view of the results
        rec, cnt = asy.device_results()
        counts = (ctypes.c_int32 * 2)()
        torch.cuda.synchronize()
        from paper_2005_10445_amd import _capi
        hip = _hip_runtime()
        assert hip.hipMemcpy(counts, ctypes.c_void_p(cnt), 8, 2) == 0          # hipMemcpyDeviceToHost
        assert counts[0] == len(ref) and counts[1] == 0
        recs = (_capi.AcqDetection * max(counts[0], 1))()
        assert hip.hipMemcpy(recs, ctypes.c_void_p(rec), ctypes.sizeof(recs), 2) == 0
        assert [(r.block, r.tag, r.lag) for r in recs[:counts[0]]] == [(k[0], k[1], k[3]) for k in ref]


def test_caller_captured_graph_of_detect(dev):
    """acq_detect of an asynchronous plan captured by the caller into a hipGraph
    on the plan's stream; replays on new data written into the same block, with
    eager searches and synchronisations in between, equal the synchronous search
    of that data every time."""
    chips, freqs, blocks = _setup(2, lens=(15037, 15037, 15037))
    s = torch.cuda.Stream()
    x = torch.empty(15037, dtype=torch.complex64, device=dev)
    x.copy_(torch.from_numpy(blocks[0][0]))
    torch.cuda.synchronize()
    with _plan(chips, asynchronous=True, stream=s) as asy, _plan(chips) as sync:
        with torch.cuda.stream(s):
            asy.enqueue(x)                   # warm-up outside the capture
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            asy.enqueue(x)
        for i in range(6):
            data = blocks[i % 3][0]
            x.copy_(torch.from_numpy(data))
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                g.replay()
            got = [_key(d) for d in asy.collect()]
            want = [_key(d) for d in sync.detect(x)]
            assert got == want, i
            eager = sync.detect(torch.from_numpy(blocks[(i + 1) % 3][0]).to(dev))     # eager work between
            torch.cuda.synchronize()
            assert eager is not None


def test_non_finite_blocks(dev):
    from paper_2005_10445_amd import AcqError, _capi
    chips, freqs, blocks = _setup(3)
    good = [torch.from_numpy(x).to(dev) for x, _ in blocks]
    bad = good[1].clone()
    bad[777] = complex(float("nan"), 0.0)
    bad2 = good[2].clone()
    bad2[5] = complex(float("inf"), 1.0)
    with _plan(chips, max_batch_blocks=4, check_finite=True) as p, _plan(chips, max_batch_blocks=4) as ref:
        assert [_key(d) for d in p.detect(good[0])] == [_key(d) for d in ref.detect(good[0])]
        with pytest.raises(AcqError) as e:
            p.detect(bad)
        assert e.value.status == _capi.ACQ_ERR_NON_FINITE
        n = 3
        ptrs = (ctypes.c_void_p * n)(good[0].data_ptr(), bad.data_ptr(), bad2.data_ptr())
        lens = (ctypes.c_int64 * n)(good[0].numel(), bad.numel(), bad2.numel())
        out = (_capi.AcqDetection * (n * T))()
        nf = ctypes.c_int32(-1)
        rc = p._lib.acq_detect_batch(p._h, ptrs, lens, n, out, n * T, ctypes.byref(nf), None)
        assert rc == _capi.ACQ_ERR_NON_FINITE and b"2 block" in p._lib.acq_last_error()
        got = [(d.block, d.tag, d.lag) for d in out[:nf.value]]
        want = [(0, d.tag, d.lag) for d in ref.detect(good[0])]
        assert got == want                   # the finite block's detections only


def test_batch_block_of(dev):
    from paper_2005_10445_amd import _capi
    chips, freqs, blocks = _setup(4)
    xs = [torch.from_numpy(x).to(dev) for x, _ in blocks]
    with _plan(chips, max_batch_blocks=4) as p:
        n = len(xs)
        ptrs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        lens = (ctypes.c_int64 * n)(*[x.numel() for x in xs])
        cap = n * T
        out = (_capi.AcqDetection * cap)()
        bo = (ctypes.c_int32 * cap)(*([-1] * cap))
        nf = ctypes.c_int32(0)
        assert p._lib.acq_detect_batch(p._h, ptrs, lens, n, out, cap, ctypes.byref(nf), bo) == 0
        assert nf.value > 0
        assert list(bo[:nf.value]) == [d.block for d in out[:nf.value]]
        assert sorted(set(bo[:nf.value])) == sorted({d.block for d in out[:nf.value]})
        # truncation: block_of follows the delivered records only
        bo2 = (ctypes.c_int32 * cap)(*([-1] * cap))
        assert p._lib.acq_detect_batch(p._h, ptrs, lens, n, out, 2, ctypes.byref(nf), bo2) == \
            _capi.ACQ_ERR_TRUNCATED
        assert list(bo2[:2]) == [d.block for d in out[:2]] and bo2[2] == -1


def test_crossing_counts_match_the_oracle(dev):
    """Threshold crossings of every detected tag, at a low threshold so each
    detection has many, against the oracle's counts at theta (1 -+ 1e-4)."""
    chips, freqs, blocks = _setup(5)
    theta = 6.0
    with _plan(chips, threshold=theta) as p:
        for x, _ in blocks:
            dets = p.detect(torch.from_numpy(x).to(dev))
            ref = {r["tag"]: r for r in oracle.acquire(x, chips, SPC, freqs, FS, theta=theta)}
            assert dets
            for d in dets:
                lo, hi = ref[d.tag]["crossings_band"]
                assert lo <= d.crossings <= hi and d.crossings >= 1, (d.tag, d.crossings, lo, hi)


def test_profiling_modes(dev):
    """Every kernel timed, the correlation kernel alone, or none; the results do
    not depend on the mode, and modes outside the three are rejected."""
    from paper_2005_10445_amd import _capi
    chips, freqs, blocks = _setup(5)
    x = torch.from_numpy(blocks[0][0]).to(dev)
    with _plan(chips) as p:
        ref = [_key(d) for d in p.detect(x)]
        p.set_profiling(True)
        assert [_key(d) for d in p.detect(x)] == ref
        kt = p.last_kernel_times()
        assert all(kt[k] > 0.0 for k in ("block_power", "forward", "correlate", "refine", "compact")), kt
        p.set_profiling(True, correlate_only=True)
        assert [_key(d) for d in p.detect(x)] == ref
        kt = p.last_kernel_times()
        assert kt["correlate"] > 0.0
        assert all(v == 0.0 for k, v in kt.items() if k != "correlate"), kt
        p.set_profiling(False)
        assert [_key(d) for d in p.detect(x)] == ref
        assert all(v == 0.0 for v in p.last_kernel_times().values())
        for bad in (-1, 3):
            assert p._lib.acq_set_profiling(p._h, bad) == _capi.ACQ_ERR_INVALID_ARG
