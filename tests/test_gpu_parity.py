"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances (stated by the acquisition contract):
  * FFT-path power (FP32): |P_gpu - P_ref| <= 1e-4 * max(P_ref, L * Pxhat);
  * detections: same tags, same (bin, lag) unless the oracle flags a near-tie
    or a near-threshold decision; ToA within 1e-3 samples;
  * reported peak power / z / energy are FP64 re-correlations on both sides:
    relative 1e-9;
  * threshold crossings (hypotheses with z >= theta, decided on FP32 powers):
    within the oracle's counts at theta (1 -+ 1e-4).
"""
import math
import os

import numpy as np
import pytest

import oracle
import siggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FS = 8e6

# (name, T, C, spc, N, K, step_hz, fft_len): span every transform size, every
# samples-per-chip value, several segments with a ragged last one, and a tag
# count that leaves a partial tag tile.
CASES = [
    ("spc2_sub1024", 3, 600, 2, 15037, 5, 20e3, 2048),
    ("spc4_sub2048", 2, 256, 4, 30011, 3, 30e3, 8192),
    ("spc1_sub4096", 2, 1000, 1, 20000, 3, 10e3, 4096),
    ("spc8_sub8192", 2, 100, 8, 25000, 3, 40e3, 65536),
    ("spc2_sub16384", 2, 2000, 2, 70001, 3, 5e3, 32768),
    ("tile_ragged", 20, 300, 2, 9001, 3, 30e3, 2048),
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _plan(chips, spc, K, step, N, fft_len, **kw):
    from paper_2005_10445_amd import Plan
    return Plan(chips, spc, FS, num_bins=K, bin_step_hz=step, max_block_len=N, fft_len=fft_len, **kw)


def _case_block(name, T, C, spc, N, K, step, M=None, seed=0, n_tx=2, snr=(-3.0, 3.0)):
    L = C * spc
    chips = siggen.make_codes(100 + seed, T, C)
    freqs, _ = oracle.snap_bins(FS, L, K, 0.0, step)
    x, txs = siggen.make_block(200 + seed, N, chips, spc, FS, freqs, min(n_tx, T), snr_db=snr)
    return chips, freqs, x, txs


def _compare_detections(dets, ref, L):
    want = {r["tag"]: r for r in ref if r["detected"]}
    loose = {r["tag"] for r in ref if r["near_threshold"]}
    got = {d.tag: d for d in dets}
    assert set(got) - loose == set(want) - loose, (sorted(got), sorted(want))
    for t in set(got) & set(want):
        r, d = want[t], got[t]
        if not r["near_tie"]:
            assert (d.bin, d.lag) == (r["bin"], r["lag"]), (t, d, r)
        assert abs(d.toa - r["toa"]) <= 1e-3, (t, d.toa, r["toa"])
        floor = max(r["peak_power"], L * r["block_power"])
        assert abs(d.peak_power - r["peak_power"]) <= 1e-9 * floor
        assert abs(d.energy - r["energy"]) <= 1e-9 * max(r["energy"], 1.0)
        assert abs(d.z - r["z"]) <= 1e-9 * max(r["z"], 1.0)
        assert abs(d.block_power - r["block_power"]) <= 1e-12 * r["block_power"]
        assert abs(d.power - r["power"]) <= 1e-9 * floor / (L * L)
        if np.isfinite(r["snr"]):
            # sigma^2 = (E - P/L)/L cancels; the bound scales the P and E errors by 1/sigma^2
            s2 = (r["energy"] - r["peak_power"] / L) / L
            assert abs(d.snr - r["snr"]) <= 1e-8 * (floor / (L * L) + r["energy"] / L) / s2 * (1 + r["snr"])
        assert d.freq_hz == r["freq_hz"]
        assert bool(d.flags & 1) == r["near_edge"]
        lo, hi = r["crossings_band"]
        assert lo <= d.crossings <= hi, (t, d.crossings, r["crossings_band"])
    return got, want


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fft_power_matches_oracle(dev, case):
    name, T, C, spc, N, K, step, M = case
    L = C * spc
    chips, freqs, x, _ = _case_block(*case)
    print(f"[power] {name} T={T} C={C} spc={spc} N={N} K={K} M={M}", flush=True)
    with _plan(chips, spc, K, step, N, M) as plan:
        assert np.array_equal(plan.freqs_hz, freqs)
        P = plan.correlate_power(torch.from_numpy(x).to(dev)).cpu().numpy().astype(np.float64)
    ref = oracle.corr_power(x, chips, spc, freqs, FS)
    Px = oracle.block_power(x)
    assert P.shape == ref.shape == (T, K, N - L + 1)
    err = np.abs(P - ref) / np.maximum(ref, L * Px)
    assert err.max() <= 1e-4, (name, float(err.max()), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_detections_match_oracle(dev, case):
    name, T, C, spc, N, K, step, M = case
    L = C * spc
    for seed in range(3):
        chips, freqs, x, txs = _case_block(*case, seed=seed, n_tx=3, snr=(-8.0, 0.0))
        theta = oracle.default_threshold(T, K, N, L)
        print(f"[detect] {name} seed={seed}", flush=True)
        with _plan(chips, spc, K, step, N, M) as plan:
            dets = plan.detect(torch.from_numpy(x).to(dev))
        ref = oracle.acquire(x, chips, spc, freqs, FS, theta=theta)
        got, want = _compare_detections(dets, ref, L)
        for tx in txs:          # strong injections are found where they were put
            if tx.snr_db > -2.0:
                assert tx.tag in got and got[tx.tag].bin == tx.bin
                assert abs(got[tx.tag].toa - tx.toa) < 0.3


def test_edges_and_segment_boundaries(dev):
    """Transmissions at lag 0, lag N-L and on both sides of segment boundaries."""
    T, C, spc, K, step, M = 6, 300, 2, 3, 30e3, 2048
    L = C * spc
    V = M - L + 1
    N = 6 * V + L + 5
    chips = siggen.make_codes(55, T, C)
    freqs, _ = oracle.snap_bins(FS, L, K, 0.0, step)
    delays = [0, N - L, V - 1, V, 3 * V - 1, 4 * V]
    x, txs = siggen.make_block(56, N, chips, spc, FS, freqs, T, snr_db=(3.0, 3.0), noise=True,
                               tags=list(range(T)), delays=delays, fracs=[0.0] * T, bins=[0, 1, 2, 0, 1, 2])
    with _plan(chips, spc, K, step, N, M) as plan:
        dets = plan.detect(torch.from_numpy(x).to(dev))
    ref = oracle.acquire(x, chips, spc, freqs, FS)
    got, want = _compare_detections(dets, ref, L)
    assert set(got) == set(range(T))
    for tx in txs:
        assert got[tx.tag].lag == tx.delay and got[tx.tag].bin == tx.bin
    assert got[0].flags & 1 and got[1].flags & 1
    assert got[0].toa == 0.0 and got[1].toa == float(N - L)


def test_short_blocks(dev):
    T, C, spc, K = 2, 300, 2, 3
    L = C * spc
    chips = siggen.make_codes(3, T, C)
    freqs, _ = oracle.snap_bins(FS, L, K, 0.0, 30e3)
    with _plan(chips, spc, K, 30e3, 5000, 2048) as plan:
        x = torch.zeros(L - 1, dtype=torch.complex64, device=dev)
        assert plan.detect(x) == []
        # exactly one lag
        xb, _ = siggen.make_block(4, L, chips, spc, FS, freqs, 1, snr_db=(10.0, 10.0), tags=[1],
                                  delays=[0], fracs=[0.0], bins=[2])
        dets = plan.detect(torch.from_numpy(xb).to(dev))
        ref = oracle.acquire(xb, chips, spc, freqs, FS)
        _compare_detections(dets, ref, L)
        P = plan.correlate_power(torch.from_numpy(xb).to(dev)).cpu().numpy()
        Pr = oracle.corr_power(xb, chips, spc, freqs, FS)
        assert P.shape == Pr.shape == (T, K, 1)
        assert np.all(np.abs(P - Pr) <= 1e-4 * np.maximum(Pr, L * oracle.block_power(xb)))
        # an all-zero block detects nothing
        assert plan.detect(torch.zeros(4000, dtype=torch.complex64, device=dev)) == []


def test_errors_and_truncation(dev):
    from paper_2005_10445_amd import AcqError, _capi
    import ctypes
    T, C, spc, K = 4, 300, 2, 1
    L = C * spc
    chips = siggen.make_codes(9, T, C)
    N = 8000
    x, txs = siggen.make_block(10, N, chips, spc, FS, [0.0], T, snr_db=(10.0, 10.0), noise=False,
                               delays=[100, 1000, 3000, 5000], fracs=[0.0] * T, bins=[0] * T)
    xt = torch.from_numpy(x).to(dev)
    with _plan(chips, spc, K, 0.0, N, 2048, threshold=5.0) as plan:
        assert len(plan.detect(xt)) == T
        out = (_capi.AcqDetection * 2)()
        nf = ctypes.c_int32(0)
        rc = plan._lib.acq_detect(plan._h, ctypes.c_void_p(xt.data_ptr()), N, out, 2, ctypes.byref(nf))
        assert rc == _capi.ACQ_ERR_TRUNCATED and nf.value == T
        assert [out[0].tag, out[1].tag] == [0, 1]
        big = torch.zeros(N + 1, dtype=torch.complex64, device=dev)
        with pytest.raises(AcqError) as e:
            plan.detect(big)
        assert e.value.status == _capi.ACQ_ERR_BLOCK_TOO_LONG


def test_deterministic_and_plan_reuse(dev):
    name, T, C, spc, N, K, step, M = CASES[0]
    chips, freqs, x, _ = _case_block(*CASES[0], seed=5, n_tx=3)
    xt = torch.from_numpy(x).to(dev)
    with _plan(chips, spc, K, step, N, M) as plan:
        P1 = plan.correlate_power(xt)
        P2 = plan.correlate_power(xt)
        assert torch.equal(P1, P2)
        d1 = plan.detect(xt)
        d2 = plan.detect(xt[: N - 3000].contiguous())      # shorter block, same plan
        d3 = plan.detect(xt)
        assert d1 == d3
    ref2 = oracle.acquire(x[: N - 3000], chips, spc, freqs, FS)
    _compare_detections(d2, ref2, C * spc)


def test_plain_workload_over_seeds(dev):
    """One 2^17-sample block, one 1024-chip tag at 4 samples/chip, one bin,
    one transmission at -10 dB with integer+fractional delay: detection,
    lag and ToA match the oracle for every seed."""
    w = siggen.workload("plain_fp32")
    N, C, spc = w["block_len"], w["num_chips"], w["spc"]
    L = C * spc
    seeds = range(w["seeds"][0], w["seeds"][0] + int(os.environ.get("ACQ_PLAIN_SEEDS", "20")))
    chips = siggen.make_codes(w["seeds"][0], 1, C)
    found = 0
    with _plan(chips, spc, 1, 0.0, N, 0) as plan:
        for seed in seeds:
            x, txs = siggen.make_block(seed, N, chips, spc, w["fs_hz"], [0.0], 1, snr_db=w["snr_db"])
            dets = plan.detect(torch.from_numpy(x).to(dev))
            ref = oracle.acquire(x, chips, spc, [0.0], w["fs_hz"])
            _compare_detections(dets, ref, L)
            if dets:
                found += 1
                assert abs(dets[0].toa - txs[0].toa) < 0.3
    assert found == len(seeds)


@pytest.mark.timeout(500)
def test_tag_bank_full_size(dev, tagbank_case):
    """The 64-tag x 11-bin x 2^20-sample workload at its own sizes and launch
    configuration: detections against the oracle's FFT-identity search, and
    FFT-path power at sampled points against the direct definition."""
    w, chips, freqs, x, txs, ref = tagbank_case
    T, C, spc, N, K = w["num_tags"], w["num_chips"], w["spc"], w["block_len"], w["num_bins"]
    L = C * spc
    xt = torch.from_numpy(x).to(dev)
    print("[tagbank] GPU", flush=True)
    with _plan(chips, spc, K, w["bin_step_hz"], N, w["fft_len"]) as plan:
        dets = plan.detect(xt)
        P = plan.correlate_power(xt)
        g = np.random.default_rng(0)
        lags = N - L + 1
        t_i = g.integers(0, T, 400)
        k_i = g.integers(0, K, 400)
        tau_i = g.integers(0, lags, 400)
        # include every transmission's peak and the segment boundaries
        V = plan.geometry["valid_per_segment"]
        for tx in txs:
            t_i = np.append(t_i, tx.tag); k_i = np.append(k_i, tx.bin); tau_i = np.append(tau_i, tx.delay)
        for b in (V - 1, V, 31 * V, lags - 1):
            t_i = np.append(t_i, 0); k_i = np.append(k_i, 0); tau_i = np.append(tau_i, b)
        idx = torch.from_numpy((t_i * K + k_i) * lags + tau_i).to(dev)
        Ps = P.reshape(-1)[idx].cpu().numpy().astype(np.float64)
        del P
    print("[tagbank] oracle points", flush=True)
    ref_pts = oracle.corr_power_at(x, chips, spc, freqs, w["fs_hz"], t_i, k_i, tau_i)
    Px = oracle.block_power(x)
    err = np.abs(Ps - ref_pts) / np.maximum(ref_pts, L * Px)
    assert err.max() <= 1e-4, float(err.max())
    got, want = _compare_detections(dets, ref, L)
    strong = [tx for tx in txs if tx.snr_db > -12.0]
    for tx in strong:
        assert tx.tag in got and got[tx.tag].bin == tx.bin
