"""Pins of the CPU oracle against things other than itself.

Each test ties one part of the oracle to a brute-force evaluation, a library
routine that computes the same quantity by another route, a closed form, or a
statistical law, so that a dropped term, wrong sign, wrong index or swapped
operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import siggen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _brute_power(x, s, freqs, fs):
    """Triple loop, pure Python, complex exponential per term."""
    x = [complex(v) for v in np.asarray(x, dtype=np.complex64)]
    T, L = len(s), len(s[0])
    N = len(x)
    out = np.zeros((T, len(freqs), N - L + 1))
    for t in range(T):
        for k, f in enumerate(freqs):
            for tau in range(N - L + 1):
                c = 0j
                for n in range(L):
                    ang = -2.0 * math.pi * f * (tau + n) / fs
                    c += x[tau + n] * s[t][n] * complex(math.cos(ang), math.sin(ang))
                out[t, k, tau] = abs(c) ** 2
    return out


def _tiny_case(seed=7, N=64, C=4, spc=2, T=2):
    chips = siggen.make_codes(seed, T, C)
    g = np.random.default_rng(seed)
    x = (g.standard_normal(N) + 1j * g.standard_normal(N)).astype(np.complex64)
    return x, chips


def test_direct_matches_bruteforce(oracle_lib):
    x, chips = _tiny_case()
    fs = 8e6
    freqs = [-250e3, 0.0, 375e3]
    s = [[float(chips[t][n // 2]) for n in range(8)] for t in range(2)]
    P = oracle.corr_power(x, chips, 2, freqs, fs)
    B = _brute_power(x, s, freqs, fs)
    assert P.shape == (2, 3, 64 - 8 + 1)
    np.testing.assert_allclose(P, B, rtol=1e-11, atol=1e-11)


def test_direct_matches_numpy_correlate(oracle_lib):
    """numpy.correlate(a, v, 'valid')[tau] = sum_n a[tau+n] conj(v[n])."""
    g = np.random.default_rng(3)
    N, C, spc, T = 500, 24, 3, 3
    chips = siggen.make_codes(11, T, C)
    x = (g.standard_normal(N) + 1j * g.standard_normal(N)).astype(np.complex64)
    fs = 1e6
    freqs = [-31250.0, 0.0, 15625.0, 62500.0]
    P = oracle.corr_power(x, chips, spc, freqs, fs)
    n = np.arange(N)
    x128 = x.astype(np.complex128)
    for t in range(T):
        v = np.repeat(chips[t].astype(np.float64), spc)
        for k, f in enumerate(freqs):
            c = np.correlate(x128 * np.exp(-2j * np.pi * f * n / fs), v, "valid")
            np.testing.assert_allclose(P[t, k], np.abs(c) ** 2, rtol=1e-10, atol=1e-9)


def test_points_match_full_array(oracle_lib):
    x, chips = _tiny_case(seed=5, N=300, C=10, spc=3, T=3)
    fs = 2e6
    freqs = [-1e5, 0.0, 2e5]
    P = oracle.corr_power(x, chips, 3, freqs, fs)
    g = np.random.default_rng(1)
    t = g.integers(0, 3, 50)
    k = g.integers(0, 3, 50)
    tau = g.integers(0, 300 - 30 + 1, 50)
    v = oracle.corr_power_at(x, chips, 3, freqs, fs, t, k, tau)
    np.testing.assert_allclose(v, P[t, k, tau], rtol=1e-10, atol=1e-9)


def test_fft_identity_matches_direct(oracle_lib):
    g = np.random.default_rng(9)
    N, C, spc, T = 4096 + 37, 128, 2, 3
    chips = siggen.make_codes(4, T, C)
    x = (g.standard_normal(N) + 1j * g.standard_normal(N)).astype(np.complex64)
    fs = 8e6
    freqs, _ = oracle.snap_bins(fs, C * spc, 5, 0.0, 40e3)
    P = oracle.corr_power(x, chips, spc, freqs, fs)
    scale = P.max()
    for t, Pt in oracle.corr_power_fft(x, chips, spc, freqs, fs):
        np.testing.assert_allclose(Pt, P[t], rtol=0, atol=1e-11 * scale)


def test_golden_handworked_example(oracle_lib):
    """A worked example computed by hand (see the fixture's note)."""
    with open(os.path.join(GOLDEN, "handworked_corr.json")) as fh:
        case = json.load(fh)
    x = np.array([complex(a, b) for a, b in case["x"]], dtype=np.complex64)
    chips = np.array(case["chips"], dtype=np.int8)
    P = oracle.corr_power(x, chips, case["spc"], case["freqs_hz"], case["fs_hz"])
    np.testing.assert_allclose(P, np.array(case["P"], dtype=np.float64), rtol=1e-12, atol=1e-12)


def test_snap_bins_grid():
    f, step = oracle.snap_bins(8e6, 16384, 11, 0.0, 1000.0)
    assert step == 976.5625
    assert f[0] == -5 * 976.5625 and f[-1] == 5 * 976.5625 and f[5] == 0.0
    m_min, q = oracle.rotation_grid(8e6, 16384)
    assert m_min == 32768 and q == 244.140625
    assert oracle.rotation_grid(8e6, 4096)[0] == 8192
    f1, _ = oracle.snap_bins(8e6, 4096, 1, 0.0, 0.0)
    assert list(f1) == [0.0]
    f21, _ = oracle.snap_bins(8e6, 16384, 21, 0.0, 1000.0)
    assert f21[0] == -10 * 976.5625
    with pytest.raises(ValueError):
        oracle.snap_bins(8e6, 16384, 4, 0.0, 1000.0)
    # every bin is an integer number of quanta, so rotations are integers at any M >= M_min
    for M in (32768, 65536, 131072):
        m = f * M / 8e6
        assert np.all(m == np.round(m))


def test_default_threshold_values():
    assert abs(oracle.default_threshold(1, 1, 1 << 17, 4096) - 18.659) < 1e-3
    assert abs(oracle.default_threshold(64, 11, 1 << 20, 16384) - 27.312) < 1e-3


def test_exact_recovery_integer_delay(oracle_lib):
    """Noise-free, unit amplitude, zero offset and phase: x holds exactly +/-1,
    so P at the true lag is exactly L^2, the neighbours are symmetric and the
    parabola vertex is exactly the integer delay."""
    C, spc, N, fs = 64, 2, 1000, 8e6
    chips = siggen.make_codes(21, 3, C)
    L = C * spc
    x, txs = siggen.make_block(5, N, chips, spc, fs, [0.0], 1, snr_db=(0.0, 0.0), noise=False,
                               tags=[1], delays=[333], fracs=[0.0], bins=[0], phases=[0.0])
    res = oracle.acquire(x, chips, spc, [0.0], fs, theta=1.0)
    r = res[1]
    assert r["lag"] == 333 and r["bin"] == 0
    assert r["peak_power"] == float(L * L)
    assert r["delta"] == 0.0 and r["toa"] == 333.0
    assert r["energy"] == float(L)


def test_exact_recovery_with_offset_and_phase(oracle_lib):
    C, spc, N, fs = 128, 2, 3000, 8e6
    L = C * spc
    chips = siggen.make_codes(22, 4, C)
    freqs, _ = oracle.snap_bins(fs, L, 5, 0.0, 60e3)
    x, txs = siggen.make_block(6, N, chips, spc, fs, freqs, 2, snr_db=(6.0, 6.0), noise=False,
                               tags=[0, 3], delays=[100, 2000], fracs=[0.0, 0.0], bins=[4, 1])
    res = oracle.acquire(x, chips, spc, freqs, fs)
    for tx in txs:
        r = res[tx.tag]
        assert r["detected"] and r["lag"] == tx.delay and r["bin"] == tx.bin
        assert abs(r["peak_power"] / (tx.amplitude ** 2 * L * L) - 1) < 1e-6
        assert abs(r["delta"]) < 1e-6


def test_dirichlet_offgrid_loss(oracle_lib):
    """Residual offset df against bin 0: P = sin^2(pi df L/Fs) / sin^2(pi df/Fs)."""
    C, spc, N, fs = 100, 2, 700, 1e6
    L = C * spc
    chips = siggen.make_codes(3, 1, C)
    D = 250
    for df in (0.0, 137.0, 1234.5, 2500.0, 4999.0):
        x, _ = siggen.make_block(1, N, chips, spc, fs, [df], 1, snr_db=(0.0, 0.0), noise=False,
                                 tags=[0], delays=[D], fracs=[0.0], bins=[0], phases=[0.3])
        v = oracle.corr_power_at(x, chips, spc, [0.0], fs, [0], [0], [D])[0]
        a = math.pi * df / fs
        expect = float(L * L) if df == 0.0 else (math.sin(a * L) / math.sin(a)) ** 2
        assert abs(v - expect) <= 2e-6 * L * L


def test_adjacent_bins_orthogonal(oracle_lib):
    """With step * L / Fs an integer number of cycles, a transmission on bin k
    gives exactly zero correlation (up to complex64 input rounding) at its lag
    in bins k-1 and k+1."""
    C, spc, N, fs = 32, 2, 400, 8e6
    L = C * spc
    chips = siggen.make_codes(8, 1, C)
    freqs, step = oracle.snap_bins(fs, L, 3, 0.0, 125e3)
    assert step * L / fs == 1.0
    x, _ = siggen.make_block(2, N, chips, spc, fs, freqs, 1, snr_db=(0.0, 0.0), noise=False,
                             tags=[0], delays=[77], fracs=[0.0], bins=[1], phases=[0.0])
    v = oracle.corr_power_at(x, chips, spc, freqs, fs, [0, 0, 0], [0, 1, 2], [77, 77, 77])
    assert abs(v[1] - L * L) < 1e-4 * L * L
    assert v[0] < 1e-8 * L * L and v[2] < 1e-8 * L * L


def test_linear_interpolation_injection(oracle_lib):
    """x = (1-phi) s[n-D] + phi s[n-D-1]  =>  c[tau] = (1-phi) R[tau-D] + phi R[tau-D-1],
    R the template autocorrelation (numpy.correlate 'full')."""
    C, spc, N = 40, 3, 400
    L = C * spc
    chips = siggen.make_codes(13, 1, C)
    s = np.repeat(chips[0].astype(np.float64), spc)
    D, phi = 120, 0.3
    x = np.zeros(N, dtype=np.complex128)
    x[D:D + L] += (1 - phi) * s
    x[D + 1:D + 1 + L] += phi * s
    R = np.correlate(s, s, "full")              # R[m + L - 1] = sum_n s[n+m] s[n]

    def Rm(m):
        return R[m + L - 1] if -L < m < L else 0.0
    P = oracle.corr_power(x.astype(np.complex64), chips, spc, [0.0], 1.0)[0, 0]
    expect = np.array([((1 - phi) * Rm(tau - D) + phi * Rm(tau - D - 1)) ** 2 for tau in range(N - L + 1)])
    np.testing.assert_allclose(P, expect, rtol=1e-6, atol=1e-6 * L * L)


def test_noise_only_statistic_is_exponential(oracle_lib):
    """Under CN(0,1) noise, z = P / (L Pxhat) ~ Exp(1) at any lag (KS test on
    lags spaced a template apart, so samples are independent), and the number
    of crossings of theta matches exp(-theta) * tests."""
    from scipy import stats
    C, spc, N = 64, 2, 20000
    L = C * spc
    chips = siggen.make_codes(99, 2, C)
    zs = []
    crossings, tests = 0, 0
    theta = 4.0
    for seed in range(6):
        x, _ = siggen.make_block(seed, N, chips, spc, 1e6, [0.0], 0)
        P = oracle.corr_power(x, chips, spc, [0.0, 1e6 / 256], 1e6)
        Px = oracle.block_power(x)
        z = P / (L * Px)
        zs.append(z[:, :, ::L].ravel())
        crossings += int(np.sum(z >= theta))
        tests += z.size
    zs = np.concatenate(zs)
    assert stats.kstest(zs, "expon").pvalue > 1e-3
    expect = math.exp(-theta) * tests
    assert abs(crossings - expect) < 0.25 * expect


def test_parabola_identities():
    # exact vertex of a sampled parabola
    for v in (-0.4, -0.1, 0.0, 0.25, 0.49):
        a, c0 = -3.0, 10.0
        p = [a * (u - v) ** 2 + c0 for u in (-1, 0, 1)]
        assert abs(oracle.parabola(*p) - v) < 1e-12
    assert oracle.parabola(2.0, 5.0, 2.0) == 0.0
    assert oracle.parabola(1.0, 5.0, 3.0, at_edge=True) == 0.0
    assert oracle.parabola(1.0, 1.0, 1.0) == 0.0           # flat: no vertex
    assert oracle.parabola(3.0, 1.0, 3.0) == 0.0           # convex: no vertex
    assert oracle.parabola(0.0, 1.0, 1.9) == 0.5          # concave, vertex beyond +1: clamped
    # ideal rectangular-chip triangle at 2 samples/chip, peak at offset d:
    # amplitude 1 - |u - d|/2, power its square  =>  delta = d / (3 - 4 d)
    for d in (0.0, 0.1, 0.3, 0.5):
        p = [(1 - abs(u - d) / 2) ** 2 for u in (-1, 0, 1)]
        assert abs(oracle.parabola(*p) - d / (3 - 4 * d)) < 1e-12


def test_argmax_tie_rules():
    P = np.zeros((3, 10))
    P[2, 4] = 5.0
    P[1, 4] = 5.0          # same lag, smaller bin wins
    P[0, 7] = 5.0          # larger lag loses
    k, tau, P0, far, near = oracle.argmax_detect(P)
    assert (k, tau, P0) == (1, 4, 5.0)
    assert far == 5.0      # the tie is visible to the near-tie flag
    P2 = np.zeros((2, 6))
    P2[1, 2] = 1.0
    P2[0, 3] = 1.0
    assert oracle.argmax_detect(P2)[:2] == (1, 2)


def test_threshold_is_inclusive(oracle_lib):
    C, spc, N = 16, 2, 100
    L = C * spc
    chips = np.ones((1, C), dtype=np.int8)
    x = np.zeros(N, dtype=np.complex64)
    x[10:10 + L] = 1.0
    Px = oracle.block_power(x)
    z = (L * L) / (L * Px)
    assert oracle.acquire(x, chips, spc, [0.0], 1.0, theta=z)[0]["detected"]
    assert not oracle.acquire(x, chips, spc, [0.0], 1.0, theta=z * (1 + 1e-12))[0]["detected"]


def test_short_block_has_no_lags(oracle_lib):
    chips = siggen.make_codes(1, 2, 50)
    x = np.ones(99, dtype=np.complex64)
    assert oracle.acquire(x, chips, 2, [0.0], 1.0) == []


def test_edge_lags_flagged(oracle_lib):
    C, spc = 32, 2
    L = C * spc
    chips = siggen.make_codes(17, 2, C)
    N = 500
    x, _ = siggen.make_block(3, N, chips, spc, 1.0, [0.0], 2, snr_db=(0.0, 0.0), noise=False,
                             tags=[0, 1], delays=[0, N - L], fracs=[0.0, 0.0], bins=[0, 0])
    res = oracle.acquire(x, chips, spc, [0.0], 1.0, theta=1.0)
    assert res[0]["lag"] == 0 and res[0]["near_edge"] and res[0]["delta"] == 0.0
    assert res[1]["lag"] == N - L and res[1]["near_edge"] and res[1]["delta"] == 0.0


def test_fractional_delay_toa_tracks_truth(oracle_lib):
    """Band-limited fractional delays: ToA is monotone in phi and within the
    interpolation bias of the truth (a loose empirical bound, not a closed form)."""
    C, spc, N = 256, 2, 2000
    chips = siggen.make_codes(31, 1, C)
    toas = []
    for phi in np.linspace(0.0, 0.95, 8):
        x, _ = siggen.make_block(4, N, chips, spc, 1.0, [0.0], 1, snr_db=(10.0, 10.0), noise=False,
                                 tags=[0], delays=[700], fracs=[float(phi)], bins=[0])
        r = oracle.acquire(x, chips, spc, [0.0], 1.0, theta=1.0)[0]
        toas.append(r["toa"])
        assert abs(r["toa"] - (700 + phi)) <= 0.2
    assert all(b > a for a, b in zip(toas, toas[1:]))


def test_generator_noise_power_and_determinism():
    x1, _ = siggen.make_block(123, 1 << 16, siggen.make_codes(1, 1, 8), 2, 1.0, [0.0], 0)
    x2, _ = siggen.make_block(123, 1 << 16, siggen.make_codes(1, 1, 8), 2, 1.0, [0.0], 0)
    assert np.array_equal(x1, x2)
    p = np.mean(np.abs(x1.astype(np.complex128)) ** 2)
    assert abs(p - 1.0) < 0.02
    assert abs(np.mean(x1.real ** 2) - 0.5) < 0.02


def test_power_and_snr_estimates_noise_free_and_statistical():
    """Noise-free replica at amplitude A: power estimate A^2 exactly, SNR +inf.
    Replica plus CN(0, s2) noise: the estimates average to A^2 and A^2/s2."""
    import math
    L = 4096
    g = np.random.default_rng(7)
    s = np.where(g.random(L) < 0.5, -1.0, 1.0)
    A = 0.7
    x = (A * np.exp(0.3j) * s).astype(np.complex64)
    c = np.sum(x.astype(np.complex128) * s)
    a2, snr = oracle.power_snr_estimates(abs(c) ** 2, oracle.energy_at(x, 0, L), L)
    assert abs(a2 - float(np.abs(np.complex64(A * np.exp(0.3j))) ** 2)) < 1e-6 and (snr == math.inf or snr > 1e6)
    s2 = 0.5
    ests = []
    for seed in range(200):
        gg = np.random.default_rng(100 + seed)
        w = np.sqrt(s2 / 2) * (gg.normal(size=L) + 1j * gg.normal(size=L))
        xx = A * s + w
        c = np.sum(xx * s)
        ests.append(oracle.power_snr_estimates(abs(c) ** 2, float(np.sum(np.abs(xx) ** 2)), L))
    a2m = np.mean([e[0] for e in ests])
    snrm = np.median([e[1] for e in ests])
    assert abs(a2m - A * A) < 0.01 and abs(snrm / (A * A / s2) - 1) < 0.05


def test_tracking_task_is_the_one_code_search(oracle_lib):
    """A tracking task for tag t: (bin, lag) is the brute-force argmax of that one
    template's |c|^2 (ties to the smaller lag, then bin) even with other tags'
    transmissions in the block, and the default threshold counts K (N-L+1)
    hypotheses, not T K (N-L+1)."""
    fs = 8e6
    chips = siggen.make_codes(31, 3, 4)
    freqs = [-250e3, 0.0, 375e3]
    x, _ = siggen.make_block(32, 64, chips, 2, fs, freqs, 3, snr_db=(3.0, 3.0), tags=[0, 1, 2],
                             delays=[3, 20, 41], fracs=[0.0, 0.0, 0.0], bins=[2, 0, 1])
    s = [[float(chips[t][n // 2]) for n in range(8)] for t in range(3)]
    B = _brute_power(x, s, freqs, fs)
    for tag in range(3):
        r = oracle.track(x, chips, 2, freqs, fs, tag)
        Bt = B[tag]
        best = max(((Bt[k, tau], -tau, -k) for k in range(3) for tau in range(Bt.shape[1])))
        assert (r["bin"], r["lag"]) == (-best[2], -best[1]) and r["tag"] == tag
        assert abs(r["peak_power"] - best[0]) <= 1e-9 * best[0]
        assert r["theta"] == math.log(3 * 57 / 1e-3)
    assert oracle.track(x[:7], chips, 2, freqs, fs, 0) is None


def test_tracking_task_exact_recovery(oracle_lib):
    """Noise-free packet of tag 2 in a block 1.5 L long among other tags' packets:
    lag exact, P = L^2 exactly, vertex exactly on the lag."""
    C, spc, fs = 256, 2, 8e6
    L = C * spc
    N = 3 * L // 2
    chips = siggen.make_codes(33, 4, C)
    x, _ = siggen.make_block(34, N, chips, spc, fs, [0.0], 2, snr_db=(0.0, 0.0), noise=False,
                             tags=[2, 0], delays=[100, 200], fracs=[0.0, 0.0], bins=[0, 0], phases=[0.0, 0.0])
    r = oracle.track(x, chips, spc, [0.0], fs, 2)
    assert r["lag"] == 100 and r["delta"] == 0.0
    # the other packet adds its cross-correlation with tag 2's code: the peak is
    # (L + cross)^2 where cross is the chip-level overlap sum, an integer
    s2 = oracle.templates(chips, spc)[2]
    s0 = oracle.templates(chips, spc)[0]
    cross = float(np.dot(s2[100:], s0[:L - 100]))
    assert r["peak_power"] == (L + cross) ** 2


def test_crossing_count_pins(oracle_lib):
    """The threshold-crossing count of `acquire` against brute force (explicit
    loops over the triple-loop powers), the limits theta -> 0 (every hypothesis
    crosses: K (N-L+1) per tag) and theta above the peak z (none), the
    exponential law under noise (e^-theta of the hypotheses cross), and the
    band around theta."""
    x, chips = _tiny_case(seed=21, N=80)
    fs = 8e6
    freqs = [-250e3, 0.0, 375e3]
    s = [[float(chips[t][n // 2]) for n in range(8)] for t in range(2)]
    B = _brute_power(x, s, freqs, fs)
    px = sum(abs(complex(v)) ** 2 for v in x) / len(x)
    theta = 1.5
    res = oracle.acquire(x, chips, 2, freqs, fs, theta=theta)
    for t in range(2):
        brute = 0
        for k in range(3):
            for tau in range(B.shape[2]):
                brute += B[t, k, tau] / (8 * px) >= theta
        assert res[t]["crossings"] == brute
        lo, hi = res[t]["crossings_band"]
        assert lo <= brute <= hi
    for r in oracle.acquire(x, chips, 2, freqs, fs, theta=1e-300):
        assert r["crossings"] == 3 * (80 - 8 + 1)
    for r in oracle.acquire(x, chips, 2, freqs, fs, theta=1e6):
        assert r["crossings"] == 0
    # noise only: about e^-theta of K (N-L+1) hypotheses per tag cross
    C, spc, N = 64, 2, 20000
    L = C * spc
    chips = siggen.make_codes(5, 3, C)
    total = tests = 0
    for seed in range(3):
        xn, _ = siggen.make_block(300 + seed, N, chips, spc, 1e6, [0.0], 0)
        for r in oracle.acquire(xn, chips, spc, [0.0, 1e6 / 256], 1e6, theta=3.0):
            total += r["crossings"]
            tests += 2 * (N - L + 1)
    expect = math.exp(-3.0) * tests
    assert abs(total - expect) < 0.1 * expect
