"""Pins of the FSK searching-pipeline oracle (oracle/fsk.py) against closed
forms, identities and brute force."""
import math

import numpy as np
import pytest

from oracle import fsk

FS = 8e6


def _brute_fir(x, h):
    y = []
    for n in range(len(x)):
        acc = 0j
        for k in range(len(h)):
            if 0 <= n - k:
                acc += complex(h[k]) * complex(x[n - k])
        y.append(acc)
    return np.array(y)


def test_iq_conversion_is_exact():
    iq = np.array([[1, -2], [32767, -32768], [0, 5]], dtype=np.int16)
    x = fsk.iq_to_complex(iq)
    assert list(x) == [1 - 2j, 32767 - 32768j, 5j]


def test_lo_mix_brings_a_tone_to_dc():
    n = np.arange(5000)
    f = 1234567.0
    x = 3.0 * np.exp(2j * np.pi * f * n / FS)
    np.testing.assert_allclose(fsk.lo_mix(x, f, FS), 3.0, rtol=0, atol=1e-9)


def test_fir_against_loops_and_composition():
    g = np.random.default_rng(1)
    x = g.standard_normal(40) + 1j * g.standard_normal(40)
    a = g.standard_normal(7) + 1j * g.standard_normal(7)
    b = g.standard_normal(4) + 1j * g.standard_normal(4)
    np.testing.assert_allclose(fsk.fir(x, a), _brute_fir(x, a), atol=1e-12)
    # filters in sequence = the composed filter (causal, same length)
    np.testing.assert_allclose(fsk.fir(fsk.fir(x, a), b), fsk.fir(x, fsk.compose(a, b)), atol=1e-12)
    assert fsk.compose(a, b).size == 10


def test_matched_filter_gains():
    """After a full bit of tone f1: |f1| = mf_len (coherent sum); |f0| is the
    Dirichlet kernel of the tone spacing."""
    mf, f1, f0 = 8, 250e3, -250e3
    n = np.arange(64)
    y = np.exp(2j * np.pi * f1 * n / FS + 0.7j)
    o1 = fsk.fir(y, fsk.tone_matched_filter(f1, mf, FS))
    o0 = fsk.fir(y, fsk.tone_matched_filter(f0, mf, FS))
    np.testing.assert_allclose(np.abs(o1[mf - 1:]), mf, atol=1e-12)
    dfe = (f1 - f0) / FS
    want = abs(math.sin(math.pi * dfe * mf) / math.sin(math.pi * dfe))
    np.testing.assert_allclose(np.abs(o0[mf - 1:]), want, atol=1e-12)


def test_demod_identities():
    g = np.random.default_rng(2)
    f1 = g.standard_normal(100) + 1j * g.standard_normal(100)
    f0 = g.standard_normal(100) + 1j * g.standard_normal(100)
    f0[3] = 0
    f1[5] = f0[5] = 0
    d, u = fsk.demod(f1, f0)
    assert np.all(np.abs(d) <= 1) and d[3] == 1.0 and d[5] == 0.0 and u[5] == 0.0
    np.testing.assert_allclose(d * (np.abs(f1) + np.abs(f0)), u, atol=1e-12)
    d2, u2 = fsk.demod(f0, f1)
    np.testing.assert_array_equal(d2, -d)
    np.testing.assert_array_equal(u2, -u)


def test_cpfsk_phase_continuity():
    bits = [1, 0, 0, 1, 1, 0]
    f1, f0, sps = 250e3, -250e3, 8
    s = fsk.cpfsk(bits, sps, f1, f0, FS)
    assert s.size == 48 and s[0] == 1.0
    np.testing.assert_allclose(np.abs(s), 1.0, atol=1e-15)
    step = s[1:] / s[:-1]
    want = np.exp(2j * np.pi * np.where(np.repeat(bits, sps)[:-1] == 1, f1, f0) / FS)
    np.testing.assert_allclose(step, want, atol=1e-12)


def test_replica_template_span():
    g = np.random.default_rng(3)
    bits = g.integers(0, 2, 40)
    bp = g.standard_normal(21) + 1j * g.standard_normal(21)
    dc = fsk.replica_template(bits, FS, bp, 250e3, -250e3, 8)
    assert dc.size == 40 * 8 + 21 + 8 - 2
    # first and last samples see one tap of each composed filter, of equal
    # magnitude (unit-modulus tones): d = 0 there, nonzero inside
    assert abs(dc[0]) < 1e-12 and dc[-1] == 0.0 and np.count_nonzero(np.abs(dc) > 1e-3) > 300
    # the same steps on a longer zero padding: nothing after the span
    r = np.concatenate((fsk.cpfsk(bits, 8, 250e3, -250e3, FS), np.zeros(200)))
    g1 = fsk.compose(bp, fsk.tone_matched_filter(250e3, 8, FS))
    g0 = fsk.compose(bp, fsk.tone_matched_filter(-250e3, 8, FS))
    d, _ = fsk.demod(fsk.fir(r, g1), fsk.fir(r, g0))
    np.testing.assert_allclose(d[:dc.size], dc, atol=1e-12)
    assert np.all(d[dc.size:] == 0.0)


def test_xcorr_brute_force_and_fft_identity():
    g = np.random.default_rng(4)
    d = g.standard_normal(50)
    dc = g.standard_normal(9)
    c = fsk.fsk_xcorr(d, dc)
    brute = [sum(dc[i] * d[i + j] for i in range(9)) for j in range(42)]
    np.testing.assert_allclose(c, brute, atol=1e-12)
    np.testing.assert_allclose(fsk.fsk_xcorr_fft(d, dc), c, atol=1e-10)


def _packet_block(bits, D, N, lo, amp, bp, f1, f0, mf, noise=0.0, seed=0):
    r = fsk.cpfsk(bits, mf, f1, f0, FS)
    x = np.zeros(N, dtype=np.complex128)
    x[D:D + r.size] = amp * r
    n = np.arange(N)
    x = x * np.exp(2j * np.pi * lo * n / FS + 0.4j)
    if noise:
        g = np.random.default_rng(seed)
        x += noise * (g.standard_normal(N) + 1j * g.standard_normal(N)) / math.sqrt(2)
    iq = np.stack([np.round(x.real), np.round(x.imag)], axis=1)
    return np.clip(iq, -32768, 32767).astype(np.int16)


def test_noise_free_packet_is_recovered_exactly():
    """Mixed down to baseband and filtered, a packet at delay D demodulates to
    the replica's d^(c) shifted by D (d is invariant to the amplitude and the
    carrier phase), so the peak is at D with z = 1 up to int16 rounding, and the
    replica's autocorrelation is symmetric, so delta = 0."""
    g = np.random.default_rng(5)
    bits = g.integers(0, 2, 64)
    bp = np.exp(-0.5 * ((np.arange(31) - 15) / 5.0) ** 2) * np.exp(2j * np.pi * 0.01 * np.arange(31))
    f1, f0, mf, lo = 250e3, -250e3, 8, 1.5e6
    tmpl = [fsk.replica_template(b, FS, bp, f1, f0, mf) for b in (g.integers(0, 2, 64), bits)]
    iq = _packet_block(bits, 333, 2000, lo, 12000.0, bp, f1, f0, mf)
    d, u = fsk.front_end(iq, FS, lo, bp, f1, f0, mf)
    r = fsk.fsk_acquire(d, u, tmpl)
    assert r[1]["lag"] == 333 and r[1]["z"] > 1 - 1e-6 and abs(r[1]["delta"]) < 1e-3
    assert r[0]["z"] < 0.2
    ec = float(np.dot(tmpl[1], tmpl[1]))
    assert abs(r[1]["xcorr"] - ec) <= 1e-5 * ec and abs(r[1]["q"] - ec) <= 1e-5 * ec


def test_noisy_packet_found_and_acquire_methods_agree():
    g = np.random.default_rng(6)
    bits = g.integers(0, 2, 128)
    bp = np.exp(-0.5 * ((np.arange(41) - 20) / 8.0) ** 2).astype(complex)
    f1, f0, mf, lo = 200e3, -200e3, 8, -0.7e6
    tmpl = [fsk.replica_template(bits, FS, bp, f1, f0, mf)]
    iq = _packet_block(bits, 1500, 4000, lo, 300.0, bp, f1, f0, mf, noise=600.0, seed=7)
    d, u = fsk.front_end(iq, FS, lo, bp, f1, f0, mf)
    a = fsk.fsk_acquire(d, u, tmpl)[0]
    b = fsk.fsk_acquire(d, u, tmpl, method="fft")[0]
    assert a["lag"] == 1500 and b["lag"] == 1500
    for key in ("xcorr", "q", "p", "z", "toa"):
        assert a[key] == pytest.approx(b[key], rel=1e-12, abs=1e-12)


def _brute_front_u(iq, lo, bp, f1, f0, mf):
    """u = |f1| - |f0| of Section 3, steps 1-5, by explicit loops: the int16 pairs,
    the mix by exp(-j 2 pi lo n / Fs), the band-pass filter, then each tone's
    matched filter as its own sum (no composed filter)."""
    x = [complex(int(i), int(q)) * complex(math.cos(2 * math.pi * lo * n / FS), -math.sin(2 * math.pi * lo * n / FS))
         for n, (i, q) in enumerate(iq)]
    y = _brute_fir(x, bp)
    out = []
    for n in range(len(y)):
        acc = []
        for f in (f1, f0):
            s = 0j
            for m in range(mf):                 # conj(tone[m]) y[n - mf + 1 + m]
                idx = n - mf + 1 + m
                if idx >= 0:
                    s += complex(math.cos(2 * math.pi * f * m / FS), -math.sin(2 * math.pi * f * m / FS)) * y[idx]
            acc.append(abs(s))
        out.append(acc[0] - acc[1])
    return np.array(out)


def test_p_c_pinned_by_loops_identity_and_noise_free_replica():
    """p_c (Section 3, step 8) is the sum over the replica span of d^(c)[i] times
    u[i + j*].  Three pins, each failing for a swapped d/u or a shifted window:
    (1) explicit loops over a brute-force u at the detected lag; (2) with u
    replaced by d the same sum is the correlation peak w_c; (3) a noise-free
    packet of amplitude A at delay D has u[D + i] = A u^(c)[i], u^(c) the
    replica's own u, so p_c = A sum d^(c) u^(c) (int16 rounding aside)."""
    g = np.random.default_rng(11)
    bits = g.integers(0, 2, 24)
    bp = np.exp(-0.5 * ((np.arange(15) - 7) / 3.0) ** 2) * np.exp(2j * np.pi * 0.02 * np.arange(15))
    f1, f0, mf, lo, D, amp = 250e3, -250e3, 8, 1.2e6, 57, 9000.0
    dc = fsk.replica_template(bits, FS, bp, f1, f0, mf)
    n = dc.size
    iq = _packet_block(bits, D, 400, lo, amp, bp, f1, f0, mf, noise=300.0, seed=12)
    d, u = fsk.front_end(iq, FS, lo, bp, f1, f0, mf)
    r = fsk.fsk_acquire(d, u, [dc])[0]
    assert r["lag"] == D
    # (1) loops over u from explicit filter sums
    ub = _brute_front_u(iq, lo, bp, f1, f0, mf)
    np.testing.assert_allclose(u, ub, rtol=0, atol=1e-8 * np.max(np.abs(ub)))
    p_loop = 0.0
    for i in range(n):
        p_loop += dc[i] * ub[i + D]
    assert r["p"] == pytest.approx(p_loop, rel=1e-10)
    shifted = sum(dc[i] * ub[i + D + 1] for i in range(n))
    assert abs(shifted - p_loop) > 1e-3 * abs(p_loop)        # the window offset matters
    # (2) u -> d turns p_c into w_c
    r_dd = fsk.fsk_acquire(d, d, [dc])[0]
    assert r_dd["p"] == pytest.approx(r["xcorr"], rel=1e-12)
    assert abs(r["p"] - r["xcorr"]) > 1.0                    # u and d differ in scale
    # (3) noise-free packet: p_c = A * sum d^(c) u^(c)
    iq0 = _packet_block(bits, D, 400, lo, amp, bp, f1, f0, mf)
    d0, u0 = fsk.front_end(iq0, FS, lo, bp, f1, f0, mf)
    r0 = fsk.fsk_acquire(d0, u0, [dc])[0]
    rep = fsk.cpfsk(bits, mf, f1, f0, FS)
    rep = np.concatenate((rep, np.zeros(len(bp) + mf - 2)))
    g1 = fsk.compose(bp, fsk.tone_matched_filter(f1, mf, FS))
    g0 = fsk.compose(bp, fsk.tone_matched_filter(f0, mf, FS))
    _, uc = fsk.demod(fsk.fir(rep, g1), fsk.fir(rep, g0))
    assert r0["lag"] == D
    assert r0["p"] == pytest.approx(amp * float(np.dot(dc, uc)), rel=2e-3)
