"""FSK searching pipeline oracle (Section 3, steps 1-8): definitions in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, and where it comes from:

* Step 1: int16 (I, Q) pairs become complex samples x = I + jQ (no scaling).
* Step 2: local-oscillator mix, x[n] <- x[n] exp(-j 2 pi f_LO n / Fs), n the
  sample index from the block start (reading: the paper's l is a given
  vector; here it is the complex exponential at f_LO).
* Step 3: band-pass FIR h_BP (200 taps in the paper), applied as a causal
  convolution y[n] = sum_k h_BP[k] x[n-k] with zero samples before the block
  (reading: the paper writes a circulant matrix; the circulant wrap is an
  artefact of its FFT description, the filter is linear).
* Step 4: two matched filters of one bit period (mf_len samples, 8 in the
  paper), one per FSK tone: h_b[k] = exp(-j 2 pi f_b (mf_len-1-k) / Fs), the
  time-reversed conjugate of the tone, so f_b[n] = sum_{m<mf_len}
  conj(tone_b[m]) y[n-mf_len+1+m].  Section 4.1 composes them with the
  band-pass filter: f_b = (h_BP * h_b) * x.
* Step 5: d = (|f1| - |f0|) / (|f1| + |f0|) (the paper's denominator repeats
  |f0|; read as |f1| + |f0|), 0 where both vanish; u = |f1| - |f0|.
* Step 6: the replica r^(c) is a noise-free continuous-phase FSK packet of
  code c (bit b held mf_len samples at tone f1 for a 1 and f0 for a 0, phase
  continuous, starting at 0), zero-padded; steps 3-5 (not 1-2) give d^(c).
  Its nonzero span is n = bits * mf_len + len(h_BP * h_b) - 1 samples.
* Step 7: xcorr[j] = sum_{i<n} d^(c)[i] d[i+j], valid lags j = 0 .. N-n.
* Step 8: j* = argmax_j |xcorr[j]| (ties to the smaller j); a parabola through
  |xcorr| at j*-1, j*, j*+1 (the rule of the acquisition oracle's
  `parabola`); w_c = xcorr[j*], q = sum_{i<n} d[i+j*]^2 and
  p_c = sum_{i<n} d^(c)[i] u[i+j*] (sums over i = 0 .. n-1).  Detection
  statistic (reading, the paper defers to other work): the squared
  normalised correlation z = w_c^2 / (q E_c), E_c = sum d^(c)^2, in [0, 1];
  reported when z >= theta.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .reference import parabola

__all__ = ["iq_to_complex", "lo_mix", "tone_matched_filter", "compose", "fir", "demod", "front_end",
           "cpfsk", "replica_template", "fsk_xcorr", "fsk_xcorr_fft", "fsk_acquire"]


def iq_to_complex(iq) -> np.ndarray:
    """Step 1: int16 [N][2] (I, Q) -> complex128 [N]."""
    a = np.asarray(iq, dtype=np.int16).reshape(-1, 2).astype(np.float64)
    return a[:, 0] + 1j * a[:, 1]


def lo_mix(x, lo_hz: float, fs_hz: float) -> np.ndarray:
    """Step 2: x[n] exp(-j 2 pi f_LO n / Fs), phase from the exact index in FP64."""
    n = np.arange(len(x), dtype=np.float64)
    cyc = np.mod(lo_hz / fs_hz * n, 1.0)
    return np.asarray(x, dtype=np.complex128) * np.exp(-2j * np.pi * cyc)


def tone_matched_filter(f_hz: float, mf_len: int, fs_hz: float) -> np.ndarray:
    """Step 4: h[k] = exp(-j 2 pi f (mf_len-1-k) / Fs), k < mf_len."""
    k = np.arange(mf_len, dtype=np.float64)
    return np.exp(-2j * np.pi * f_hz * (mf_len - 1 - k) / fs_hz)


def compose(h_a, h_b) -> np.ndarray:
    """Section 4.1: the filter equal to h_a followed by h_b (full convolution)."""
    return np.convolve(np.asarray(h_a, dtype=np.complex128), np.asarray(h_b, dtype=np.complex128))


def fir(x, h) -> np.ndarray:
    """Causal FIR: y[n] = sum_k h[k] x[n-k], zero before the block, len(y) = len(x)."""
    x = np.asarray(x, dtype=np.complex128)
    return np.convolve(x, np.asarray(h, dtype=np.complex128))[:len(x)]


def demod(f1, f0):
    """Step 5: (d, u)."""
    a1, a0 = np.abs(f1), np.abs(f0)
    s = a1 + a0
    d = np.where(s > 0, (a1 - a0) / np.where(s > 0, s, 1.0), 0.0)
    return d, a1 - a0


def front_end(iq, fs_hz: float, lo_hz: float, bp, f1_hz: float, f0_hz: float, mf_len: int):
    """Steps 1-5 on an int16 IQ block: (d, u), FP64."""
    x = lo_mix(iq_to_complex(iq), lo_hz, fs_hz)
    g1 = compose(bp, tone_matched_filter(f1_hz, mf_len, fs_hz))
    g0 = compose(bp, tone_matched_filter(f0_hz, mf_len, fs_hz))
    return demod(fir(x, g1), fir(x, g0))


def cpfsk(bits, sps: int, f1_hz: float, f0_hz: float, fs_hz: float) -> np.ndarray:
    """Noise-free continuous-phase FSK: bit b held sps samples at f1 (1) or f0 (0),
    phase starting at 0 and advancing 2 pi f_b / Fs per sample; the phase is
    accumulated in cycles and reduced exactly (FP64)."""
    bits = np.asarray(bits).astype(np.int64)
    f = np.where(np.repeat(bits, sps) == 1, f1_hz, f0_hz) / fs_hz       # cycles per sample
    cyc = np.concatenate(([0.0], np.cumsum(f)[:-1]))
    return np.exp(2j * np.pi * np.mod(cyc, 1.0))


def replica_template(bits, fs_hz: float, bp, f1_hz: float, f0_hz: float, mf_len: int) -> np.ndarray:
    """Step 6: d^(c) over its nonzero span, n = bits*mf_len + len(bp) + mf_len - 2."""
    r = cpfsk(bits, mf_len, f1_hz, f0_hz, fs_hz)
    lg = len(bp) + mf_len - 1
    r = np.concatenate((r, np.zeros(lg - 1)))
    g1 = compose(bp, tone_matched_filter(f1_hz, mf_len, fs_hz))
    g0 = compose(bp, tone_matched_filter(f0_hz, mf_len, fs_hz))
    d, _ = demod(fir(r, g1), fir(r, g0))
    return d


def fsk_xcorr(d, dc) -> np.ndarray:
    """Step 7 by its definition (library correlate, direct sums): lags 0 .. N-n."""
    return np.correlate(np.asarray(d, dtype=np.float64), np.asarray(dc, dtype=np.float64), "valid")


def fsk_xcorr_fft(d, dc) -> np.ndarray:
    """Step 7 through the FFT identity (one full-length transform, no segmentation);
    for blocks too long for the direct sums."""
    d = np.asarray(d, dtype=np.float64)
    dc = np.asarray(dc, dtype=np.float64)
    N, n = d.size, dc.size
    m = 1 << int(np.ceil(np.log2(N + n)))
    c = np.fft.irfft(np.fft.rfft(d, m) * np.conj(np.fft.rfft(dc, m)), m)
    return c[:N - n + 1]


def fsk_acquire(d, u, templates: Sequence[np.ndarray], theta: float = 0.0, method: str = "direct",
                tags: Optional[Sequence[int]] = None):
    """Step 8 for every tag: list of result dicts (all tags, `detected` = z >= theta)."""
    d = np.asarray(d, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    out = []
    tag_list = range(len(templates)) if tags is None else tags
    for t in tag_list:
        dc = np.asarray(templates[t], dtype=np.float64)
        n = dc.size
        if d.size < n:
            continue
        c = fsk_xcorr(d, dc) if method == "direct" else fsk_xcorr_fft(d, dc)
        a = np.abs(c)
        j = int(np.argmax(a))                          # first maximum: the smaller lag
        lags = a.size
        if method != "direct":                         # exact values at the peak triple
            for q in (j - 1, j, j + 1):
                if 0 <= q < lags:
                    c[q] = float(np.dot(dc, d[q:q + n]))
            a = np.abs(c)
            j2 = int(np.argmax(a[max(j - 1, 0):j + 2])) + max(j - 1, 0)
            j = j2
        edge = j == 0 or j == lags - 1
        pm = a[j - 1] if j > 0 else 0.0
        pp = a[j + 1] if j + 1 < lags else 0.0
        delta = parabola(pm, a[j], pp, at_edge=edge)
        w = float(c[j])
        q = float(np.dot(d[j:j + n], d[j:j + n]))
        p = float(np.dot(dc, u[j:j + n]))
        ec = float(np.dot(dc, dc))
        z = w * w / (q * ec) if q > 0 and ec > 0 else 0.0
        second = np.partition(a, -2)[-2] if lags > 1 else 0.0
        out.append(dict(tag=int(t), lag=j, delta=float(delta), toa=float(j + delta), xcorr=w, q=q, p=p, z=z,
                        detected=bool(z >= theta), near_edge=bool(edge),
                        near_tie=bool(lags > 1 and second >= a[j] * (1 - 1e-5))))
    return out
