"""Acquisition oracle: definitions in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, and where it comes from:

* Replica (Section 3, step 6): tag t's stored replica is the noise-free
  waveform of its code; for BPSK codes that is each +/-1 chip held for `spc`
  samples, s_t[n] = chip_t[floor(n / spc)], n < L = C * spc.
* Correlation (Section 3, step 7; the FFT identity of Section 4.1 is only a
  faster route to it): for each tag t, carrier-offset bin k and valid lag tau,
      c[t,k,tau] = sum_{n<L} x[tau+n] s_t[n] exp(-j 2 pi f_k (tau+n) / Fs),
  tau = 0 .. N-L.  Power P = |c|^2.
* Peak (Section 3, step 8): j = argmax |xcorr|, here over all bins and lags of
  one tag, ties to the smaller lag, then the smaller bin; one detection per
  tag per block.  Detected iff z = P / (L * Pxhat) >= theta, where Pxhat is the
  mean power of the whole block.
* Interpolation (Section 3, step 8 says the neighbours of the peak are
  interpolated; the interpolant is not named): a parabola through the powers at
  tau*-1, tau*, tau*+1 of bin k*, vertex offset
      delta = (P- - P+) / (2 (P- - 2 P0 + P+)),
  0 at the first/last valid lag or when the parabola is not concave, clamped to
  [-1/2, 1/2]; ToA = tau* + delta.  Also E = sum_{n<L} |x[tau*+n]|^2 (the
  block-side energy under the replica, the paper's q of step 8).
* Frequency grid (readings, no passage): bins are snapped to multiples of
  q = Fs / M_min, M_min = 2^ceil(log2(L+1)), step = max(1, round(step/q)) q,
  centre = round(centre/q) q, f_k = centre + (k - (K-1)/2) step, K odd.
* Default threshold (reading): theta = ln(T K (N-L+1) / 1e-3), a 1e-3
  expected false alarms per block under noise, where z ~ Exp(1).
* Threshold crossings (reading: the detection test applied to every
  hypothesis, not only to the peak): the number of (bin, lag) of a tag with
  z >= theta.  Reported with a band, the counts at theta (1 +- CROSS_REL),
  inside which an implementation deciding on FP32 powers must fall.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

__all__ = [
    "build_library", "library_path", "rotation_grid", "snap_bins", "templates",
    "block_power", "corr_power", "corr_power_at", "corr_power_fft",
    "default_threshold", "argmax_detect", "parabola", "energy_at", "power_snr_estimates",
    "acquire", "track", "crossings", "NEAR_TIE_REL", "NEAR_THRESHOLD_REL", "CROSS_REL", "num_threads",
    "set_threads",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")

# Decisions this close to a tie (or to the threshold) are flagged, not pinned.
NEAR_TIE_REL = 1e-5
NEAR_THRESHOLD_REL = 1e-5
# Relative band of the threshold-crossing count (FP32 powers err by <= 1e-4 P).
CROSS_REL = 1e-4


# --------------------------------------------------------------------------- C library
def library_path() -> str:
    return _LIB


def build_library(force: bool = True) -> str:
    """Compile direct.c -> _direct.so with gcc (OpenMP, -O3, IEEE arithmetic, baseline
    x86-64 so the same object runs on any host)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_library(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.oracle_corr_power.argtypes = [P(ctypes.c_float), ctypes.c_int64, P(ctypes.c_double),
                                          ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double),
                                          ctypes.c_int32, ctypes.c_double, P(ctypes.c_double)]
        lib.oracle_corr_power.restype = ctypes.c_int
        lib.oracle_corr_power_at.argtypes = [P(ctypes.c_float), ctypes.c_int64, P(ctypes.c_double),
                                             ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double),
                                             ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                             P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int64),
                                             P(ctypes.c_double)]
        lib.oracle_corr_power_at.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def set_threads(n: int) -> int:
    """Threads used by the C library's following calls (n < 1: the default).
    Returns the count now in effect."""
    return int(_lib().oracle_set_threads(int(n)))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------- definitions
def rotation_grid(fs_hz: float, template_len: int):
    """(M_min, q): smallest power of two > L, and the frequency quantum Fs / M_min."""
    m_min = 1 << int(math.ceil(math.log2(template_len + 1)))
    return m_min, fs_hz / m_min


def snap_bins(fs_hz: float, template_len: int, num_bins: int, center_hz: float, step_hz: float):
    """Snapped bin frequencies (Hz, float64 [K]) and the snapped step."""
    if num_bins < 1 or num_bins % 2 == 0:
        raise ValueError("num_bins must be odd and positive")
    _, q = rotation_grid(fs_hz, template_len)
    step_q = max(1, int(round(step_hz / q))) if num_bins > 1 else 0
    centre_q = int(round(center_hz / q))
    half = (num_bins - 1) // 2
    f = np.array([(centre_q + (k - half) * step_q) * q for k in range(num_bins)], dtype=np.float64)
    return f, step_q * q


def templates(chips: np.ndarray, spc: int) -> np.ndarray:
    """s_t[n] = chip_t[floor(n/spc)] as float64 [T][L]."""
    chips = np.asarray(chips, dtype=np.float64)
    T, C = chips.shape
    s = np.empty((T, C * spc), dtype=np.float64)
    for n in range(C * spc):
        s[:, n] = chips[:, n // spc]
    return s


def block_power(x: np.ndarray) -> float:
    """Pxhat = (1/N) sum |x|^2 over the whole block, FP64."""
    x = np.asarray(x).astype(np.complex128)
    return float(np.sum(x.real * x.real + x.imag * x.imag) / x.size)


def _as_c64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex64))


def corr_power(x, chips, spc, freqs_hz, fs_hz) -> np.ndarray:
    """Full P[t][k][tau] by the direct FP64 definition (C, OpenMP)."""
    x = _as_c64(x)
    s = np.ascontiguousarray(templates(chips, spc))
    f = np.ascontiguousarray(np.asarray(freqs_hz, dtype=np.float64))
    T, L = s.shape
    N = x.size
    if N < L:
        return np.zeros((T, f.size, 0))
    P = np.empty((T, f.size, N - L + 1), dtype=np.float64)
    xf = x.view(np.float32)
    rc = _lib().oracle_corr_power(_ptr(xf, ctypes.c_float), N, _ptr(s, ctypes.c_double), T, L,
                                  _ptr(f, ctypes.c_double), f.size, float(fs_hz),
                                  _ptr(P, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle_corr_power failed")
    return P


def corr_power_at(x, chips, spc, freqs_hz, fs_hz, t_idx, k_idx, taus) -> np.ndarray:
    """P at explicit points (t, k, tau) by the direct FP64 definition."""
    x = _as_c64(x)
    s = np.ascontiguousarray(templates(chips, spc))
    f = np.ascontiguousarray(np.asarray(freqs_hz, dtype=np.float64))
    tt = np.ascontiguousarray(np.asarray(t_idx, dtype=np.int32))
    kk = np.ascontiguousarray(np.asarray(k_idx, dtype=np.int32))
    ta = np.ascontiguousarray(np.asarray(taus, dtype=np.int64))
    out = np.empty(tt.size, dtype=np.float64)
    T, L = s.shape
    xf = x.view(np.float32)
    rc = _lib().oracle_corr_power_at(_ptr(xf, ctypes.c_float), x.size, _ptr(s, ctypes.c_double), T, L,
                                     _ptr(f, ctypes.c_double), f.size, float(fs_hz), tt.size,
                                     _ptr(tt, ctypes.c_int32), _ptr(kk, ctypes.c_int32),
                                     _ptr(ta, ctypes.c_int64), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle_corr_power_at failed (bad point)")
    return out


def corr_power_fft(x, chips, spc, freqs_hz, fs_hz, tags: Optional[Iterable[int]] = None):
    """P[k][tau] per tag via the FFT identity of Section 4.1 (FP64, one full-length
    transform, no segmentation): c = ifft(fft(x_k) * conj(fft(s_t)))[tau] for
    tau <= N-L, with transforms of length F >= N so no lag wraps.
    Yields (t, P[K][N-L+1])."""
    try:
        import scipy.fft as sfft
        fft, ifft = (lambda a, n=None: sfft.fft(a, n=n, workers=-1)), (lambda a: sfft.ifft(a, workers=-1))
    except ImportError:  # pragma: no cover
        fft, ifft = np.fft.fft, np.fft.ifft
    x = np.asarray(x, dtype=np.complex64).astype(np.complex128)
    f = np.asarray(freqs_hz, dtype=np.float64)
    s = templates(chips, spc)
    T, L = s.shape
    N = x.size
    lags = N - L + 1
    F = 1 << int(math.ceil(math.log2(max(N, 2))))
    n = np.arange(N, dtype=np.float64)
    Xk = [fft(x * np.exp(-2j * np.pi * fk * n / fs_hz), n=F) for fk in f]
    for t in (range(T) if tags is None else tags):
        St = np.conj(fft(s[t], n=F))
        P = np.empty((f.size, lags))
        for k in range(f.size):
            c = ifft(Xk[k] * St)[:lags]
            P[k] = c.real * c.real + c.imag * c.imag
        yield t, P


def default_threshold(num_tags: int, num_bins: int, n: int, template_len: int) -> float:
    """theta = ln(T K (N-L+1) / 1e-3)."""
    tests = num_tags * num_bins * max(n - template_len + 1, 1)
    return math.log(tests / 1e-3)


def argmax_detect(Pt: np.ndarray, window: int = 1):
    """Global argmax of one tag's P[k][tau]: ties to the smaller tau, then the
    smaller k.  Returns (k, tau, P0, runner_up_far, runner_up_near) where the
    runner-ups are the largest other values outside / inside a +/-window lag
    neighbourhood of the peak in the same bin."""
    K, lags = Pt.shape
    flat = Pt.T.reshape(-1)                 # index = tau*K + k
    i = int(np.argmax(flat))                # first maximum: smallest tau, then k
    tau, k = divmod(i, K)
    P0 = float(Pt[k, tau])
    lo, hi = max(0, tau - window), min(lags, tau + window + 1)
    near = Pt[k, lo:hi].copy()
    near[tau - lo] = -np.inf
    masked = Pt.copy()
    masked[k, lo:hi] = -np.inf
    far = float(np.max(masked)) if masked.size else -np.inf
    nr = float(np.max(near)) if near.size else -np.inf
    return k, tau, P0, far, nr


def parabola(p_minus: float, p0: float, p_plus: float, at_edge: bool = False) -> float:
    """Vertex offset of the parabola through (-1, P-), (0, P0), (+1, P+)."""
    if at_edge:
        return 0.0
    den = p_minus - 2.0 * p0 + p_plus
    if not den < 0.0:
        return 0.0
    d = 0.5 * (p_minus - p_plus) / den
    return min(0.5, max(-0.5, d))


def energy_at(x, tau: int, template_len: int) -> float:
    seg = np.asarray(x[tau:tau + template_len]).astype(np.complex128)
    return float(np.sum(seg.real * seg.real + seg.imag * seg.imag))


def power_snr_estimates(P0: float, E: float, L: int):
    """Relative power and SNR at a peak (the paper's power and SNR sums of
    Section 3 step 8, read for a unit-modulus replica): x = A s e^{j phi} + w
    gives c = A L e^{j phi} + noise, so A^2 is estimated by P / L^2; the
    energy under the replica is E = L (A^2 + sigma^2), so
    sigma^2 = (E - P / L) / L and SNR = A^2 / sigma^2 (+inf when sigma^2 <= 0)."""
    a2 = P0 / (float(L) * float(L))
    s2 = (E - P0 / float(L)) / float(L)
    return a2, (a2 / s2 if s2 > 0.0 else float("inf"))


def crossings(Pt: np.ndarray, theta: float, template_len: int, px: float):
    """(count, low, high): hypotheses of one tag's P[k][tau] with z = P / (L Pxhat) >= theta,
    and the counts at theta (1 + CROSS_REL) and theta (1 - CROSS_REL).  None cross when
    Pxhat is 0."""
    if not px > 0.0:
        return 0, 0, 0
    thr = theta * float(template_len) * px
    return (int(np.count_nonzero(Pt >= thr)), int(np.count_nonzero(Pt >= thr * (1.0 + CROSS_REL))),
            int(np.count_nonzero(Pt >= thr * (1.0 - CROSS_REL))))


def acquire(x, chips, spc, freqs_hz, fs_hz, theta: Optional[float] = None, method: str = "direct",
            refine_window: int = 1, tags: Optional[Sequence[int]] = None):
    """Per-tag acquisition result (list of dicts) by the definitions above.

    method="direct": full P from the C definition (small shapes);
    method="fft": argmax from the FFT identity, peak triple from the direct
    definition at the three lags (large shapes).
    """
    chips = np.asarray(chips)
    T, C = chips.shape
    L = C * spc
    x64 = np.asarray(x, dtype=np.complex64)
    N = x64.size
    f = np.asarray(freqs_hz, dtype=np.float64)
    K = f.size
    if theta is None:
        theta = default_threshold(T, K, N, L)
    Px = block_power(x64)
    out = []
    if N < L:
        return out
    tag_list = list(range(T)) if tags is None else list(tags)
    if method == "direct":
        P = corr_power(x64, chips, spc, f, fs_hz)
        it = ((t, P[t]) for t in tag_list)
    elif method == "fft":
        it = corr_power_fft(x64, chips, spc, f, fs_hz, tags=tag_list)
    else:
        raise ValueError(method)
    lags = N - L + 1
    for t, Pt in it:
        cross = crossings(Pt, theta, L, Px)
        k, tau, P0, far, near = argmax_detect(Pt, window=refine_window)
        trip_taus = [tau - 1, tau, tau + 1]
        if method == "fft":
            ok = [q for q in trip_taus if 0 <= q < lags]
            vals = corr_power_at(x64, chips, spc, f, fs_hz, [t] * len(ok), [k] * len(ok), ok)
            pv = dict(zip(ok, vals))
            P0 = pv[tau]
        else:
            pv = {q: float(Pt[k, q]) for q in trip_taus if 0 <= q < lags}
        edge = tau == 0 or tau == lags - 1
        d = parabola(pv.get(tau - 1, 0.0), P0, pv.get(tau + 1, 0.0), at_edge=edge)
        z = P0 / (L * Px) if Px > 0 else 0.0
        E = energy_at(x64, tau, L)
        a2, snr = power_snr_estimates(P0, E, L)
        out.append(dict(
            tag=int(t), detected=bool(z >= theta), bin=int(k), lag=int(tau), delta=float(d),
            toa=float(tau + d), peak_power=float(P0), z=float(z), energy=E, power=a2, snr=snr,
            block_power=Px, freq_hz=float(f[k]), near_edge=bool(edge),
            near_tie=bool(far >= P0 * (1 - NEAR_TIE_REL) or near >= P0 * (1 - 1e-12)),
            near_threshold=bool(abs(z - theta) <= NEAR_THRESHOLD_REL * theta), theta=float(theta),
            crossings=cross[0], crossings_band=(cross[1], cross[2]),
        ))
    return out


def track(x, chips, spc, freqs_hz, fs_hz, tag: int, theta: Optional[float] = None, method: str = "direct"):
    """One tracking-mode task (Section 2): look for one packet of one given tag
    in a block.  The acquisition of `acquire` restricted to that single code;
    the default threshold counts the hypotheses of one code, K (N-L+1).
    Returns the tag's result dict (tag = the given index)."""
    chips = np.asarray(chips)
    one = chips[int(tag):int(tag) + 1]
    res = acquire(x, one, spc, freqs_hz, fs_hz, theta=theta, method=method)
    if not res:
        return None
    r = dict(res[0])
    r["tag"] = int(tag)
    return r
