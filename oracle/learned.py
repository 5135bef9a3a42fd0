"""Learned-proposal oracle: STFT power map, 1-D CNN, loss, optimiser and the
proposal-to-segment mapping, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper searches exhaustively; the proposal stage is an extension with no
passage of its own, so everything here is a stated reading, built from
textbook definitions:

* Power map.  Frames of 256 samples with hop 128, f = 0 .. F-1,
  F = floor((N - 256) / 128) + 1.  Periodic Hann window
  w[n] = (1 - cos(2 pi n / 256)) / 2.  P[f][b] = |sum_n w[n] x[128 f + n]
  exp(-j 2 pi b n / 256)|^2, b in FFT order.  The map is ln(P / med), med the
  lower median of all F*256 values of the block (the ceil(F*256/2)-th
  smallest), so that the map does not depend on the receiver gain (0 when
  that median is 0).
* Network.  Four "same"-padded dilated convolutions over frames, kernel 5,
  dilations 1, 2, 4, 8, channels 256 -> 64 -> 64 -> 64 -> 64, each followed by
  ReLU, then a 1x1 head 64 -> 1 giving one logit per frame:
      h_l[f][o] = relu(b_l[o] + sum_{i<5} sum_c W_l[i][c][o] h_{l-1}[f + d_l (i - 2)][c])
  with h_{l-1} = 0 outside 0 .. F-1.
* Reduced-precision network.  A bf16 network stores its conv weights and every
  layer's output rounded to bf16 (nearest, ties to even); biases, the head and
  all sums stay exact.  Its gradient is the FP64 gradient of that function.
* Training.  Frame label 1 when at least half of the frame (128 samples) lies
  inside a transmission [D, D + L).  Loss: mean over frames of the binary
  cross-entropy with logits and a positive-class weight,
      l = -(pw * y * log s(z) + (1 - y) * log(1 - s(z))).
  Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
* Proposals.  Window score c[f] = sum of the logits of frames f-63 .. f+64
  (128 frames, the span of a 16384-sample transmission at hop 128; frames
  outside the block count 0).  Every frame with c[f] >= kappa is proposed.
  Frame f proposes every lag whose replica covers the whole frame,
  tau in [128 f + 256 - L, 128 f] intersected with [0, N - L]; the search then
  runs on every overlap-save segment j (lags jV .. jV+V-1) meeting a proposed
  range, so its values are those of the exhaustive search on those lags.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

WIN = 256
HOP = 128
SPAN = 128              # window-score length, frames
CHANNELS = 64
KERNEL = 5
DILATIONS = (1, 2, 4, 8)

__all__ = [
    "WIN", "HOP", "SPAN", "CHANNELS", "KERNEL", "DILATIONS",
    "num_frames", "hann", "stft_power", "lower_median", "power_map", "frame_labels",
    "CNN", "init_cnn", "conv_same", "cnn_forward", "cnn_backward", "bce_with_logits", "bf16_round",
    "bf16_network",
    "adam_step", "window_scores", "propose", "frame_lag_range", "segments_for_ranges",
]


# ---------------------------------------------------------------- power map
def num_frames(n: int) -> int:
    return 0 if n < WIN else (n - WIN) // HOP + 1


def hann(n: int = WIN) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * i / n))


def stft_power(x) -> np.ndarray:
    """P[f][b] = |DFT_256(w * frame f)|^2, FP64, [F][256]."""
    x = np.asarray(x).astype(np.complex128)
    F = num_frames(x.size)
    idx = np.arange(F)[:, None] * HOP + np.arange(WIN)[None, :]
    fr = x[idx] * hann()[None, :]
    X = np.fft.fft(fr, axis=1)
    return X.real ** 2 + X.imag ** 2


def lower_median(v) -> float:
    """The ceil(n/2)-th smallest value (index (n-1)//2 in ascending order)."""
    a = np.sort(np.asarray(v, dtype=np.float64).reshape(-1))
    return float(a[(a.size - 1) // 2])


def power_map(x) -> Tuple[np.ndarray, float]:
    """ln(P / med) and med.  Bins with P == 0 map to ln(tiny / med); a block
    whose median is 0 (more than half the bins exactly empty) maps to 0."""
    P = stft_power(x)
    med = lower_median(P)
    if med == 0.0:
        return np.zeros_like(P), 0.0
    tiny = np.finfo(np.float64).tiny
    return np.log(np.maximum(P, tiny) / med), med


def frame_labels(n: int, delays: Sequence[float], L: int) -> np.ndarray:
    """1 where at least HOP samples of frame f lie in some [D, D+L), integer D."""
    F = num_frames(n)
    cover = np.zeros(n + 1, dtype=np.int64)
    for D in delays:
        a = int(D)
        b = min(a + L, n)
        if b > a:
            cover[a] += 1
            cover[b] -= 1
    inside = np.cumsum(cover)[:n] > 0
    csum = np.concatenate([[0], np.cumsum(inside)])
    starts = np.arange(F) * HOP
    return ((csum[starts + WIN] - csum[starts]) >= WIN // 2).astype(np.float64)


# ---------------------------------------------------------------- network
@dataclass
class CNN:
    W: List[np.ndarray]                 # [5][cin][64] per layer
    b: List[np.ndarray]                 # [64] per layer
    wh: np.ndarray                      # [64]
    bh: float

    def params(self) -> Dict[str, np.ndarray]:
        out = {}
        for l in range(len(self.W)):
            out[f"W{l}"] = self.W[l]
            out[f"b{l}"] = self.b[l]
        out["wh"] = self.wh
        out["bh"] = np.array([self.bh])
        return out

    @staticmethod
    def from_params(p: Dict[str, np.ndarray]) -> "CNN":
        n = sum(1 for k in p if k.startswith("W"))
        return CNN([np.asarray(p[f"W{l}"], np.float64) for l in range(n)],
                   [np.asarray(p[f"b{l}"], np.float64) for l in range(n)],
                   np.asarray(p["wh"], np.float64), float(np.asarray(p["bh"]).reshape(-1)[0]))


def init_cnn(seed: int, cin: int = WIN) -> CNN:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    g = np.random.default_rng(seed)
    W, b = [], []
    c = cin
    for _ in DILATIONS:
        W.append(g.normal(0.0, np.sqrt(2.0 / (KERNEL * c)), size=(KERNEL, c, CHANNELS)))
        b.append(np.zeros(CHANNELS))
        c = CHANNELS
    return CNN(W, b, g.normal(0.0, np.sqrt(1.0 / CHANNELS), size=CHANNELS), 0.0)


def _shift(h: np.ndarray, s: int) -> np.ndarray:
    """out[f] = h[f + s], zero outside."""
    F = h.shape[0]
    out = np.zeros_like(h)
    if s >= 0:
        if s < F:
            out[:F - s] = h[s:]
    else:
        if -s < F:
            out[-s:] = h[:F + s]
    return out


def conv_same(h: np.ndarray, W: np.ndarray, b: np.ndarray, d: int) -> np.ndarray:
    """b[o] + sum_i sum_c W[i][c][o] h[f + d (i - 2)][c] (pre-activation)."""
    out = np.broadcast_to(b, (h.shape[0], W.shape[2])).copy()
    for i in range(W.shape[0]):
        out += _shift(h, d * (i - KERNEL // 2)) @ W[i]
    return out


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bf16 value (8-bit significand), ties to even, via the
    FP32 bit pattern: keep the top 16 bits after adding 0x7fff plus the lowest
    kept bit.  Finite inputs; returned as FP64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_network(net: CNN) -> CNN:
    """The network with its conv weights stored in bf16 (biases and head stay FP32-exact)."""
    return CNN([bf16_round(W) for W in net.W], [b.copy() for b in net.b], net.wh.copy(), net.bh)


def cnn_forward(net: CNN, m: np.ndarray, act_round=None):
    """Logits [F] and the activations needed by the backward pass.  act_round,
    when given, is applied to every layer's output (bf16 activation storage)."""
    h = [np.asarray(m, np.float64)]
    for l, d in enumerate(DILATIONS):
        a = np.maximum(conv_same(h[-1], net.W[l], net.b[l], d), 0.0)
        h.append(act_round(a) if act_round is not None else a)
    y = h[-1] @ net.wh + net.bh
    return y, h


def cnn_backward(net: CNN, h: List[np.ndarray], dy: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of sum_f dy[f] y[f] with respect to every parameter."""
    grads = {"wh": h[-1].T @ dy, "bh": np.array([dy.sum()])}
    dh = np.outer(dy, net.wh)                       # d/dh_4
    for l in reversed(range(len(DILATIONS))):
        d = DILATIONS[l]
        da = dh * (h[l + 1] > 0)                    # through ReLU (h = relu(a), a > 0 <=> h > 0)
        grads[f"b{l}"] = da.sum(axis=0)
        gW = np.zeros_like(net.W[l])
        dprev = np.zeros_like(h[l])
        for i in range(KERNEL):
            s = d * (i - KERNEL // 2)
            hs = _shift(h[l], s)
            gW[i] = hs.T @ da
            dprev += _shift(da @ net.W[l][i].T, -s)  # adjoint of the shift
        grads[f"W{l}"] = gW
        dh = dprev
    return grads


def bce_with_logits(z: np.ndarray, y: np.ndarray, pos_weight: float = 1.0):
    """Mean weighted binary cross-entropy and its gradient with respect to z."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    log_s = -np.logaddexp(0.0, -z)                  # log sigmoid(z)
    log_1ms = -np.logaddexp(0.0, z)                 # log(1 - sigmoid(z))
    loss = -(pos_weight * y * log_s + (1.0 - y) * log_1ms)
    s = 1.0 / (1.0 + np.exp(-z))
    dz = (pos_weight * y * (s - 1.0) + (1.0 - y) * s) / z.size
    return float(loss.mean()), dz


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update in place (t counts from 1)."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)


# ---------------------------------------------------------------- proposals
def window_scores(y: np.ndarray) -> np.ndarray:
    """c[f] = sum_{i=-63}^{64} y[f + i], zero outside."""
    y = np.asarray(y, np.float64)
    F = y.size
    c = np.zeros(F)
    lo, hi = -(SPAN // 2 - 1), SPAN // 2
    for f in range(F):
        a, b = max(0, f + lo), min(F, f + hi + 1)
        c[f] = y[a:b].sum()
    return c


def propose(c: np.ndarray, kappa: float) -> np.ndarray:
    """Frames whose window score reaches kappa, ascending."""
    return np.flatnonzero(np.asarray(c, np.float64) >= kappa).astype(np.int64)


def frame_lag_range(f: int, n: int, L: int):
    """Lags whose replica covers frame f entirely, within the valid lags; None if empty."""
    lo = max(HOP * f + WIN - L, 0)
    hi = min(HOP * f, n - L)
    return (lo, hi) if lo <= hi else None


def segments_for_ranges(ranges, V: int, n: int, L: int) -> np.ndarray:
    """Overlap-save segments j (lags jV .. min(jV+V, N-L+1)-1) meeting any range."""
    lags = n - L + 1
    S = -(-lags // V) if lags > 0 else 0
    hit = np.zeros(S, dtype=bool)
    for r in ranges:
        if r is None:
            continue
        lo, hi = r
        hit[lo // V: hi // V + 1] = True
    return np.flatnonzero(hit)
