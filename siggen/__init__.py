"""Seeded synthetic receiver blocks for the acquisition workloads.

This module synthesises what an acquisition receiver records: random BPSK tag
codes, complex white Gaussian noise and transmissions injected at a chosen
integer+fractional delay, carrier offset, phase and per-sample SNR.  It is the
one module that both the oracle tests and the GPU path consume; it holds none
of the acquisition arithmetic (no correlation, no matched filtering, no peak
search, no detection rule).

Conventions (stated once, used everywhere):
  * noise w ~ CN(0, 1): real and imaginary parts i.i.d. N(0, 1/2), so E|w|^2 = 1;
  * a transmission of amplitude A has per-sample SNR A^2 / E|w|^2 = A^2;
  * a tag transmits the rectangular-chip waveform of its +/-1 code, `spc`
    samples per chip, delayed by D + phi samples (D integer, 0 <= phi < 1),
    shifted in frequency by f Hz with absolute sample index n and a random
    carrier phase:  A * wave(n - D - phi) * exp(j(2 pi f n / Fs + theta0));
  * fractional delays are band-limited (phase ramp in the DFT domain of a
    zero-padded copy): sampling a rectangular chip train at a sub-sample
    offset is otherwise indistinguishable from an integer shift;
  * within one block, transmissions come from distinct tags (tags transmit at
    most once per second, far longer than one block).

Every draw comes from numpy's Philox counter-based generator keyed by a
SeedSequence of (seed, stream, ...), so a block is a pure function of its
arguments.  The block is produced in complex128 and rounded once to complex64;
that complex64 array is the input of both the oracle and the GPU path.
"""
from __future__ import annotations

from dataclasses import dataclass, asdict
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "rng", "make_codes", "chip_waveform", "delayed_waveform", "Transmission",
    "make_block", "add_noise", "WORKLOADS", "workload", "batch_lengths", "make_stream_batch",
    "make_tracking_batch", "fsk_bandpass", "make_fsk_bits", "make_fsk_block",
]

# stream identifiers (second SeedSequence word)
_STREAM_CODES = 1
_STREAM_BLOCK = 2
_STREAM_NOISE = 3
_STREAM_LENGTHS = 4


def rng(seed: int, *stream: int) -> np.random.Generator:
    """Philox4x32-10 generator keyed by the seed sequence (seed, *stream)."""
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, *[int(s) & 0xFFFFFFFF for s in stream]])
    return np.random.Generator(np.random.Philox(ss))


def make_codes(seed: int, num_tags: int, num_chips: int) -> np.ndarray:
    """Random +/-1 chip codes, int8 [num_tags][num_chips]; tag t uses stream (CODES, t)."""
    out = np.empty((num_tags, num_chips), dtype=np.int8)
    for t in range(num_tags):
        bits = rng(seed, _STREAM_CODES, t).integers(0, 2, size=num_chips, dtype=np.int8)
        out[t] = (2 * bits - 1).astype(np.int8)
    return out


def chip_waveform(chips: np.ndarray, spc: int) -> np.ndarray:
    """The transmitted baseband waveform of one code: each chip held for spc samples (float64)."""
    return np.repeat(np.asarray(chips, dtype=np.float64), int(spc))


def delayed_waveform(wave: np.ndarray, phi: float):
    """Band-limited copy of `wave` delayed by phi in [0, 1) samples.

    Returns (w, h): w[i] is the delayed waveform at sample offset i - h from the
    integer delay point, so it is added to a block at index D - h + i.  With
    phi == 0 the waveform is returned unchanged (h = 0), no transform applied.
    """
    wave = np.asarray(wave, dtype=np.float64)
    if phi == 0.0:
        return wave.copy(), 0
    L = wave.size
    P = 1 << int(np.ceil(np.log2(L + 128)))
    h = (P - L) // 2
    buf = np.zeros(P)
    buf[h:h + L] = wave
    spec = np.fft.fft(buf)
    k = np.fft.fftfreq(P, d=1.0 / P)           # integer frequencies -P/2..P/2-1
    ramp = np.exp(-2j * np.pi * k * phi / P)
    ramp[P // 2] = np.cos(np.pi * phi)         # Nyquist term: keep the result real
    w = np.fft.ifft(spec * ramp).real
    return w, h


@dataclass
class Transmission:
    """One injected transmission (ground truth of a synthetic block)."""
    tag: int
    delay: int          # integer part D of the delay (samples)
    frac: float         # fractional part phi in [0, 1)
    snr_db: float
    amplitude: float
    phase: float        # carrier phase theta0 (rad)
    freq_hz: float
    bin: int            # index into the candidate frequency list

    @property
    def toa(self) -> float:
        return self.delay + self.frac

    def as_dict(self):
        return asdict(self)


def add_noise(x: np.ndarray, seed: int, sub: int = 0) -> None:
    """Add CN(0,1) noise in place (stream NOISE, sub)."""
    g = rng(seed, _STREAM_NOISE, sub)
    n = x.size
    x += (g.standard_normal(n) + 1j * g.standard_normal(n)) * np.sqrt(0.5)


def make_block(seed: int, n: int, chips: np.ndarray, spc: int, fs_hz: float,
               freqs_hz: Sequence[float], n_tx: int,
               snr_db=(-10.0, -10.0), noise: bool = True,
               tags: Optional[Sequence[int]] = None,
               delays: Optional[Sequence[int]] = None,
               fracs: Optional[Sequence[float]] = None,
               bins: Optional[Sequence[int]] = None,
               phases: Optional[Sequence[float]] = None,
               sub: int = 0):
    """Synthesise one receiver block.

    chips: int8 [T][C] codes; freqs_hz: candidate carrier offsets (the caller
    passes the on-grid frequencies it wants transmissions drawn from);
    snr_db: (lo, hi) per-transmission SNR drawn uniformly in dB.
    Explicit tags/delays/fracs/bins/phases override the random draws.
    Returns (x complex64 [n], list[Transmission]).
    """
    chips = np.asarray(chips)
    T, C = chips.shape
    L = C * spc
    g = rng(seed, _STREAM_BLOCK, sub)
    x = np.zeros(n, dtype=np.complex128)
    txs = []
    if n_tx > 0:
        if n < L:
            raise ValueError("block shorter than a transmission")
        tag_list = list(tags) if tags is not None else list(g.choice(T, size=n_tx, replace=False))
        for i in range(n_tx):
            D = int(delays[i]) if delays is not None else int(g.integers(0, max(n - L, 1)))
            phi = float(fracs[i]) if fracs is not None else float(g.random())
            if D + phi > n - L:
                raise ValueError("transmission does not fit in the block")
            k = int(bins[i]) if bins is not None else int(g.integers(0, len(freqs_hz)))
            lo, hi = snr_db
            snr = float(lo + (hi - lo) * g.random())
            th0 = float(phases[i]) if phases is not None else float(2 * np.pi * g.random())
            A = 10.0 ** (snr / 20.0)
            f = float(freqs_hz[k])
            w, h = delayed_waveform(chip_waveform(chips[tag_list[i]], spc), phi)
            start = D - h
            i0 = max(0, start)
            i1 = min(n, start + w.size)
            idx = np.arange(i0, i1)
            carrier = np.exp(1j * (2 * np.pi * f * idx / fs_hz + th0))
            x[i0:i1] += A * w[i0 - start:i1 - start] * carrier
            txs.append(Transmission(int(tag_list[i]), D, phi, snr, A, th0, f, k))
    if noise:
        add_noise(x, seed, sub)
    return x.astype(np.complex64), txs


# ---------------------------------------------------------------------------
# Workload shapes.  Sizes, rates and distributions of the five acquisition
# workloads; each is a plain description, the arithmetic lives elsewhere.
# ---------------------------------------------------------------------------
WORKLOADS = {
    # one 2^17-sample block, one 1024-chip code at 4 samples/chip, zero offset
    "plain_fp32": dict(num_tags=1, num_chips=1024, spc=4, block_len=1 << 17, fs_hz=8e6,
                       num_bins=1, bin_center_hz=0.0, bin_step_hz=0.0, fft_len=0,
                       n_tx=1, snr_db=(-10.0, -10.0), precision="fp32", seeds=(1000, 1100)),
    # 64 tags x 8192 chips x 2 spc, 2^20 samples at 8 Msps, 11 bins over +/-5 kHz, M = 2^15
    "tagbank_fp32": dict(num_tags=64, num_chips=8192, spc=2, block_len=1 << 20, fs_hz=8e6,
                         num_bins=11, bin_center_hz=0.0, bin_step_hz=1000.0, fft_len=1 << 15,
                         n_tx=10, snr_db=(-15.0, -5.0), precision="fp32", seeds=(2000, 2020)),
    # same bank/signal, spectra stored in fp16 / bf16, fp64 +/-8 re-correlation
    "tagbank_fp16": dict(num_tags=64, num_chips=8192, spc=2, block_len=1 << 20, fs_hz=8e6,
                         num_bins=11, bin_center_hz=0.0, bin_step_hz=1000.0, fft_len=1 << 15,
                         n_tx=10, snr_db=(-15.0, -5.0), precision="fp16", refine_radius=8,
                         seeds=(2000, 2020)),
    "tagbank_bf16": dict(num_tags=64, num_chips=8192, spc=2, block_len=1 << 20, fs_hz=8e6,
                         num_bins=11, bin_center_hz=0.0, bin_step_hz=1000.0, fft_len=1 << 15,
                         n_tx=10, snr_db=(-15.0, -5.0), precision="bf16", refine_radius=8,
                         seeds=(2000, 2020)),
    # 256 tags, 21 bins over +/-10 kHz, 64 uneven blocks in [2^18, 2^21] from 8 receivers
    "batched_stream": dict(num_tags=256, num_chips=8192, spc=2, fs_hz=8e6, num_bins=21,
                           bin_center_hz=0.0, bin_step_hz=1000.0, fft_len=0, num_blocks=64,
                           block_len_log2=(18.0, 21.0), receivers=8, n_tx=(0, 20),
                           snr_db=(-15.0, -5.0), precision="fp32", seeds=(4000, 4005)),
    # tracking tasks: one code per task, blocks 1.5 templates long (the 12 ms
    # window around an 8 ms packet), 256 tasks per batch over the same bank
    "tracking": dict(num_tags=256, num_chips=8192, spc=2, fs_hz=8e6, num_bins=21,
                     bin_center_hz=0.0, bin_step_hz=1000.0, fft_len=0, num_tasks=256,
                     block_factor=1.5, p_present=0.9, n_other=(0, 1), snr_db=(-15.0, -5.0),
                     precision="fp32", seeds=(5000, 5005)),
    # FSK searching task of the paper's shape: a 100 ms window at 8 Msps, 8192-bit
    # packets at 1 Mb/s (8 samples per bit, tones +/-250 kHz), 200-tap band-pass,
    # 128 codes; six packets per window at -10..0 dB, int16 samples
    "fsk_search": dict(num_tags=128, num_bits=8192, sps=8, fs_hz=8e6, block_len=800000, lo_hz=1.0e6,
                       f1_hz=250e3, f0_hz=-250e3, bp_taps=200, bp_cutoff_hz=600e3, n_tx=6,
                       snr_db=(-10.0, 0.0), noise_rms=1000.0, seeds=(6000, 6005)),
    # FSK tracking tasks: 64 tasks per call, each a 12 ms block (96,000 samples) for
    # one of the 128 codes, the code's packet present with probability 0.9
    "fsk_tracking": dict(num_tags=128, num_bits=8192, sps=8, fs_hz=8e6, block_len=96000, lo_hz=1.0e6,
                         f1_hz=250e3, f0_hz=-250e3, bp_taps=200, bp_cutoff_hz=600e3, num_tasks=64,
                         p_present=0.9, snr_db=(-10.0, 0.0), noise_rms=1000.0, seeds=(6100, 6105)),
}


def workload(name: str) -> dict:
    return dict(WORKLOADS[name])


def batch_lengths(seed: int, num_blocks: int, log2_lo: float, log2_hi: float):
    """Block lengths drawn log-uniform: floor(2^U[lo, hi])."""
    g = rng(seed, _STREAM_LENGTHS)
    return [int(np.floor(2.0 ** (log2_lo + (log2_hi - log2_lo) * g.random()))) for _ in range(num_blocks)]


def make_stream_batch(seed: int, chips: np.ndarray, spc: int, fs_hz: float, freqs_hz: Sequence[float],
                      num_blocks: int, log2_len=(18.0, 21.0), receivers: int = 8, n_tx=(0, 20),
                      snr_db=(-15.0, -5.0)):
    """A batch of blocks of uneven length from several receivers.

    Block b comes from receiver b mod receivers (a seed component: blocks are
    independent); its length is log-uniform in [2^lo, 2^hi]; it carries a
    uniform integer number of transmissions in [n_tx[0], n_tx[1]] from distinct
    tags.  Returns a list of (x complex64, list[Transmission]).
    """
    lens = batch_lengths(seed, num_blocks, *log2_len)
    g = rng(seed, _STREAM_LENGTHS, 1)
    L = np.asarray(chips).shape[1] * spc
    out = []
    for b, n in enumerate(lens):
        k = int(g.integers(n_tx[0], n_tx[1] + 1)) if n >= L + 1 else 0
        sub = (b % receivers) * 100000 + b
        out.append(make_block(seed, n, chips, spc, fs_hz, freqs_hz, k, snr_db=snr_db, sub=sub))
    return out


def make_tracking_batch(seed: int, chips: np.ndarray, spc: int, fs_hz: float, freqs_hz: Sequence[float],
                        num_tasks: int, block_factor: float = 1.5, p_present: float = 0.9, n_other=(0, 1),
                        snr_db=(-15.0, -5.0)):
    """Tracking tasks: task i looks for one tag in a block of floor(block_factor * L)
    samples.  The tag is drawn uniformly; its packet is in the block with
    probability p_present, joined by a uniform number in [n_other[0], n_other[1]]
    of other tags' packets.  Returns a list of (x complex64, tag, list[Transmission])."""
    chips = np.asarray(chips)
    T = chips.shape[0]
    L = chips.shape[1] * spc
    n = int(np.floor(block_factor * L))
    g = rng(seed, _STREAM_LENGTHS, 2)
    out = []
    for i in range(num_tasks):
        tag = int(g.integers(0, T))
        present = bool(g.random() < p_present)
        k_other = int(g.integers(n_other[0], n_other[1] + 1))
        others = [int(t) for t in g.choice([t for t in range(T) if t != tag], size=k_other, replace=False)]
        tags = ([tag] if present else []) + others
        x, txs = make_block(seed, n, chips, spc, fs_hz, freqs_hz, len(tags), snr_db=snr_db, tags=tags,
                            sub=300000 + i)
        out.append((x, tag, txs))
    return out


def fsk_bandpass(num_taps: int, cutoff_hz: float, fs_hz: float) -> np.ndarray:
    """Band-pass taps of the FSK workload, centred at 0 Hz after the mix: a
    Hann-windowed sinc low-pass of the given cutoff, unit gain at 0 Hz, complex128."""
    k = np.arange(num_taps) - (num_taps - 1) / 2.0
    h = np.sinc(2.0 * cutoff_hz / fs_hz * k) * np.hanning(num_taps + 2)[1:-1]
    return (h / h.sum()).astype(np.complex128)


def make_fsk_bits(seed: int, num_tags: int, num_bits: int) -> np.ndarray:
    """Random 0/1 codes, uint8 [num_tags][num_bits]; tag t uses stream (CODES, t, 1)."""
    out = np.empty((num_tags, num_bits), dtype=np.uint8)
    for t in range(num_tags):
        out[t] = rng(seed, _STREAM_CODES, t, 1).integers(0, 2, size=num_bits, dtype=np.uint8)
    return out


def make_fsk_block(seed: int, n: int, bits: np.ndarray, sps: int, fs_hz: float, f1_hz: float, f0_hz: float,
                   lo_hz: float, n_tx: int, snr_db=(-10.0, 0.0), noise_rms: float = 1000.0,
                   tags=None, delays=None, noise: bool = True):
    """Receiver block of int16 (I, Q) pairs [n][2]: continuous-phase FSK packets
    (bit b held sps samples at f1 or f0, random start phase) on a carrier at
    lo_hz, at integer delays, per-sample SNR drawn in dB against complex noise
    of rms noise_rms, rounded and clipped to int16.  Returns (iq, list of
    (tag, delay, snr_db))."""
    bits = np.asarray(bits)
    T, nb = bits.shape
    plen = nb * sps
    g = rng(seed, _STREAM_BLOCK, 7)
    x = np.zeros(n, dtype=np.complex128)
    txs = []
    tag_list = list(tags) if tags is not None else list(g.choice(T, size=n_tx, replace=False))
    for i in range(n_tx):
        D = int(delays[i]) if delays is not None else int(g.integers(0, max(n - plen, 1)))
        if D + plen > n:
            raise ValueError("packet does not fit in the block")
        snr = float(snr_db[0] + (snr_db[1] - snr_db[0]) * g.random())
        th0 = float(2 * np.pi * g.random())
        f = np.where(np.repeat(bits[tag_list[i]], sps) == 1, f1_hz, f0_hz) / fs_hz
        cyc = np.mod(np.concatenate(([0.0], np.cumsum(f)[:-1])), 1.0)
        A = noise_rms * 10.0 ** (snr / 20.0)
        x[D:D + plen] += A * np.exp(1j * (2 * np.pi * cyc + th0))
        txs.append((int(tag_list[i]), D, snr))
    x *= np.exp(2j * np.pi * np.mod(lo_hz / fs_hz * np.arange(n), 1.0))
    if noise:
        w = rng(seed, _STREAM_NOISE, 7).standard_normal((n, 2)) * (noise_rms / np.sqrt(2.0))
        x += w[:, 0] + 1j * w[:, 1]
    iq = np.stack([np.round(x.real), np.round(x.imag)], axis=1)
    return np.clip(iq, -32768, 32767).astype(np.int16), txs
