"""Python face of the proposal stage (acq_cnn_* and acq_detect_learned in
include/acq.h).  Argument marshalling only: power maps, the network, its
training and the proposal search run in libacq.so."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _capi
from ._capi import check

__all__ = ["Network", "SynthTransmission", "LearnedParams", "LearnedReport", "num_frames", "num_params"]

_PRECISION = {"fp32": _capi.ACQ_FP32, "bf16": _capi.ACQ_BF16}


def num_frames(n: int) -> int:
    return 0 if n < 256 else (n - 256) // 128 + 1


def num_params(in_channels: int = 256) -> int:
    return int(_capi.lib().acq_cnn_num_params(int(in_channels)))


@dataclass
class SynthTransmission:
    delay: int
    freq_over_fs: float
    amp: float
    phase0: float
    code: int


@dataclass
class LearnedParams:
    kappa: float
    max_fraction: float = 0.5
    floor_db: float = 1.0


@dataclass
class LearnedReport:
    proposals: int
    segments: int
    total_segments: int
    fallback: int
    median: float
    floor: float


def _dev(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous CUDA (HIP) tensor")
    return t.data_ptr()


class Network:
    """The proposal CNN on the device (precision "bf16" or "fp32")."""

    def __init__(self, precision: str = "bf16", in_channels: int = 256, max_rows: int = 1 << 16,
                 max_block_len: int = 1 << 21, stream=None):
        import torch
        self._lib = _capi.lib()
        cfg = _capi.AcqCnnConfig(_PRECISION[precision], int(in_channels), int(max_rows), int(max_block_len))
        if stream is None:
            stream = torch.cuda.current_stream()
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self.precision, self.in_channels, self.max_rows = precision, int(in_channels), int(max_rows)
        self.dtype = torch.bfloat16 if precision == "bf16" else torch.float32
        self._h = ctypes.c_void_p()
        check(self._lib.acq_cnn_create(ctypes.byref(cfg), ctypes.c_void_p(handle), ctypes.byref(self._h)),
              "acq_cnn_create")
        self.num_params = int(self._lib.acq_cnn_num_params(self.in_channels))

    # -------------------------------------------------------------- parameters
    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        check(self._lib.acq_cnn_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size),
              "acq_cnn_set_params")

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.num_params, dtype=np.float32)
        check(self._lib.acq_cnn_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size),
              "acq_cnn_get_params")
        return p

    # -------------------------------------------------------------- compute
    def forward(self, inp, nblocks: int = 1):
        """Logits (device FP32 [rows]) of input [nblocks*frames][in_channels]."""
        import torch
        rows = inp.shape[0]
        out = torch.empty(rows, dtype=torch.float32, device=inp.device)
        check(self._lib.acq_cnn_forward(self._h, ctypes.c_void_p(_dev(inp, "input")), int(nblocks),
                                        rows // int(nblocks), ctypes.c_void_p(out.data_ptr())), "acq_cnn_forward")
        return out

    def gradients(self, inp, labels, pos_weight: float, nblocks: int = 1):
        """(mean loss, device FP32 gradient [num_params])."""
        import torch
        rows = inp.shape[0]
        grad = torch.empty(self.num_params, dtype=torch.float32, device=inp.device)
        loss = ctypes.c_float(0.0)
        check(self._lib.acq_cnn_gradients(self._h, ctypes.c_void_p(_dev(inp, "input")), int(nblocks),
                                          rows // int(nblocks), ctypes.c_void_p(_dev(labels, "labels")),
                                          float(pos_weight), ctypes.c_void_p(grad.data_ptr()),
                                          ctypes.byref(loss)), "acq_cnn_gradients")
        return loss.value, grad

    def adam_step(self, lr: float):
        check(self._lib.acq_cnn_adam_step(self._h, float(lr)), "acq_cnn_adam_step")

    def power_map(self, block):
        """(map device [F][256], median) of a 1-D complex64 device block."""
        import torch
        n = block.numel()
        F = num_frames(n)
        out = torch.empty((F, 256), dtype=self.dtype, device=block.device)
        med = ctypes.c_float(0.0)
        check(self._lib.acq_power_map(self._h, ctypes.c_void_p(_dev(block, "block")), n,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.byref(med)), "acq_power_map")
        return out, med.value

    @staticmethod
    def _batch(seed: int, first_block: int, block_len: int, num_chips: int, spc: int,
               txs: Sequence[Sequence[SynthTransmission]]):
        nb = len(txs)
        tx = (_capi.AcqSynthTx * (nb * _capi.ACQ_SYNTH_MAX_TX))()
        ntx = (ctypes.c_int32 * nb)()
        for b, lst in enumerate(txs):
            if len(lst) > _capi.ACQ_SYNTH_MAX_TX:
                raise ValueError("too many transmissions in a block")
            ntx[b] = len(lst)
            for i, t in enumerate(lst):
                tx[b * _capi.ACQ_SYNTH_MAX_TX + i] = _capi.AcqSynthTx(int(t.delay), float(t.freq_over_fs),
                                                                     float(t.amp), float(t.phase0),
                                                                     int(t.code) & 0xffffffff, 0)
        batch = _capi.AcqSynthBatch(int(seed) & (2 ** 64 - 1), int(first_block), nb, int(num_chips), int(spc),
                                    int(block_len), ctypes.cast(tx, ctypes.POINTER(_capi.AcqSynthTx)),
                                    ctypes.cast(ntx, ctypes.POINTER(ctypes.c_int32)))
        return batch, (tx, ntx)

    def synth_block(self, seed: int, block: int, block_len: int, num_chips: int, spc: int,
                    txs: Sequence[SynthTransmission]):
        """Samples (device complex64) of one generated block."""
        import torch
        batch, keep = self._batch(seed, block, block_len, num_chips, spc, [txs])
        out = torch.empty(int(block_len), dtype=torch.complex64, device="cuda")
        check(self._lib.acq_synth_block(self._h, ctypes.byref(batch), ctypes.c_void_p(out.data_ptr())),
              "acq_synth_block")
        return out

    def synth_labels(self, seed: int, first_block: int, block_len: int, num_chips: int, spc: int,
                     txs: Sequence[Sequence[SynthTransmission]]):
        """Training labels (device FP32 [len(txs) * frames]) of a generated batch."""
        import torch
        batch, keep = self._batch(seed, first_block, block_len, num_chips, spc, txs)
        out = torch.empty(len(txs) * num_frames(int(block_len)), dtype=torch.float32, device="cuda")
        check(self._lib.acq_synth_labels(self._h, ctypes.byref(batch), ctypes.c_void_p(out.data_ptr())),
              "acq_synth_labels")
        return out

    def train_synthetic(self, seed: int, first_block: int, block_len: int, num_chips: int, spc: int,
                        txs: Sequence[Sequence[SynthTransmission]], pos_weight: float, lr: float) -> float:
        """One generated batch (len(txs) blocks): map, labels, forward, backward, Adam.  Mean loss."""
        batch, keep = self._batch(seed, first_block, block_len, num_chips, spc, txs)
        loss = ctypes.c_float(0.0)
        check(self._lib.acq_cnn_train_synthetic(self._h, ctypes.byref(batch), float(pos_weight), float(lr),
                                                ctypes.byref(loss)), "acq_cnn_train_synthetic")
        return loss.value

    def detect(self, plan, block, params: LearnedParams):
        """acq_detect_learned: (detections, LearnedReport)."""
        from . import _det
        n = block.numel()
        out = (_capi.AcqDetection * plan.num_tags)()
        nf = ctypes.c_int32(0)
        rep = _capi.AcqLearnedReport()
        lp = _capi.AcqLearnedParams(float(params.kappa), float(params.max_fraction), float(params.floor_db))
        check(self._lib.acq_detect_learned(plan._h, self._h, ctypes.c_void_p(_dev(block, "block")), n,
                                           ctypes.byref(lp), out, plan.num_tags, ctypes.byref(nf),
                                           ctypes.byref(rep)), "acq_detect_learned")
        dets = [_det(d) for d in out[:nf.value]]
        return dets, LearnedReport(rep.proposals, rep.segments, rep.total_segments, rep.fallback, rep.median,
                                   rep.floor)

    def detect_batch(self, plan, blocks, params: LearnedParams):
        """acq_detect_batch_learned over a list of device blocks: (detections, [LearnedReport])."""
        from . import _det
        n = len(blocks)
        ptrs = (ctypes.c_void_p * n)()
        lens = (ctypes.c_int64 * n)()
        for i, b in enumerate(blocks):
            ptrs[i], lens[i] = _dev(b, "block"), b.numel()
        cap = n * plan.num_tags
        out = (_capi.AcqDetection * cap)()
        reps = (_capi.AcqLearnedReport * n)()
        nf = ctypes.c_int32(0)
        lp = _capi.AcqLearnedParams(float(params.kappa), float(params.max_fraction), float(params.floor_db))
        check(self._lib.acq_detect_batch_learned(plan._h, self._h, ptrs, lens, n, ctypes.byref(lp), out, cap,
                                                 ctypes.byref(nf), reps), "acq_detect_batch_learned")
        dets = [_det(d) for d in out[:nf.value]]
        return dets, [LearnedReport(r.proposals, r.segments, r.total_segments, r.fallback, r.median, r.floor)
                      for r in reps]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.acq_cnn_release(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
