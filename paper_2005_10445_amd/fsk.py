"""Python face of the FSK searching pipeline (acq_fsk_* in include/acq.h).
Argument marshalling only: demodulation, replica templates, correlation and
the peak sums run in libacq.so."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List

import numpy as np

from . import _capi
from ._capi import check

__all__ = ["FskPlan", "FskDetection", "fsk_geometry"]


@dataclass
class FskDetection:
    tag: int
    lag: int
    toa: float
    xcorr: float
    q: float
    p: float
    z: float
    flags: int
    block: int = 0


def _config(bits, fs_hz, lo_hz, f1_hz, f0_hz, bp_taps, mf_len, max_block_len, fft_len=0, threshold=0.0,
            max_track_tasks=0):
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
    if b.ndim != 2:
        raise ValueError("bits must be [num_tags][num_bits]")
    taps = np.asarray(bp_taps, dtype=np.complex128).ravel()
    t = np.ascontiguousarray(np.stack([taps.real, taps.imag], axis=1).astype(np.float32))
    cfg = _capi.AcqFskConfig()
    cfg.sample_rate_hz = float(fs_hz)
    cfg.lo_hz = float(lo_hz)
    cfg.f1_hz = float(f1_hz)
    cfg.f0_hz = float(f0_hz)
    cfg.threshold = float(threshold)
    cfg.bp_taps = t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    cfg.bits = b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    cfg.max_block_len = int(max_block_len)
    cfg.bp_len = int(taps.size)
    cfg.mf_len = int(mf_len)
    cfg.num_tags, cfg.num_bits = int(b.shape[0]), int(b.shape[1])
    cfg.fft_len = int(fft_len)
    cfg.max_track_tasks = int(max_track_tasks)
    return cfg, (b, t)


def fsk_geometry(**kw) -> dict:
    """acq_fsk_plan_geometry (no GPU involved)."""
    cfg, keep = _config(**kw)
    g = _capi.AcqFskGeometry()
    check(_capi.lib().acq_fsk_plan_geometry(ctypes.byref(cfg), ctypes.byref(g)), "acq_fsk_plan_geometry")
    return {name: getattr(g, name) for name, _ in _capi.AcqFskGeometry._fields_}


def _iq_ptr(iq):
    import torch
    if not isinstance(iq, torch.Tensor) or not iq.is_cuda or iq.dtype != torch.int16 or not iq.is_contiguous():
        raise TypeError("iq must be a contiguous int16 CUDA (HIP) tensor of shape [n, 2]")
    if iq.dim() != 2 or iq.shape[1] != 2:
        raise TypeError("iq must have shape [n, 2]")
    return iq.data_ptr(), iq.shape[0]


class FskPlan:
    """An FSK searching plan bound to one HIP stream (default: torch's current stream)."""

    def __init__(self, bits, fs_hz: float, lo_hz: float, f1_hz: float, f0_hz: float, bp_taps, mf_len: int,
                 max_block_len: int, fft_len: int = 0, threshold: float = 0.0, max_track_tasks: int = 0,
                 stream=None):
        import torch
        self._lib = _capi.lib()
        cfg, keep = _config(bits, fs_hz, lo_hz, f1_hz, f0_hz, bp_taps, mf_len, max_block_len, fft_len, threshold,
                            max_track_tasks)
        self.max_track_tasks = int(max_track_tasks) if max_track_tasks > 0 else 16
        g = _capi.AcqFskGeometry()
        check(self._lib.acq_fsk_plan_geometry(ctypes.byref(cfg), ctypes.byref(g)), "acq_fsk_plan_geometry")
        self.geometry = {name: getattr(g, name) for name, _ in _capi.AcqFskGeometry._fields_}
        self.num_tags = int(cfg.num_tags)
        self.template_len = int(g.template_len)
        if stream is None:
            stream = torch.cuda.current_stream()
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._h = ctypes.c_void_p()
        check(self._lib.acq_fsk_plan(ctypes.byref(cfg), ctypes.c_void_p(handle), ctypes.byref(self._h)),
              "acq_fsk_plan")
        self._out = (_capi.AcqFskDetection * self.num_tags)()

    def demod(self, iq):
        """(d, u) device float32 tensors of steps 1-5."""
        import torch
        ptr, n = _iq_ptr(iq)
        d = torch.empty(n, dtype=torch.float32, device=iq.device)
        u = torch.empty(n, dtype=torch.float32, device=iq.device)
        check(self._lib.acq_fsk_demod(self._h, ctypes.c_void_p(ptr), n, ctypes.c_void_p(d.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr())), "acq_fsk_demod")
        return d, u

    def template(self, tag: int):
        import torch
        out = torch.empty(self.template_len, dtype=torch.float32, device="cuda")
        check(self._lib.acq_fsk_template(self._h, int(tag), ctypes.c_void_p(out.data_ptr())), "acq_fsk_template")
        return out

    def xcorr(self, iq):
        """FFT-path correlation of every tag at every lag: device float32 [T][n - n_t + 1]."""
        import torch
        ptr, n = _iq_ptr(iq)
        out = torch.empty((self.num_tags, max(n - self.template_len + 1, 1)), dtype=torch.float32, device=iq.device)
        check(self._lib.acq_fsk_xcorr(self._h, ctypes.c_void_p(ptr), n, ctypes.c_void_p(out.data_ptr())),
              "acq_fsk_xcorr")
        return out

    def detect(self, iq) -> List[FskDetection]:
        ptr, n = _iq_ptr(iq)
        nf = ctypes.c_int32(0)
        check(self._lib.acq_fsk_detect(self._h, ctypes.c_void_p(ptr), n, self._out, self.num_tags,
                                       ctypes.byref(nf)), "acq_fsk_detect")
        return [FskDetection(d.tag, d.lag, d.toa_samples, d.xcorr, d.q, d.p, d.z, d.flags, d.block)
                for d in self._out[:nf.value]]

    @staticmethod
    def task_array(tasks):
        """acq_fsk_task array of (int16 [n, 2] device tensor, tag) pairs (the tensors must stay alive)."""
        arr = (_capi.AcqFskTask * len(tasks))()
        for i, (iq, tag) in enumerate(tasks):
            ptr, n = _iq_ptr(iq)
            arr[i] = _capi.AcqFskTask(ptr, n, int(tag), 0)
        return arr

    def track_raw(self, arr) -> int:
        """acq_fsk_track on a prebuilt task_array, without building Python records (for
        timing); returns the count."""
        n = len(arr)
        if getattr(self, "_track_out", None) is None or len(self._track_out) < n:
            self._track_out = (_capi.AcqFskDetection * n)()
        nf = ctypes.c_int32(0)
        check(self._lib.acq_fsk_track(self._h, arr, n, self._track_out, n, ctypes.byref(nf)), "acq_fsk_track")
        return nf.value

    def track(self, tasks) -> List[FskDetection]:
        """acq_fsk_track over (int16 [n, 2] device tensor, tag) pairs; detection.block = task index."""
        arr = self.task_array(tasks)
        out = (_capi.AcqFskDetection * len(tasks))()
        nf = ctypes.c_int32(0)
        check(self._lib.acq_fsk_track(self._h, arr, len(tasks), out, len(tasks), ctypes.byref(nf)), "acq_fsk_track")
        return [FskDetection(d.tag, d.lag, d.toa_samples, d.xcorr, d.q, d.p, d.z, d.flags, d.block)
                for d in out[:nf.value]]

    def detect_raw(self, iq) -> int:
        ptr, n = _iq_ptr(iq)
        nf = ctypes.c_int32(0)
        check(self._lib.acq_fsk_detect(self._h, ctypes.c_void_p(ptr), n, self._out, self.num_tags,
                                       ctypes.byref(nf)), "acq_fsk_detect")
        return nf.value

    def set_profiling(self, on: bool):
        check(self._lib.acq_fsk_set_profiling(self._h, 1 if on else 0), "acq_fsk_set_profiling")

    def last_kernel_times(self) -> dict:
        ms = (ctypes.c_double * 4)()
        check(self._lib.acq_fsk_last_kernel_times(self._h, ms, 4), "acq_fsk_last_kernel_times")
        return dict(zip(("front", "forward", "correlate", "refine"), list(ms)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.acq_fsk_release(self._h)
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
