"""Acquisition-mode correlation search on AMD Instinct MI355X.

Python face of libacq.so (include/acq.h).  It marshals arguments only: the
block power, segment spectra, replica bank, correlation, peak search and FP64
refinement all run in the library's HIP kernels.  PyTorch provides device
memory and the stream.  There is no CPU fallback: constructing a Plan without
the built library raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import _capi
from ._capi import AcqConfig, AcqDetection, AcqGeometry, AcqError, check

__all__ = ["Plan", "Detection", "geometry", "workspace_size", "bin_frequencies", "tune_fft_len", "AcqError",
           "make_config"]

_PRECISION = {"fp32": _capi.ACQ_FP32, "fp16": _capi.ACQ_FP16, "bf16": _capi.ACQ_BF16}


@dataclass
class Detection:
    tag: int
    bin: int
    lag: int
    toa: float
    freq_hz: float
    peak_power: float
    z: float
    energy: float
    block_power: float
    block: int
    flags: int
    power: float = 0.0          # relative power A^2 = P / L^2
    snr: float = 0.0            # A^2 / sigma^2, sigma^2 = (E - P/L) / L
    crossings: int = 0          # (bin, lag) hypotheses of the tag with z >= threshold


def _det(d) -> Detection:
    return Detection(d.tag, d.bin, d.lag, d.toa_samples, d.freq_hz, d.peak_power, d.z, d.energy, d.block_power,
                     d.block, d.flags, d.power, d.snr, d.crossings)


def make_config(chips: np.ndarray, spc: int, fs_hz: float, num_bins: int = 1,
                bin_center_hz: float = 0.0, bin_step_hz: float = 0.0, max_block_len: int = 1 << 20,
                fft_len: int = 0, threshold: float = 0.0, precision: str = "fp32",
                refine_radius: int = 1, tag_tile: int = 0, max_batch_blocks: int = 0,
                max_batch_samples: int = 0, graph: bool = False, exact_bins: bool = False,
                asynchronous: bool = False, check_finite: bool = False):
    """Build an AcqConfig; returns (config, chips array that must outlive the call)."""
    ch = np.ascontiguousarray(np.asarray(chips, dtype=np.int8))
    if ch.ndim != 2:
        raise ValueError("chips must be [num_tags][num_chips]")
    cfg = AcqConfig()
    cfg.sample_rate_hz = float(fs_hz)
    cfg.bin_center_hz = float(bin_center_hz)
    cfg.bin_step_hz = float(bin_step_hz)
    cfg.threshold = float(threshold)
    cfg.chips = ch.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    cfg.max_block_len = int(max_block_len)
    cfg.num_tags, cfg.num_chips = int(ch.shape[0]), int(ch.shape[1])
    cfg.samples_per_chip = int(spc)
    cfg.num_bins = int(num_bins)
    cfg.fft_len = int(fft_len)
    cfg.precision = _PRECISION[precision]
    cfg.refine_radius = int(refine_radius)
    cfg.tag_tile = int(tag_tile)
    cfg.flags = ((_capi.ACQ_FLAG_GRAPH if graph else 0) | (_capi.ACQ_FLAG_EXACT_BINS if exact_bins else 0) |
                 (_capi.ACQ_FLAG_ASYNC if asynchronous else 0) | (_capi.ACQ_FLAG_CHECK_FINITE if check_finite else 0))
    cfg.max_batch_blocks = int(max_batch_blocks)
    cfg.max_batch_samples = int(max_batch_samples)
    return cfg, ch


def workspace_size(**kw) -> int:
    """acq_workspace_size for a configuration (no GPU involved)."""
    cfg, _keep = make_config(**kw)
    n = ctypes.c_size_t(0)
    check(_capi.lib().acq_workspace_size(ctypes.byref(cfg), ctypes.byref(n)), "acq_workspace_size")
    return int(n.value)


def geometry(**kw) -> dict:
    """acq_plan_geometry for a configuration (no GPU involved)."""
    cfg, _keep = make_config(**kw)
    g = AcqGeometry()
    check(_capi.lib().acq_plan_geometry(ctypes.byref(cfg), ctypes.byref(g)), "acq_plan_geometry")
    return {name: getattr(g, name) for name, _ in AcqGeometry._fields_}


def bin_frequencies(**kw) -> np.ndarray:
    cfg, _keep = make_config(**kw)
    out = np.zeros(cfg.num_bins, dtype=np.float64)
    check(_capi.lib().acq_bin_frequencies(ctypes.byref(cfg),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          cfg.num_bins), "acq_bin_frequencies")
    return out


def tune_fft_len(block, reps: int = 2, stream=None, **kw):
    """acq_tune_fft_len: time every segment length the library can run for this
    configuration (make_config's keywords) on a device block; returns (best M,
    table of {fft_len, engine, tag_tile, batch_launch, ms})."""
    import torch
    cfg, _keep = make_config(**kw)
    ptr, n = _device_ptr(block)
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    out = (_capi.AcqTuneEntry * 8)()
    cnt, best = ctypes.c_int32(0), ctypes.c_int32(0)
    check(_capi.lib().acq_tune_fft_len(ctypes.byref(cfg), ctypes.c_void_p(ptr), n, int(reps), ctypes.c_void_p(handle),
                                       out, 8, ctypes.byref(cnt), ctypes.byref(best)), "acq_tune_fft_len")
    return best.value, [{"fft_len": e.fft_len, "engine": e.tuning.engine, "tag_tile": e.tuning.tag_tile,
                         "batch_launch": e.tuning.batch_launch, "ms": e.ms} for e in out[:cnt.value]]


def _device_ptr(block):
    import torch
    if not isinstance(block, torch.Tensor) or not block.is_cuda:
        raise TypeError("block must be a CUDA (HIP) torch tensor")
    if block.dtype != torch.complex64 or not block.is_contiguous() or block.dim() != 1:
        raise TypeError("block must be a contiguous 1-D complex64 tensor")
    return block.data_ptr(), block.numel()


class Plan:
    """An acquisition plan bound to one HIP stream (default: torch's current stream).

    workspace: optional uint8 CUDA tensor of at least workspace_size(...) bytes that the
    plan uses for every per-search buffer (kept referenced by the plan); None lets the
    library allocate it.  asynchronous: searches only enqueue (results via collect() or
    device_results()).  check_finite: blocks with NaN/inf samples raise AcqError."""

    def __init__(self, chips, spc: int, fs_hz: float, *, num_bins: int = 1, bin_center_hz: float = 0.0,
                 bin_step_hz: float = 0.0, max_block_len: int = 1 << 20, fft_len: int = 0,
                 threshold: float = 0.0, precision: str = "fp32", refine_radius: int = 1,
                 tag_tile: int = 0, max_batch_blocks: int = 0, max_batch_samples: int = 0,
                 graph: bool = False, exact_bins: bool = False, stream=None, workspace=None,
                 asynchronous: bool = False, check_finite: bool = False):
        import torch
        self._lib = _capi.lib()
        cfg, ch = make_config(chips, spc, fs_hz, num_bins, bin_center_hz, bin_step_hz, max_block_len,
                              fft_len, threshold, precision, refine_radius, tag_tile, max_batch_blocks,
                              max_batch_samples, graph, exact_bins, asynchronous, check_finite)
        self.asynchronous = bool(asynchronous)
        self.max_batch_blocks = max(int(max_batch_blocks), 1)
        self.num_tags, self.num_chips = ch.shape
        self.precision = precision
        self.spc = int(spc)
        self.num_bins = int(num_bins)
        self.template_len = self.num_chips * self.spc
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        g = AcqGeometry()
        check(self._lib.acq_plan_geometry(ctypes.byref(cfg), ctypes.byref(g)), "acq_plan_geometry")
        self.geometry = {name: getattr(g, name) for name, _ in AcqGeometry._fields_}
        self.freqs_hz = np.zeros(self.num_bins)
        check(self._lib.acq_bin_frequencies(ctypes.byref(cfg),
                                            self.freqs_hz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            self.num_bins), "acq_bin_frequencies")
        self._h = ctypes.c_void_p()
        self._workspace = workspace                 # the caller's memory must outlive the plan
        if workspace is not None:
            if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or not workspace.is_contiguous():
                raise TypeError("workspace must be a contiguous CUDA tensor")
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        else:
            ws_ptr, ws_bytes = None, 0
        check(self._lib.acq_plan(ctypes.byref(cfg), ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes),
                                 ctypes.c_void_p(handle), ctypes.byref(self._h)), "acq_plan")
        self._out = (AcqDetection * self.num_tags)()

    def detect(self, block) -> List[Detection]:
        ptr, n = _device_ptr(block)
        nf = ctypes.c_int32(0)
        check(self._lib.acq_detect(self._h, ctypes.c_void_p(ptr), n, self._out, self.num_tags,
                                   ctypes.byref(nf)), "acq_detect")
        if self.asynchronous:
            return self.collect()
        return [_det(d) for d in self._out[:nf.value]]

    def enqueue(self, block):
        """acq_detect on an asynchronous plan: enqueue the search and return at once
        (capturable into a hipGraph on the plan's stream)."""
        if not self.asynchronous:
            raise RuntimeError("enqueue needs a plan made with asynchronous=True")
        ptr, n = _device_ptr(block)
        check(self._lib.acq_detect(self._h, ctypes.c_void_p(ptr), n, None, 0, None), "acq_detect")

    def collect(self, capacity: Optional[int] = None) -> List[Detection]:
        """acq_collect: wait for the plan's stream and return the last search's detections."""
        cap = capacity if capacity is not None else self.max_batch_blocks * self.num_tags
        out = (AcqDetection * max(cap, 1))()
        nf = ctypes.c_int32(0)
        check(self._lib.acq_collect(self._h, out, cap, ctypes.byref(nf)), "acq_collect")
        return [_det(d) for d in out[:min(nf.value, cap)]]

    def device_results(self):
        """acq_device_results: (device address of the records, device address of the int32[2] counts)."""
        rec, cnt = ctypes.c_void_p(), ctypes.c_void_p()
        check(self._lib.acq_device_results(self._h, ctypes.byref(rec), ctypes.byref(cnt)), "acq_device_results")
        return rec.value, cnt.value

    def detect_batch(self, blocks) -> List[Detection]:
        """acq_detect_batch over a list of 1-D complex64 device tensors of any lengths."""
        n = len(blocks)
        ptrs = (ctypes.c_void_p * n)()
        lens = (ctypes.c_int64 * n)()
        for i, b in enumerate(blocks):
            ptr, m = _device_ptr(b)
            ptrs[i], lens[i] = ptr, m
        cap = n * self.num_tags
        out = (AcqDetection * cap)()
        nf = ctypes.c_int32(0)
        check(self._lib.acq_detect_batch(self._h, ptrs, lens, n, out, cap, ctypes.byref(nf), None),
              "acq_detect_batch")
        if self.asynchronous:
            return self.collect(cap)
        return [_det(d) for d in out[:nf.value]]

    def track(self, tasks) -> List[Detection]:
        """acq_track_batch over (1-D complex64 device tensor, tag) pairs: at most one
        detection per task, detection.block = task index."""
        arr = self.task_array(tasks)
        n = len(arr)
        out = (AcqDetection * n)()
        nf = ctypes.c_int32(0)
        check(self._lib.acq_track_batch(self._h, arr, n, out, n, ctypes.byref(nf)), "acq_track_batch")
        if self.asynchronous:
            return self.collect(n)
        return [_det(d) for d in out[:nf.value]]

    @staticmethod
    def task_array(tasks):
        """acq_track_task array of (device tensor, tag) pairs (the tensors must stay alive)."""
        arr = (_capi.AcqTrackTask * len(tasks))()
        for i, (b, tag) in enumerate(tasks):
            ptr, m = _device_ptr(b)
            arr[i] = _capi.AcqTrackTask(ptr, m, int(tag), 0)
        return arr

    def track_raw(self, arr) -> int:
        """acq_track_batch on a prebuilt task_array, without building Python records (for
        timing); returns the count."""
        n = len(arr)
        if getattr(self, "_track_out", None) is None or len(self._track_out) < n:
            self._track_out = (AcqDetection * n)()
        nf = ctypes.c_int32(0)
        check(self._lib.acq_track_batch(self._h, arr, n, self._track_out, n, ctypes.byref(nf)), "acq_track_batch")
        return nf.value

    @property
    def tuning(self) -> dict:
        t = _capi.AcqTuning()
        check(self._lib.acq_get_tuning(self._h, ctypes.byref(t)), "acq_get_tuning")
        return {"engine": t.engine, "tag_tile": t.tag_tile, "batch_launch": t.batch_launch,
                "track_bins": t.track_bins}

    def set_tuning(self, engine: int, tag_tile: int, batch_launch: Optional[int] = None,
                   track_bins: Optional[int] = None):
        """batch_launch: 0 grid over work items (default), 1 persistent workgroups; track_bins:
        bins per tracking work item (0: chosen per launch); None keeps the current value."""
        cur = self.tuning
        if batch_launch is None:
            batch_launch = cur["batch_launch"]
        if track_bins is None:
            track_bins = cur["track_bins"]
        t = _capi.AcqTuning(int(engine), int(tag_tile), int(batch_launch), int(track_bins))
        check(self._lib.acq_set_tuning(self._h, ctypes.byref(t)), "acq_set_tuning")

    def tune(self, block, reps: int = 3) -> list:
        """acq_tune: time every candidate tuning on `block`, keep the fastest; returns the table."""
        ptr, n = _device_ptr(block)
        out = (_capi.AcqTuneEntry * 32)()
        cnt = ctypes.c_int32(0)
        check(self._lib.acq_tune(self._h, ctypes.c_void_p(ptr), n, int(reps), out, 32, ctypes.byref(cnt)),
              "acq_tune")
        return [{"engine": e.tuning.engine, "tag_tile": e.tuning.tag_tile, "batch_launch": e.tuning.batch_launch,
                 "fft_len": e.fft_len, "ms": e.ms} for e in out[:cnt.value]]

    def detect_raw(self, block) -> int:
        """acq_detect without building Python records (for timing); returns the count."""
        ptr, n = _device_ptr(block)
        nf = ctypes.c_int32(0)
        check(self._lib.acq_detect(self._h, ctypes.c_void_p(ptr), n, self._out, self.num_tags,
                                   ctypes.byref(nf)), "acq_detect")
        return nf.value

    def correlate_power(self, block, out=None):
        """FFT-path power P[t][k][tau] (FP32, device tensor [T][K][n-L+1])."""
        import torch
        ptr, n = _device_ptr(block)
        lags = max(n - self.template_len + 1, 0)
        if out is None:
            out = torch.empty((self.num_tags, self.num_bins, lags), dtype=torch.float32, device=block.device)
        if lags > 0:
            check(self._lib.acq_correlate_power(self._h, ctypes.c_void_p(ptr), n,
                                                ctypes.c_void_p(out.data_ptr())), "acq_correlate_power")
        return out

    def set_profiling(self, on: bool = True, correlate_only: bool = False):
        """Time the kernels of each call with HIP events on the plan's stream (every
        kernel, or with correlate_only the correlation kernel alone)."""
        mode = (_capi.PROFILE_CORRELATE if correlate_only else _capi.PROFILE_ALL) if on else _capi.PROFILE_OFF
        check(self._lib.acq_set_profiling(self._h, mode), "acq_set_profiling")

    def last_kernel_times(self) -> dict:
        """Durations (ms) of the kernels of the last call, from HIP events on the plan's stream."""
        ms = (ctypes.c_double * len(_capi.KERNELS))()
        cnt = ctypes.c_int32(0)
        check(self._lib.acq_last_kernel_times(self._h, ms, len(_capi.KERNELS), ctypes.byref(cnt)),
              "acq_last_kernel_times")
        return dict(zip(_capi.KERNELS, list(ms)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.acq_release(self._h)
            self._h = ctypes.c_void_p()
            self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
