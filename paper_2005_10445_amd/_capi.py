"""ctypes mirror of include/acq.h.

Argument marshalling only: every computation happens in libacq.so.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# ACQ_LIBRARY selects another build of the same library (e.g. to compare variants)
LIB_PATH = os.environ.get("ACQ_LIBRARY") or os.path.join(_PKG, "libacq.so")

ACQ_OK = 0
ACQ_ERR_INVALID_ARG = -1
ACQ_ERR_OOM = -2
ACQ_ERR_DEVICE = -3
ACQ_ERR_TRUNCATED = -4
ACQ_ERR_BLOCK_TOO_LONG = -5
ACQ_ERR_WORKSPACE_TOO_SMALL = -6
ACQ_ERR_UNSUPPORTED = -7
ACQ_ERR_NON_FINITE = -8

ACQ_FP32, ACQ_FP16, ACQ_BF16 = 0, 1, 2
ACQ_DET_NEAR_EDGE = 0x1
ACQ_DET_WINDOW_EDGE = 0x2
ACQ_FLAG_GRAPH = 0x1
ACQ_FLAG_EXACT_BINS = 0x2
ACQ_FLAG_ASYNC = 0x4
ACQ_FLAG_CHECK_FINITE = 0x8

# every symbol include/acq.h declares
EXPORTED = ("acq_plan_geometry", "acq_workspace_size", "acq_bin_frequencies", "acq_plan", "acq_detect",
            "acq_detect_batch", "acq_track_batch", "acq_collect", "acq_device_results", "acq_detect_noalloc",
            "acq_get_tuning", "acq_set_tuning", "acq_tune", "acq_tune_fft_len", "acq_correlate_power",
            "acq_set_profiling",
            "acq_last_kernel_times", "acq_release", "acq_cnn_num_params", "acq_cnn_create", "acq_cnn_release",
            "acq_cnn_set_params", "acq_cnn_get_params", "acq_cnn_forward", "acq_cnn_gradients",
            "acq_cnn_adam_step", "acq_power_map", "acq_synth_block", "acq_synth_labels", "acq_cnn_train_synthetic",
            "acq_detect_learned", "acq_detect_batch_learned", "acq_fsk_plan_geometry", "acq_fsk_plan",
            "acq_fsk_release", "acq_fsk_demod", "acq_fsk_template", "acq_fsk_xcorr", "acq_fsk_detect",
            "acq_fsk_track", "acq_fsk_set_profiling", "acq_fsk_last_kernel_times", "acq_strerror",
            "acq_last_error")
ACQ_SYNTH_MAX_TX = 32
ACQ_FALLBACK_NONE, ACQ_FALLBACK_FRACTION, ACQ_FALLBACK_FLOOR = 0, 1, 2
KERNELS = ("block_power", "forward", "correlate", "refine", "compact")
PROFILE_OFF, PROFILE_ALL, PROFILE_CORRELATE = 0, 1, 2


class AcqConfig(ctypes.Structure):
    _fields_ = [
        ("sample_rate_hz", ctypes.c_double),
        ("bin_center_hz", ctypes.c_double),
        ("bin_step_hz", ctypes.c_double),
        ("threshold", ctypes.c_double),
        ("chips", ctypes.POINTER(ctypes.c_int8)),
        ("max_block_len", ctypes.c_int64),
        ("num_tags", ctypes.c_int32),
        ("num_chips", ctypes.c_int32),
        ("samples_per_chip", ctypes.c_int32),
        ("num_bins", ctypes.c_int32),
        ("fft_len", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("refine_radius", ctypes.c_int32),
        ("tag_tile", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("max_batch_blocks", ctypes.c_int32),
        ("max_batch_samples", ctypes.c_int64),
    ]


class AcqGeometry(ctypes.Structure):
    _fields_ = [
        ("template_len", ctypes.c_int64),
        ("min_fft_len", ctypes.c_int64),
        ("fft_len", ctypes.c_int64),
        ("sub_fft_len", ctypes.c_int64),
        ("valid_per_segment", ctypes.c_int64),
        ("max_segments", ctypes.c_int64),
        ("freq_quantum_hz", ctypes.c_double),
        ("bin_center_hz", ctypes.c_double),
        ("bin_step_hz", ctypes.c_double),
        ("device_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
    ]


class AcqDetection(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int32),
        ("bin", ctypes.c_int32),
        ("lag", ctypes.c_int64),
        ("toa_samples", ctypes.c_double),
        ("freq_hz", ctypes.c_double),
        ("peak_power", ctypes.c_double),
        ("z", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("block_power", ctypes.c_double),
        ("power", ctypes.c_double),
        ("snr", ctypes.c_double),
        ("block", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("crossings", ctypes.c_int64),
    ]


class AcqTuning(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("tag_tile", ctypes.c_int32), ("batch_launch", ctypes.c_int32),
                ("track_bins", ctypes.c_int32)]


ACQ_BATCH_GRID, ACQ_BATCH_PERSISTENT = 0, 1


class AcqTuneEntry(ctypes.Structure):
    _fields_ = [("tuning", AcqTuning), ("fft_len", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class AcqCnnConfig(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("in_channels", ctypes.c_int32),
        ("max_rows", ctypes.c_int64),
        ("max_block_len", ctypes.c_int64),
    ]


class AcqFskConfig(ctypes.Structure):
    _fields_ = [("sample_rate_hz", ctypes.c_double), ("lo_hz", ctypes.c_double), ("f1_hz", ctypes.c_double),
                ("f0_hz", ctypes.c_double), ("threshold", ctypes.c_double),
                ("bp_taps", ctypes.POINTER(ctypes.c_float)), ("bits", ctypes.POINTER(ctypes.c_uint8)),
                ("max_block_len", ctypes.c_int64), ("bp_len", ctypes.c_int32), ("mf_len", ctypes.c_int32),
                ("num_tags", ctypes.c_int32), ("num_bits", ctypes.c_int32), ("fft_len", ctypes.c_int32),
                ("max_track_tasks", ctypes.c_int32)]


class AcqFskDetection(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int32), ("flags", ctypes.c_uint32), ("lag", ctypes.c_int64),
                ("toa_samples", ctypes.c_double), ("xcorr", ctypes.c_double), ("q", ctypes.c_double),
                ("p", ctypes.c_double), ("z", ctypes.c_double), ("block", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class AcqFskTask(ctypes.Structure):
    _fields_ = [("iq", ctypes.c_void_p), ("n", ctypes.c_int64), ("tag", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class AcqFskGeometry(ctypes.Structure):
    _fields_ = [("template_len", ctypes.c_int64), ("fft_len", ctypes.c_int64), ("valid_per_segment", ctypes.c_int64),
                ("filter_len", ctypes.c_int64), ("front_fft_len", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class AcqTrackTask(ctypes.Structure):
    _fields_ = [("block", ctypes.c_void_p), ("n", ctypes.c_int64), ("tag", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class AcqSynthTx(ctypes.Structure):
    _fields_ = [
        ("delay", ctypes.c_int64),
        ("freq_over_fs", ctypes.c_double),
        ("amp", ctypes.c_float),
        ("phase0", ctypes.c_float),
        ("code", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class AcqSynthBatch(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("first_block", ctypes.c_int64),
        ("nblocks", ctypes.c_int32),
        ("num_chips", ctypes.c_int32),
        ("samples_per_chip", ctypes.c_int32),
        ("block_len", ctypes.c_int64),
        ("tx", ctypes.POINTER(AcqSynthTx)),
        ("ntx", ctypes.POINTER(ctypes.c_int32)),
    ]


class AcqLearnedParams(ctypes.Structure):
    _fields_ = [
        ("kappa", ctypes.c_float),
        ("max_fraction", ctypes.c_float),
        ("floor_db", ctypes.c_float),
    ]


class AcqLearnedReport(ctypes.Structure):
    _fields_ = [
        ("proposals", ctypes.c_int32),
        ("segments", ctypes.c_int32),
        ("total_segments", ctypes.c_int32),
        ("fallback", ctypes.c_int32),
        ("median", ctypes.c_float),
        ("floor", ctypes.c_float),
    ]


_lib = None


def lib(path: str = LIB_PATH):
    """Load libacq.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libacq.so not built ({path}); run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.acq_plan_geometry.argtypes = [P(AcqConfig), P(AcqGeometry)]
    L.acq_bin_frequencies.argtypes = [P(AcqConfig), P(ctypes.c_double), ctypes.c_int32]
    L.acq_workspace_size.argtypes = [P(AcqConfig), P(ctypes.c_size_t)]
    L.acq_plan.argtypes = [P(AcqConfig), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, P(ctypes.c_void_p)]
    L.acq_detect.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, P(AcqDetection),
                             ctypes.c_int32, P(ctypes.c_int32)]
    L.acq_correlate_power.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    L.acq_detect_batch.argtypes = [ctypes.c_void_p, P(ctypes.c_void_p), P(ctypes.c_int64), ctypes.c_int32,
                                   P(AcqDetection), ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.acq_collect.argtypes = [ctypes.c_void_p, P(AcqDetection), ctypes.c_int32, P(ctypes.c_int32)]
    L.acq_device_results.argtypes = [ctypes.c_void_p, P(ctypes.c_void_p), P(ctypes.c_void_p)]
    L.acq_detect_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_void_p]
    L.acq_track_batch.argtypes = [ctypes.c_void_p, P(AcqTrackTask), ctypes.c_int32, P(AcqDetection),
                                  ctypes.c_int32, P(ctypes.c_int32)]
    L.acq_get_tuning.argtypes = [ctypes.c_void_p, P(AcqTuning)]
    L.acq_set_tuning.argtypes = [ctypes.c_void_p, P(AcqTuning)]
    L.acq_tune_fft_len.argtypes = [P(AcqConfig), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                   P(AcqTuneEntry), ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.acq_tune.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, P(AcqTuneEntry),
                           ctypes.c_int32, P(ctypes.c_int32)]
    L.acq_release.argtypes = [ctypes.c_void_p]
    L.acq_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.acq_last_kernel_times.argtypes = [ctypes.c_void_p, P(ctypes.c_double), ctypes.c_int32,
                                        P(ctypes.c_int32)]
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.acq_cnn_num_params.argtypes = [i32]
    L.acq_cnn_num_params.restype = i64
    L.acq_cnn_create.argtypes = [P(AcqCnnConfig), vp, P(vp)]
    L.acq_cnn_release.argtypes = [vp]
    L.acq_cnn_set_params.argtypes = [vp, P(ctypes.c_float), i64]
    L.acq_cnn_get_params.argtypes = [vp, P(ctypes.c_float), i64]
    L.acq_cnn_forward.argtypes = [vp, vp, i32, i64, vp]
    L.acq_cnn_gradients.argtypes = [vp, vp, i32, i64, vp, f32, vp, P(ctypes.c_float)]
    L.acq_cnn_adam_step.argtypes = [vp, f32]
    L.acq_power_map.argtypes = [vp, vp, i64, vp, P(ctypes.c_float)]
    L.acq_synth_block.argtypes = [vp, P(AcqSynthBatch), vp]
    L.acq_synth_labels.argtypes = [vp, P(AcqSynthBatch), vp]
    L.acq_cnn_train_synthetic.argtypes = [vp, P(AcqSynthBatch), f32, f32, P(ctypes.c_float)]
    L.acq_detect_learned.argtypes = [vp, vp, vp, i64, P(AcqLearnedParams), P(AcqDetection), i32, P(i32),
                                     P(AcqLearnedReport)]
    L.acq_detect_batch_learned.argtypes = [vp, vp, P(vp), P(i64), i32, P(AcqLearnedParams), P(AcqDetection), i32,
                                           P(i32), P(AcqLearnedReport)]
    L.acq_fsk_plan_geometry.argtypes = [P(AcqFskConfig), P(AcqFskGeometry)]
    L.acq_fsk_plan.argtypes = [P(AcqFskConfig), vp, P(vp)]
    L.acq_fsk_release.argtypes = [vp]
    L.acq_fsk_demod.argtypes = [vp, vp, i64, vp, vp]
    L.acq_fsk_template.argtypes = [vp, i32, vp]
    L.acq_fsk_detect.argtypes = [vp, vp, i64, P(AcqFskDetection), i32, P(i32)]
    L.acq_fsk_xcorr.argtypes = [vp, vp, i64, vp]
    L.acq_fsk_track.argtypes = [vp, P(AcqFskTask), i32, P(AcqFskDetection), i32, P(i32)]
    L.acq_fsk_set_profiling.argtypes = [vp, ctypes.c_int]
    L.acq_fsk_last_kernel_times.argtypes = [vp, P(ctypes.c_double), i32]
    for name in ("acq_fsk_plan_geometry", "acq_fsk_plan", "acq_fsk_release", "acq_fsk_demod", "acq_fsk_template",
                 "acq_fsk_xcorr", "acq_fsk_detect", "acq_fsk_track", "acq_fsk_set_profiling",
                 "acq_fsk_last_kernel_times"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("acq_plan_geometry", "acq_workspace_size", "acq_bin_frequencies", "acq_plan", "acq_detect",
                 "acq_detect_batch", "acq_track_batch", "acq_collect", "acq_device_results", "acq_detect_noalloc",
                 "acq_get_tuning", "acq_set_tuning", "acq_tune", "acq_tune_fft_len", "acq_correlate_power",
                 "acq_release", "acq_set_profiling", "acq_last_kernel_times", "acq_cnn_create",
                 "acq_cnn_release", "acq_cnn_set_params", "acq_cnn_get_params", "acq_cnn_forward",
                 "acq_cnn_gradients", "acq_cnn_adam_step", "acq_power_map", "acq_synth_block", "acq_synth_labels",
                 "acq_cnn_train_synthetic", "acq_detect_learned", "acq_detect_batch_learned"):
        getattr(L, name).restype = ctypes.c_int
    L.acq_strerror.argtypes = [ctypes.c_int]
    L.acq_strerror.restype = ctypes.c_char_p
    L.acq_last_error.argtypes = []
    L.acq_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


class AcqError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.acq_last_error().decode() or L.acq_strerror(status).decode()
        super().__init__(f"{where}: {L.acq_strerror(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str) -> int:
    if status != ACQ_OK:
        raise AcqError(status, where)
    return status
