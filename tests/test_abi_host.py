"""Host-side checks of the C ABI: the library loads, exports what the header
declares, and validates configurations before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import siggen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_2005_10445_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2005_10445_amd.build import build
        build()
    return _capi


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "acq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(acq_\w+)\s*\(", src, flags=re.M))


def test_header_symbols_exported(capi):
    declared = _declared_functions()
    assert declared == set(capi.EXPORTED)
    L = capi.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_header_constants_mirrored(capi):
    """The binding's copies of the header's constants: profiling modes, kernel
    timer order, proposal fallbacks."""
    src = open(os.path.join(ROOT, "include", "acq.h")).read()
    defs = {k: int(v) for k, v in re.findall(r"^#define\s+ACQ_(\w+)\s+\(?(-?\d+)\)?\s*$", src, flags=re.M)}
    assert (defs["PROFILE_OFF"], defs["PROFILE_ALL"], defs["PROFILE_CORRELATE"]) == \
        (capi.PROFILE_OFF, capi.PROFILE_ALL, capi.PROFILE_CORRELATE)
    assert defs["NUM_KERNELS"] == len(capi.KERNELS)
    for i, name in enumerate(capi.KERNELS):
        assert defs["KERNEL_" + name.upper()] == i
    assert (defs["FALLBACK_NONE"], defs["FALLBACK_FRACTION"], defs["FALLBACK_FLOOR"]) == \
        (capi.ACQ_FALLBACK_NONE, capi.ACQ_FALLBACK_FRACTION, capi.ACQ_FALLBACK_FLOOR)


def _cfg(capi, **over):
    from paper_2005_10445_amd import make_config
    kw = dict(chips=siggen.make_codes(1, 4, 8192), spc=2, fs_hz=8e6, num_bins=11, bin_step_hz=1000.0,
              max_block_len=1 << 20, fft_len=1 << 15)
    kw.update(over)
    return make_config(**kw)


def _status(capi, cfg):
    g = capi.AcqGeometry()
    return capi.lib().acq_plan_geometry(ctypes.byref(cfg), ctypes.byref(g)), g


def test_geometry_of_the_tag_bank_workload(capi):
    cfg, keep = _cfg(capi)
    rc, g = _status(capi, cfg)
    assert rc == 0
    assert (g.template_len, g.min_fft_len, g.fft_len, g.sub_fft_len) == (16384, 32768, 32768, 16384)
    assert g.valid_per_segment == 16385
    assert g.max_segments == 63
    assert g.freq_quantum_hz == 244.140625 and g.bin_step_hz == 976.5625


def test_bins_agree_with_oracle_reading(capi):
    from paper_2005_10445_amd import bin_frequencies
    for K, step, centre in ((11, 1000.0, 0.0), (21, 1000.0, 0.0), (5, 3333.0, 1234.0), (1, 0.0, 0.0)):
        f = bin_frequencies(chips=siggen.make_codes(1, 2, 8192), spc=2, fs_hz=8e6, num_bins=K,
                            bin_step_hz=step, bin_center_hz=centre, max_block_len=1 << 20)
        ref, _ = oracle.snap_bins(8e6, 16384, K, centre, step)
        np.testing.assert_array_equal(f, ref)


def test_default_segment_length_choice(capi):
    from paper_2005_10445_amd import geometry
    g = geometry(chips=siggen.make_codes(1, 1, 1024), spc=4, fs_hz=8e6, max_block_len=1 << 17)
    assert g["template_len"] == 4096 and g["min_fft_len"] == 8192
    assert g["fft_len"] >= 8192 and g["fft_len"] // 4 <= 16384
    assert g["max_segments"] * g["valid_per_segment"] >= (1 << 17) - 4096 + 1


@pytest.mark.parametrize("over,status", [
    (dict(num_bins=4), -1),
    (dict(spc=3), -7),
    (dict(fft_len=3 << 14), -1),
    (dict(fft_len=1 << 14), -1),
    (dict(fft_len=1 << 16), -7),
    (dict(refine_radius=9), -1),
    (dict(fs_hz=0.0), -1),
    (dict(max_block_len=0), -1),
    (dict(bin_step_hz=0.0), -1),
])
def test_invalid_configs_rejected(capi, over, status):
    cfg, keep = _cfg(capi, **over)
    rc, _ = _status(capi, cfg)
    assert rc == status, capi.lib().acq_last_error()


def test_chips_must_be_pm1(capi):
    chips = siggen.make_codes(1, 2, 64)
    chips[1, 5] = 0
    cfg, keep = _cfg(capi, chips=chips, fft_len=0)
    rc, _ = _status(capi, cfg)
    assert rc == -1 and b"chips" in capi.lib().acq_last_error()


def test_null_handles_rejected_without_gpu(capi):
    L = capi.lib()
    n = ctypes.c_int32(5)
    out = (capi.AcqDetection * 1)()
    assert L.acq_detect(None, None, 10, out, 1, ctypes.byref(n)) == -1
    assert L.acq_correlate_power(None, None, 10, None) == -1
    assert L.acq_release(None) == 0
    assert L.acq_plan(None, None, 0, None, None) == -1
    assert L.acq_collect(None, out, 1, ctypes.byref(n)) == -1
    rec, cnt = ctypes.c_void_p(), ctypes.c_void_p()
    assert L.acq_device_results(None, ctypes.byref(rec), ctypes.byref(cnt)) == -1
    assert L.acq_detect_batch(None, None, None, 1, out, 1, ctypes.byref(n), None) == -1
    assert L.acq_strerror(-4) == b"output truncated"
    assert L.acq_strerror(-6) == b"workspace too small"
    assert L.acq_strerror(-8) == b"non-finite samples"
    assert L.acq_strerror(0) == b"ok"


def test_detection_record_layout(capi):
    # tag, bin, lag, 8 doubles (toa .. snr), block, flags, crossings
    assert ctypes.sizeof(capi.AcqDetection) == 4 + 4 + 8 + 8 * 8 + 4 + 4 + 8
    assert capi.AcqDetection.crossings.offset == 88


def test_workspace_size_and_caller_workspace_checked_before_the_gpu(capi):
    """The per-search workspace (Section 4.2: buffers allocated once): its size is
    the same from acq_workspace_size and the geometry, grows with the batch
    capacity, and a caller workspace that is too small or misaligned is refused
    before any device call."""
    L = capi.lib()
    cfg, keep = _cfg(capi)
    need = ctypes.c_size_t(0)
    assert L.acq_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == 0
    rc, g = _status(capi, cfg)
    assert rc == 0 and g.workspace_bytes == need.value and g.device_bytes > g.workspace_bytes
    # 63 segment spectra of 2^15 FP32 complex values dominate
    assert 63 * (1 << 15) * 8 <= need.value <= 63 * (1 << 15) * 8 + (4 << 20)
    big, keep2 = _cfg(capi, max_batch_blocks=4)
    need4 = ctypes.c_size_t(0)
    assert L.acq_workspace_size(ctypes.byref(big), ctypes.byref(need4)) == 0 and need4.value > need.value
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)                  # never dereferenced: the size check comes first
    assert L.acq_plan(ctypes.byref(cfg), fake, need.value - 1, None, ctypes.byref(h)) == capi.ACQ_ERR_WORKSPACE_TOO_SMALL
    assert not h.value and b"workspace" in L.acq_last_error()
    assert L.acq_plan(ctypes.byref(cfg), ctypes.c_void_p((1 << 20) + 8), need.value, None,
                      ctypes.byref(h)) == capi.ACQ_ERR_INVALID_ARG
    assert L.acq_workspace_size(None, ctypes.byref(need)) == -1


def test_async_and_finite_flags_accepted_unknown_flags_refused(capi):
    from paper_2005_10445_amd import geometry
    kw = dict(chips=siggen.make_codes(1, 2, 1000), spc=2, fs_hz=8e6, max_block_len=50000)
    assert geometry(asynchronous=True, check_finite=True, **kw)["fft_len"] > 0
    cfg, keep = _cfg(capi)
    cfg.flags = 0x10
    assert _status(capi, cfg)[0] == -1


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_2005_10445_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "direct.c" not in text, f


def test_network_parameter_count_matches_the_oracle_layout(capi):
    from oracle import learned as ol
    L = capi.lib()
    for cin in (256, 64, 5):
        net = ol.init_cnn(0, cin=cin)
        assert L.acq_cnn_num_params(cin) == sum(v.size for v in net.params().values())
    assert L.acq_cnn_num_params(0) == 0


def test_network_calls_reject_null_handles_without_gpu(capi):
    L = capi.lib()
    loss = ctypes.c_float(0)
    assert L.acq_cnn_create(None, None, None) == -1
    assert L.acq_cnn_release(None) == 0
    assert L.acq_cnn_set_params(None, None, 0) == -1
    assert L.acq_cnn_forward(None, None, 1, 1, None) == -1
    assert L.acq_cnn_gradients(None, None, 1, 1, None, 1.0, None, ctypes.byref(loss)) == -1
    assert L.acq_cnn_adam_step(None, 1e-3) == -1
    assert L.acq_power_map(None, None, 0, None, None) == -1
    assert L.acq_synth_block(None, None, None) == -1
    assert L.acq_cnn_train_synthetic(None, None, 1.0, 1e-3, ctypes.byref(loss)) == -1
    n = ctypes.c_int32(0)
    assert L.acq_detect_learned(None, None, None, 0, None, None, 0, ctypes.byref(n), None) == -1


def test_network_config_validation_without_gpu(capi):
    L = capi.lib()
    h = ctypes.c_void_p()
    bad = [capi.AcqCnnConfig(capi.ACQ_FP16, 256, 1024, 1 << 17),   # precision
           capi.AcqCnnConfig(capi.ACQ_BF16, 100, 1024, 1 << 17),   # bf16 needs multiples of 64
           capi.AcqCnnConfig(capi.ACQ_BF16, 256, 0, 0),            # rows
           capi.AcqCnnConfig(capi.ACQ_BF16, 256, 100, 1 << 17)]    # block needs more frames than rows
    for cfg in bad:
        assert L.acq_cnn_create(ctypes.byref(cfg), None, ctypes.byref(h)) in (-1, -7)
        assert not h.value


def test_exact_bins_report_the_requested_frequencies(capi):
    import numpy as np
    from paper_2005_10445_amd import bin_frequencies, geometry
    chips = np.ones((2, 1000), np.int8)
    kw = dict(chips=chips, spc=2, fs_hz=8e6, num_bins=5, bin_center_hz=123.4, bin_step_hz=1000.3,
              max_block_len=50000)
    f = bin_frequencies(exact_bins=True, **kw)
    assert np.array_equal(f, 123.4 + (np.arange(5) - 2) * 1000.3)
    snapped = bin_frequencies(**kw)
    q = 8e6 / 2048
    assert np.allclose(snapped / q, np.round(snapped / q)) and not np.array_equal(f, snapped)
    g = geometry(exact_bins=True, **kw)
    assert g["device_bytes"] > geometry(**kw)["device_bytes"]      # one set of spectra per residual


def test_track_batch_validates_without_a_gpu(capi):
    import ctypes
    from paper_2005_10445_amd import _capi
    L = _capi.lib()
    assert ctypes.sizeof(_capi.AcqTrackTask) == 24
    nf = ctypes.c_int32(7)
    task = _capi.AcqTrackTask(None, 0, 0, 0)
    assert L.acq_track_batch(None, ctypes.byref(task), 1, None, 0, ctypes.byref(nf)) == _capi.ACQ_ERR_INVALID_ARG
