"""FSK configuration checks of the C ABI that need no GPU."""
import ctypes

import numpy as np
import pytest

from paper_2005_10445_amd import AcqError, _capi
from paper_2005_10445_amd.fsk import fsk_geometry


def _kw(**over):
    kw = dict(bits=np.zeros((3, 100), np.uint8), fs_hz=8e6, lo_hz=0.0, f1_hz=250e3, f0_hz=-250e3,
              bp_taps=np.ones(31), mf_len=8, max_block_len=5000)
    kw.update(over)
    return kw


def test_geometry():
    g = fsk_geometry(**_kw())
    assert g["template_len"] == 100 * 8 + 31 + 8 - 2 and g["filter_len"] == 38 and g["front_fft_len"] == 4096
    assert g["fft_len"] == 2048 and g["valid_per_segment"] == 2048 - g["template_len"] + 1
    # the paper's template: a 100 ms window takes 4 segments of 2^18 points (2
    # transforms) rather than 12 of 2^17 (6 transforms); tracking tasks of 12 ms
    # take one 2^17-point segment each
    p = fsk_geometry(**_kw(bits=np.zeros((2, 8192), np.uint8), bp_taps=np.ones(200), max_block_len=800000))
    assert p["template_len"] == 65742 and p["fft_len"] == 1 << 18
    assert p["valid_per_segment"] == (1 << 18) - 65742 + 1
    t = fsk_geometry(**_kw(bits=np.zeros((2, 8192), np.uint8), bp_taps=np.ones(200), max_block_len=64 * 96000,
                           max_track_tasks=64))
    assert t["fft_len"] == 1 << 17
    f = fsk_geometry(**_kw(bits=np.zeros((2, 8192), np.uint8), bp_taps=np.ones(200), max_block_len=800000,
                           fft_len=1 << 17))
    assert f["fft_len"] == 1 << 17


@pytest.mark.parametrize("over, status", [
    (dict(bp_taps=np.ones(1025)), -1), (dict(mf_len=0), -1), (dict(fs_hz=0.0), -1),
    (dict(max_block_len=0), -1), (dict(fft_len=3000), -7), (dict(fft_len=512), -7), (dict(fft_len=1 << 19), -7),
    (dict(bits=np.zeros((1, 40000), np.uint8)), -7), (dict(max_track_tasks=-1), -1),
])
def test_invalid_configurations(over, status):
    with pytest.raises(AcqError) as e:
        fsk_geometry(**_kw(**over))
    assert e.value.status == status


def test_entry_points_reject_null_plans():
    L = _capi.lib()
    nf = ctypes.c_int32(0)
    assert L.acq_fsk_detect(None, None, 0, None, 0, ctypes.byref(nf)) == -1
    assert L.acq_fsk_release(None) == 0
    assert ctypes.sizeof(_capi.AcqFskDetection) == 64 and ctypes.sizeof(_capi.AcqFskTask) == 24
    assert L.acq_fsk_track(None, None, 0, None, 0, ctypes.byref(nf)) == -1
