import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build_library(force=False)
    return oracle


@pytest.fixture(scope="session")
def tagbank_case():
    """The 64-tag x 11-bin x 2^20-sample block (first seed of the workload) and
    the oracle's per-tag result for it (FFT-identity search, FP64), shared by
    the full-size GPU tests."""
    import oracle
    import siggen
    w = siggen.workload("tagbank_fp32")
    T, C, spc, N, K = w["num_tags"], w["num_chips"], w["spc"], w["block_len"], w["num_bins"]
    seed = w["seeds"][0]
    chips = siggen.make_codes(seed, T, C)
    freqs, _ = oracle.snap_bins(w["fs_hz"], C * spc, K, 0.0, w["bin_step_hz"])
    x, txs = siggen.make_block(seed, N, chips, spc, w["fs_hz"], freqs, w["n_tx"], snr_db=w["snr_db"])
    print("[fixture] oracle search of the tag-bank block", flush=True)
    ref = oracle.acquire(x, chips, spc, freqs, w["fs_hz"], method="fft")
    return w, chips, freqs, x, txs, ref
