"""Write the expected detection sets of whole stream blocks (oracle only).

The batched-stream workload (256 tags x 21 bins over +/-10 kHz, 64 blocks of
uneven length log-uniform in [2^18, 2^21], seed 4000) is too large for the FP64
oracle to run inside a GPU test, so its results for the two shortest blocks are
computed here, once, by `oracle.acquire(method="fft")` (argmax from the FFT
identity over every tag and bin, peak triple and values from the direct
definition) and stored as JSON.  The blocks themselves are regenerated from
the seed by `siggen` wherever the file is used.

    python tests/golden/make_stream_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import siggen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stream_seed4000_shortest2.json")
FIELDS = ("tag", "detected", "bin", "lag", "toa", "peak_power", "z", "energy", "power", "snr", "block_power",
          "freq_hz", "near_edge", "near_tie", "near_threshold", "theta", "crossings", "crossings_band")


def main():
    w = siggen.workload("batched_stream")
    T, C, spc, K = w["num_tags"], w["num_chips"], w["spc"], w["num_bins"]
    L = C * spc
    seed = w["seeds"][0]
    chips = siggen.make_codes(seed, T, C)
    freqs, _ = oracle.snap_bins(w["fs_hz"], L, K, 0.0, w["bin_step_hz"])
    blocks = siggen.make_stream_batch(seed, chips, spc, w["fs_hz"], freqs, w["num_blocks"], w["block_len_log2"],
                                      w["receivers"], w["n_tx"], w["snr_db"])
    order = [int(b) for b in np.argsort([x.size for x, _ in blocks])[:2]]
    out = {"what": "oracle.acquire(method='fft') over every tag of the two shortest blocks of the "
                   "batched-stream workload, seed 4000 (default threshold)",
           "command": "python tests/golden/make_stream_golden.py",
           "seed": seed, "blocks": {}}
    for b in order:
        x, txs = blocks[b]
        t0 = time.perf_counter()
        res = oracle.acquire(x, chips, spc, freqs, w["fs_hz"], method="fft")
        print(f"block {b}: {x.size} samples, {sum(r['detected'] for r in res)} detections, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
        keep = [r for r in res if r["detected"] or r["near_threshold"]]
        out["blocks"][str(b)] = {"n": int(x.size), "injected": [t.as_dict() for t in txs],
                                 "results": [{k: r[k] for k in FIELDS} for r in keep]}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
