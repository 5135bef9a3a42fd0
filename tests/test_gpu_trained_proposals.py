"""The committed trained proposal network against the exhaustive search.

The network in paper_2005_10445_amd/weights/ (trained on the GPU by the
library's own kernels on synthetic tag-bank blocks) and its calibrated window
threshold kappa are loaded as a user would load them.  On held-out data the
proposal search must:
  * return a bit-exact subset of the exhaustive search's detections (inside a
    searched segment every value is the exhaustive one);
  * keep recall >= 0.995 over the exhaustive detections of injected
    transmissions, on the 64-block batched stream (seed 4001: 256 tags x 21
    bins, blocks log-uniform in [2^18, 2^21], 0-20 transmissions each);
  * search fewer segments than the exhaustive search, and take less GPU time.
"""
import json
import os

import numpy as np
import pytest

import siggen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2005_10445_amd",
                       "weights")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _trained_net(max_rows, max_block_len):
    from paper_2005_10445_amd.proposals import Network, num_params
    params = np.load(os.path.join(WEIGHTS, "proposal_cnn.npy"), allow_pickle=False)
    assert params.dtype == np.float32 and params.size == num_params(256)
    with open(os.path.join(WEIGHTS, "proposal_cnn.json")) as f:
        kappa = float(json.load(f)["kappa"])
    net = Network("bf16", 256, max_rows=max_rows, max_block_len=max_block_len)
    net.set_params(params)
    return net, kappa


def _key(d):
    return (d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power, d.z, d.energy, d.flags)


def _is_injected(d, txs, tol=2):
    return any(d.tag == t.tag and d.bin == t.bin and abs(d.lag - t.delay) <= tol for t in txs)


def _timed(fn, reps=2):
    """Mean GPU time (ms) of fn between events on the current stream, after one warm-up."""
    out = fn()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = fn()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return out, float(np.mean(ms))


@pytest.mark.timeout(900)
def test_trained_network_on_held_out_stream(dev):
    from paper_2005_10445_amd import Plan
    from paper_2005_10445_amd.proposals import LearnedParams
    w = siggen.workload("batched_stream")
    T, C, spc, K = w["num_tags"], w["num_chips"], w["spc"], w["num_bins"]
    chips = siggen.make_codes(w["seeds"][0], T, C)
    from paper_2005_10445_amd import bin_frequencies
    freqs = bin_frequencies(chips=chips, spc=spc, fs_hz=w["fs_hz"], num_bins=K, bin_step_hz=w["bin_step_hz"],
                            max_block_len=1 << 21, fft_len=1 << 15)
    print("[trained] generating 64 held-out stream blocks (seed 4001)", flush=True)
    data = siggen.make_stream_batch(4001, chips, spc, w["fs_hz"], freqs, w["num_blocks"], w["block_len_log2"],
                                    w["receivers"], w["n_tx"], w["snr_db"])
    xs = [torch.from_numpy(x).to(dev) for x, _ in data]
    total = sum(x.numel() for x in xs)
    net, kappa = _trained_net(1 << 15, 1 << 21)
    lp = LearnedParams(kappa=kappa, max_fraction=0.5, floor_db=1.0)
    with Plan(chips, spc, w["fs_hz"], num_bins=K, bin_step_hz=w["bin_step_hz"], max_block_len=max(
            x.numel() for x in xs), fft_len=1 << 15, max_batch_blocks=len(xs), max_batch_samples=total) as plan:
        full, ms_full = _timed(lambda: plan.detect_batch(xs))
        print(f"[trained] exhaustive batch {ms_full:.1f} ms, {len(full)} detections", flush=True)
        (learned, reps), ms_learned = _timed(lambda: net.detect_batch(plan, xs, lp))
        print(f"[trained] proposal batch {ms_learned:.1f} ms, {len(learned)} detections", flush=True)
    net.close()
    fk = {_key(d) for d in full}
    lk = {_key(d) for d in learned}
    assert lk <= fk, sorted(lk - fk)[:5]                  # bit-exact subset
    inj = [d for d in full if _is_injected(d, data[d.block][1])]
    hit_inj = sum(_key(d) in lk for d in inj)
    recall_inj = hit_inj / len(inj)
    recall_all = len(lk) / len(fk)
    seg = sum(r.segments for r in reps) / sum(r.total_segments for r in reps)
    fallbacks = sum(r.fallback != 0 for r in reps)
    print(f"[trained] kappa {kappa:.2f}: recall {recall_inj:.4f} of {len(inj)} injected exhaustive detections, "
          f"{recall_all:.4f} of all {len(fk)}; segments searched {seg:.3f}; fallbacks {fallbacks}/{len(xs)}; "
          f"GPU time {ms_learned:.1f} ms vs {ms_full:.1f} ms exhaustive ({ms_full / ms_learned:.2f}x)", flush=True)
    assert len(inj) >= 500
    assert recall_inj >= 0.995
    assert seg < 0.75
    assert ms_learned < ms_full


@pytest.mark.timeout(600)
def test_trained_network_on_held_out_tagbank_blocks(dev):
    """Tag-bank blocks (64 tags, 11 bins, 2^20 samples, ten transmissions at -15..-5 dB)
    from seeds the calibration did not see: a bit-exact subset, fewer segments,
    and the injected detections kept (at most one miss in the sample)."""
    from paper_2005_10445_amd import Plan
    from paper_2005_10445_amd.proposals import LearnedParams
    w = siggen.workload("tagbank_fp32")
    T, C, spc, K, N = w["num_tags"], w["num_chips"], w["spc"], w["num_bins"], w["block_len"]
    chips = siggen.make_codes(w["seeds"][0], T, C)
    net, kappa = _trained_net(1 << 14, 1 << 21)
    lp = LearnedParams(kappa=kappa, max_fraction=0.5, floor_db=0.0)
    hit = total = 0
    segs = segs_total = 0
    with Plan(chips, spc, w["fs_hz"], num_bins=K, bin_step_hz=w["bin_step_hz"], max_block_len=N,
              fft_len=w["fft_len"]) as plan:
        for i in range(12):
            x, txs = siggen.make_block(2_100_000 + i, N, chips, spc, w["fs_hz"], plan.freqs_hz, w["n_tx"],
                                       snr_db=w["snr_db"])
            xd = torch.from_numpy(x).to(dev)
            full = plan.detect(xd)
            dets, rep = net.detect(plan, xd, lp)
            fk = {_key(d) for d in full}
            lk = {_key(d) for d in dets}
            assert lk <= fk, i
            for d in full:
                if _is_injected(d, txs):
                    total += 1
                    hit += _key(d) in lk
            segs += rep.segments
            segs_total += rep.total_segments
    net.close()
    print(f"[trained] tag-bank held-out: {hit}/{total} injected detections kept, "
          f"segments searched {segs / segs_total:.3f}", flush=True)
    assert total >= 100 and total - hit <= 1
    assert segs < segs_total
