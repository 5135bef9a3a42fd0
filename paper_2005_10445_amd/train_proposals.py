"""Train, calibrate and evaluate the proposal network on the GPU.

Training data are generated on the device (acq_cnn_train_synthetic): blocks
of the tag-bank workload's shape -- 2^20 samples at 8 Msps, ten BPSK
transmissions of 8192 chips at 2 samples per chip, per-sample SNR uniform in
[-15, -5] dB, carrier offsets on the 11-bin grid over +/-5 kHz, integer delays
-- with CN(0,1) noise.  Only the transmission parameters are drawn on the
host.  Calibration picks the proposal threshold kappa on held-out blocks so
that the proposal search keeps a target share of the exhaustive search's
detections; the exhaustive search is the reference.

    python -m paper_2005_10445_amd.train_proposals train --blocks 200000 --batch 8
    python -m paper_2005_10445_amd.train_proposals calibrate
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import List, Sequence

import numpy as np

from .proposals import LearnedParams, Network, SynthTransmission, num_params

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
WEIGHTS = os.path.join(WEIGHTS_DIR, "proposal_cnn.npy")
META = os.path.join(WEIGHTS_DIR, "proposal_cnn.json")

FS = 8e6
BLOCK_LEN = 1 << 20
CHIPS, SPC = 8192, 2
N_TX = 10
SNR_DB = (-15.0, -5.0)
BINS, BIN_STEP_HZ = 11, 976.5625       # the snapped 1 kHz grid of 16384-sample templates


def log(*a):
    print(*a, flush=True)


def he_init(seed: int, in_channels: int = 256) -> np.ndarray:
    """He-normal conv and head weights, zero biases, in the library's parameter order."""
    g = np.random.default_rng(seed)
    parts, c = [], in_channels
    for _ in range(4):
        parts.append(g.normal(0.0, math.sqrt(2.0 / (5 * c)), size=5 * c * 64))
        parts.append(np.zeros(64))
        c = 64
    parts.append(g.normal(0.0, math.sqrt(1.0 / 64), size=64))
    parts.append(np.zeros(1))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == num_params(in_channels)
    return p


def draw_transmissions(g: np.random.Generator, nblocks: int, n: int = BLOCK_LEN, n_tx: int = N_TX,
                       snr_db=SNR_DB) -> List[List[SynthTransmission]]:
    L = CHIPS * SPC
    out = []
    for _ in range(nblocks):
        lst = []
        for _ in range(n_tx):
            k = int(g.integers(0, BINS)) - BINS // 2
            snr = float(g.uniform(*snr_db))
            lst.append(SynthTransmission(delay=int(g.integers(0, n - L)), freq_over_fs=k * BIN_STEP_HZ / FS,
                                         amp=10.0 ** (snr / 20.0), phase0=float(g.random()),
                                         code=int(g.integers(0, 2 ** 32))))
        out.append(lst)
    return out


def train(blocks: int, batch: int, seed: int, lr: float, lr_final: float, pos_weight: float,
          init: np.ndarray | None = None, log_every: int = 1000):
    rows = batch * ((BLOCK_LEN - 256) // 128 + 1)
    net = Network("bf16", 256, max_rows=rows, max_block_len=BLOCK_LEN)
    net.set_params(he_init(seed) if init is None else init)
    g = np.random.default_rng(seed)
    steps = blocks // batch
    losses = []
    t0 = time.time()
    for s in range(steps):
        # cosine decay from lr to lr_final
        a = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * s / max(steps - 1, 1)))
        txs = draw_transmissions(g, batch)
        losses.append(net.train_synthetic(seed, s * batch, BLOCK_LEN, CHIPS, SPC, txs, pos_weight, a))
        if (s + 1) % log_every == 0 or s == steps - 1 or s < 3:
            log(f"[train] step {s + 1}/{steps} blocks {(s + 1) * batch} loss {np.mean(losses[-log_every:]):.4f} "
                f"lr {a:.2e} {time.time() - t0:.0f} s")
    return net, losses, time.time() - t0


def _true_key(d, txs, tol: int = 2):
    """True when detection d is the detection of an injected transmission."""
    return any(d.tag == t.tag and d.bin == t.bin and abs(d.lag - t.delay) <= tol for t in txs)


def recall_at(plan, net: Network, blocks, kappa: float, exhaustive, truth=None):
    """(recall over all exhaustive detections, recall over the exhaustive detections of injected
    transmissions, mean share of segments searched, fallbacks) of the proposal search at kappa,
    the exhaustive search being the reference (same values required)."""
    hit = total = thit = ttotal = 0
    frac = []
    fallbacks = 0
    for i, x in enumerate(blocks):
        full = exhaustive[i]
        dets, rep = net.detect(plan, x, LearnedParams(kappa=kappa, max_fraction=1.0, floor_db=0.0))
        got = {(d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in dets}
        for d in full:
            ok = (d.tag, d.bin, d.lag, d.toa, d.peak_power) in got
            total += 1
            hit += ok
            if truth is not None and _true_key(d, truth[i]):
                ttotal += 1
                thit += ok
        frac.append(rep.segments / max(rep.total_segments, 1))
        fallbacks += rep.fallback != 0
    return (hit / total if total else 1.0, thit / ttotal if ttotal else 1.0, float(np.mean(frac)), fallbacks)


def calibrate(plan, net: Network, blocks, truth, target: float, lo: float = -5000.0, hi: float = 5000.0,
              iters: int = 30):
    """Largest kappa (bisection: a larger kappa proposes a subset) whose recall over the
    exhaustive detections of injected transmissions reaches target."""
    exhaustive = [plan.detect(x) for x in blocks]
    if recall_at(plan, net, blocks, lo, exhaustive, truth)[1] < target:
        return lo
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if recall_at(plan, net, blocks, mid, exhaustive, truth)[1] >= target:
            lo = mid
        else:
            hi = mid
    return lo


def load_model(path: str = WEIGHTS, meta: str = META):
    p = np.load(path)
    with open(meta) as f:
        m = json.load(f)
    return p, m


def cmd_calibrate(args):
    """kappa for the target recall on held-out tag-bank blocks (64 tags, 11 bins, 2^20 samples)."""
    import torch
    import siggen
    from . import Plan
    w = siggen.workload("tagbank_fp32")
    chips = siggen.make_codes(w["seeds"][0], w["num_tags"], w["num_chips"])
    plan = Plan(chips, w["spc"], w["fs_hz"], num_bins=w["num_bins"], bin_step_hz=w["bin_step_hz"],
                max_block_len=w["block_len"], fft_len=w["fft_len"])
    blocks, truth = [], []
    for i in range(args.blocks):
        x, txs = siggen.make_block(args.seed + i, w["block_len"], chips, w["spc"], w["fs_hz"], plan.freqs_hz,
                                   w["n_tx"], snr_db=w["snr_db"])
        blocks.append(torch.from_numpy(x).cuda())
        truth.append(txs)
        if (i + 1) % 10 == 0:
            log(f"[calibrate] generated {i + 1}/{args.blocks}")
    net = Network("bf16", 256, max_rows=1 << 14, max_block_len=1 << 21)
    net.set_params(np.load(args.weights))
    kappa = calibrate(plan, net, blocks, truth, args.target)
    exhaustive = [plan.detect(x) for x in blocks]
    r, rt, frac, fb = recall_at(plan, net, blocks, kappa, exhaustive, truth)
    meta = {"kappa": kappa, "target_recall_injected": args.target, "recall_injected": rt, "recall_all": r,
            "segment_fraction": frac, "blocks": args.blocks, "seed": args.seed, "workload": "tagbank_fp32"}
    with open(args.meta, "w") as f:
        json.dump(meta, f, indent=1)
    log(json.dumps(meta))


def cmd_evaluate(args):
    """Recall, searched share and speed of the proposal search against the exhaustive search
    on the batched-stream workload (256 tags, 21 bins, uneven blocks)."""
    import torch
    import siggen
    from . import Plan
    w = siggen.workload("batched_stream")
    chips = siggen.make_codes(w["seeds"][0], w["num_tags"], w["num_chips"])
    with open(args.meta) as f:
        meta = json.load(f)
    from . import bin_frequencies
    freqs = bin_frequencies(chips=chips, spc=w["spc"], fs_hz=w["fs_hz"], num_bins=w["num_bins"],
                            bin_step_hz=w["bin_step_hz"], max_block_len=1 << 21, fft_len=1 << 15)
    data = siggen.make_stream_batch(args.seed, chips, w["spc"], w["fs_hz"], freqs, args.blocks,
                                    w["block_len_log2"], w["receivers"], w["n_tx"], w["snr_db"])
    xs = [torch.from_numpy(x).cuda() for x, _ in data]
    plan = Plan(chips, w["spc"], w["fs_hz"], num_bins=w["num_bins"], bin_step_hz=w["bin_step_hz"],
                max_block_len=max(x.numel() for x in xs), fft_len=1 << 15, max_batch_blocks=len(xs),
                max_batch_samples=sum(x.numel() for x in xs))
    net = Network("bf16", 256, max_rows=1 << 15, max_block_len=1 << 21)
    net.set_params(np.load(args.weights))
    lp = LearnedParams(kappa=meta["kappa"], max_fraction=args.max_fraction, floor_db=args.floor_db)
    for x in xs[:2]:                      # warm up both paths
        plan.detect(x)
        net.detect(plan, x, lp)
    torch.cuda.synchronize()
    t_full = t_learned = 0.0
    hit = total = extra = thit = ttotal = 0
    segs = segs_total = fallbacks = 0
    full_keys = set()
    for b, (x, (_, txs)) in enumerate(zip(xs, data)):
        t0 = time.perf_counter()
        full = plan.detect(x)
        full_keys |= {(b, d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in full}
        t1 = time.perf_counter()
        dets, rep = net.detect(plan, x, lp)
        t2 = time.perf_counter()
        t_full += t1 - t0
        t_learned += t2 - t1
        fk = {(d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in full}
        lk = {(d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in dets}
        total += len(fk)
        hit += len(fk & lk)
        extra += len(lk - fk)
        for d in full:
            if _true_key(d, txs):
                ttotal += 1
                thit += (d.tag, d.bin, d.lag, d.toa, d.peak_power) in lk
        segs += rep.segments
        segs_total += rep.total_segments
        fallbacks += rep.fallback != 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.detect_batch(xs)
    t_batch = time.perf_counter() - t0
    # the batched proposal search (fresh noise floor, as for the per-block pass)
    net2 = Network("bf16", 256, max_rows=1 << 15, max_block_len=1 << 21)
    net2.set_params(np.load(args.weights))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bdets, breps = net2.detect_batch(plan, xs, lp)
    t_batch_learned = time.perf_counter() - t0
    bk = {(d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power) for d in bdets}

    out = {"blocks": len(xs), "samples": int(sum(x.numel() for x in xs)), "kappa": meta["kappa"],
           "recall_all": hit / max(total, 1), "recall_injected": thit / max(ttotal, 1),
           "exhaustive_detections": total, "exhaustive_injected_detections": ttotal, "extra_detections": extra,
           "segments_searched": segs / max(segs_total, 1), "fallbacks": fallbacks,
           "ms_exhaustive_per_block_calls": 1e3 * t_full, "ms_exhaustive_batch": 1e3 * t_batch,
           "ms_learned": 1e3 * t_learned, "speedup_vs_per_block": t_full / t_learned,
           "speedup_vs_batch": t_batch / t_learned,
           "ms_learned_batch": 1e3 * t_batch_learned, "speedup_batch_learned_vs_batch": t_batch / t_batch_learned,
           "recall_all_batch_learned": len(full_keys & bk) / max(len(full_keys), 1),
           "extra_detections_batch_learned": len(bk - full_keys)}
    log(json.dumps(out))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(out, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("calibrate")
    c.add_argument("--blocks", type=int, default=50)
    c.add_argument("--seed", type=int, default=2_000_000)
    c.add_argument("--target", type=float, default=0.995)
    c.add_argument("--weights", default=WEIGHTS)
    c.add_argument("--meta", default=META)
    e = sub.add_parser("evaluate")
    e.add_argument("--blocks", type=int, default=64)
    e.add_argument("--seed", type=int, default=4001)
    e.add_argument("--max-fraction", type=float, default=0.5)
    e.add_argument("--floor-db", type=float, default=1.0)
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--meta", default=META)
    e.add_argument("--report", default="")
    t = sub.add_parser("train")
    t.add_argument("--blocks", type=int, default=200000)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--seed", type=int, default=1_000_000)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--lr-final", type=float, default=1e-4)
    t.add_argument("--pos-weight", type=float, default=4.0)
    t.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args(argv)
    if args.cmd == "calibrate":
        return cmd_calibrate(args)
    if args.cmd == "evaluate":
        return cmd_evaluate(args)
    if args.cmd == "train":
        net, losses, secs = train(args.blocks, args.batch, args.seed, args.lr, args.lr_final, args.pos_weight)
        os.makedirs(os.path.dirname(args.out), exist_ok=True)
        np.save(args.out, net.get_params())
        meta = {"blocks": args.blocks, "batch": args.batch, "seed": args.seed, "lr": args.lr,
                "lr_final": args.lr_final, "pos_weight": args.pos_weight, "seconds": secs,
                "loss_first": float(np.mean(losses[:50])), "loss_last": float(np.mean(losses[-50:])),
                "loss_curve": [float(np.mean(losses[i:i + 500])) for i in range(0, len(losses), 500)]}
        with open(os.path.splitext(args.out)[0] + ".train.json", "w") as f:
            json.dump(meta, f, indent=1)
        log(json.dumps({k: v for k, v in meta.items() if k != "loss_curve"}))


if __name__ == "__main__":
    sys.exit(main())
