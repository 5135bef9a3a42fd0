"""Throughput of the acquisition hot path on one MI355X.

One step = one acq_detect call on one resident block: block power, segment
spectra, correlation of every tag x bin x lag, peak keys, FP64 refinement and
the copy of the detections to the host (--workload batched_stream: one
acq_detect_batch call over 64 resident blocks of uneven length, 256 tags x 21
bins, optionally replayed from a captured hipGraph; --workload tracking: one
acq_track_batch call over 256 tracking tasks, each one tag x 21 bins over a
block 1.5 templates long; --workload fsk_search: one acq_fsk_detect call on a
100 ms window of int16 samples at 8 Msps against 128 FSK codes of 8192 bits,
the paper's searching task).  Default workload: 64 tags with
8192-chip codes at 2 samples/chip, 11 carrier-offset bins over +/-5 kHz,
2^20-sample blocks at 8 Msps, overlap-save segments of 2^15 samples, ten
transmissions per block at -15..-5 dB (synthetic, seeded).

Prints one JSON line on stdout.  Reported beside the throughput:
  roofline     : the correlation kernel's algorithmic FLOP rate (5 M log2 M per
                 inverse transform + 6 M per spectrum product + 4 per valid
                 lag, per tag x bin x segment) over its mean duration from HIP
                 events recorded on the plan's stream during the timed steps,
                 against the FP32 vector peak;
  cpu_baseline : the FP64 CPU oracle (direct definition) on a bounded sample
                 of tag x bin pairs of the same block, on this host's cores
                 (all of them, and one);
and, for the default workload, the extra legs of --legs: mixed (the block
with FP16 and with BF16 storage against the FP32 detections), stream (the
64-block batched stream, eager and graph-replayed) and learned (the trained
proposal network on that stream against its exhaustive search).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# rocprofv3 HBM byte counts of the correlation kernel, per workload
TRAFFIC_FILES = {"tagbank_fp32": os.path.join(ROOT, "profiles", "correlate_tagbank_traffic.json"),
                 "tagbank_fp16": os.path.join(ROOT, "profiles", "correlate_tagbank_fp16_traffic.json"),
                 "tagbank_bf16": os.path.join(ROOT, "profiles", "correlate_tagbank_bf16_traffic.json"),
                 "batched_stream": os.path.join(ROOT, "profiles", "correlate_stream_traffic.json"),
                 "tracking": os.path.join(ROOT, "profiles", "correlate_tracking_traffic.json"),
                 "fsk_search": os.path.join(ROOT, "profiles", "fsk_correlate_traffic.json"),
                 "fsk_tracking": os.path.join(ROOT, "profiles", "fsk_tracking_correlate_traffic.json")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def correlate_flops(T, K, S, M, V) -> float:
    return float(T) * K * S * (5.0 * M * math.log2(M) + 6.0 * M + 4.0 * V)


def traffic_per_launch(workload: str):
    """HBM bytes per correlation launch from the committed counter summary of the
    workload, if it was taken on the current kernel source; else None."""
    if workload not in TRAFFIC_FILES:
        return None
    try:
        with open(TRAFFIC_FILES[workload]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2005_10445_amd.profiling import KERNEL_SOURCES, kernel_source_hash
    if t.get("kernel_source_hash") != kernel_source_hash(tuple(t.get("kernel_sources", KERNEL_SOURCES))):
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(x, chips, spc, freqs, fs, budget_s: float):
    """Direct FP64 oracle over (tag, bin) pairs of the full block until the time budget is used."""
    import numpy as np
    import oracle
    oracle.build_library(force=False)
    T, K, N = chips.shape[0], len(freqs), x.size
    done = 0
    t0 = time.perf_counter()
    for t in range(T):
        for k in range(K):
            oracle.corr_power(x, chips[t:t + 1], spc, [freqs[k]], fs)
            done += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done * N / dt / 1e6, "unit": "tag*freq*Msample/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{done} (tag, bin) pairs x {N} samples, direct FP64 correlation, {dt:.1f} s"}


def cpu_baseline_one_core(x, chips, spc, freqs, fs, budget_s: float):
    """The same oracle restricted to one thread (the paper's CPU baseline is one core):
    whole (tag, bin) pairs of the block until the budget is used."""
    import oracle
    oracle.build_library(force=False)
    cores = oracle.set_threads(1)
    try:
        out = cpu_baseline(x, chips, spc, freqs, fs, budget_s)
    finally:
        oracle.set_threads(0)
    out["cores"] = cores
    return out


def cpu_baseline_tasks(tasks, chips, spc, freqs, fs, budget_s: float):
    """Direct FP64 oracle over (task, bin) pairs of tracking tasks until the time budget is used."""
    import oracle
    oracle.build_library(force=False)
    done, samples = 0, 0
    t0 = time.perf_counter()
    for x, tag in tasks:
        for f in freqs:
            oracle.corr_power(x, chips[tag:tag + 1], spc, [f], fs)
            done += 1
            samples += x.size
            if time.perf_counter() - t0 >= budget_s:
                break
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": samples / dt / 1e6, "unit": "tag*freq*Msample/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{done} (task, bin) pairs, {samples} samples in all, direct FP64 correlation, {dt:.1f} s"}


def cpu_baseline_fsk(iq, bits, w, budget_s: float):
    """FP64 FSK oracle: the front end once, then direct correlation over slices of
    lags of successive codes until the budget is used; extrapolated to the whole
    window and every code (cost is linear in lags and codes)."""
    import numpy as np
    import siggen
    from oracle import fsk as ofsk
    fs = w["fs_hz"]
    bp = siggen.fsk_bandpass(w["bp_taps"], w["bp_cutoff_hz"], fs)
    t0 = time.perf_counter()
    d, u = ofsk.front_end(iq, fs, w["lo_hz"], bp, w["f1_hz"], w["f0_hz"], w["sps"])
    t_front = time.perf_counter() - t0
    n_t = w["num_bits"] * w["sps"] + w["bp_taps"] + w["sps"] - 2
    lags = d.size - n_t + 1
    t1 = time.perf_counter()
    done = 0
    codes = 0
    while time.perf_counter() - t1 < budget_s and codes < bits.shape[0]:
        dc = ofsk.replica_template(bits[codes], fs, bp, w["f1_hz"], w["f0_hz"], w["sps"])
        step = 4096
        for j0 in range(0, lags, step):
            j1 = min(lags, j0 + step)
            ofsk.fsk_xcorr(d[j0:j1 + n_t - 1], dc)
            done += j1 - j0
            if time.perf_counter() - t1 >= budget_s:
                break
        codes += 1
    t_corr = time.perf_counter() - t1
    per_code = t_corr / (done / lags)
    T = bits.shape[0]
    total = t_front + T * per_code
    return {"value": T * d.size / total / 1e6, "unit": "tag*freq*Msample/s", "cores": 1, "kind": "oracle",
            "sample": f"front end once ({t_front:.1f} s) + direct FP64 correlation of {done} lags "
                      f"({done / lags:.3f} codes, {t_corr:.1f} s), extrapolated to {T} codes over the window"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed ones (default 50; 1 for the batched stream, whose "
                         "steps take a second): short steps need that many before the GPU's clocks settle")
    ap.add_argument("--workload", default="tagbank_fp32")
    ap.add_argument("--fft-len", type=int, default=0, help="override the workload's segment length")
    ap.add_argument("--tag-tile", type=int, default=0)
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the plan-time autotuner (by default every launch configuration is timed once "
                         "before the timed steps and the fastest kept)")
    ap.add_argument("--graph", action="store_true", help="batched workloads: replay one captured hipGraph per step")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle time on all host cores, and half of it on one core (0: skip)")
    ap.add_argument("--legs", default="mixed,stream,learned",
                    help="tag-bank workload only: comma-separated extra legs reported in the same line "
                         "(mixed: the same block with FP16 and with BF16 storage; stream: the 64-block "
                         "batched stream, eager and graph-replayed; learned: the trained proposal network "
                         "on that stream against the exhaustive search; none)")
    ap.add_argument("--leg-steps", type=int, default=3, help="timed batches per extra leg")
    ap.add_argument("--max-fraction", type=float, default=0.5,
                    help="learned leg: full search of a block whose proposals cover more than this fraction")
    ap.add_argument("--floor-db", type=float, default=1.0,
                    help="learned leg: full search when the map median leaves the noise floor by more (dB)")
    ap.add_argument("--mode", choices=("bench", "copy"), default="bench",
                    help="copy: a plain 256 MiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the library runs on a single GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.mode == "copy":
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")   # 256 MiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4}))
        return

    import siggen
    from paper_2005_10445_amd import Plan, bin_frequencies

    w = siggen.workload(args.workload)
    if args.warmup is None:
        args.warmup = 1 if "num_blocks" in w else 50
    if "num_bits" in w:
        return bench_fsk(args, w)
    batched = "num_blocks" in w
    tracking = "num_tasks" in w
    T, C, spc, K = w["num_tags"], w["num_chips"], w["spc"], w["num_bins"]
    fs = w["fs_hz"]
    seed = w["seeds"][0]
    dev = torch.device("cuda:0")
    chips = siggen.make_codes(seed, T, C)
    prec = w.get("precision", "fp32")
    L = C * spc
    bins = dict(num_bins=K, bin_center_hz=w["bin_center_hz"], bin_step_hz=w["bin_step_hz"])
    if batched:
        fft_len = args.fft_len or w["fft_len"] or (1 << 15)
        freqs = bin_frequencies(chips=chips, spc=spc, fs_hz=fs, max_block_len=1 << 21, fft_len=fft_len, **bins)
        log(f"[bench] generating {w['num_blocks']} blocks")
        blocks = siggen.make_stream_batch(seed, chips, spc, fs, freqs, w["num_blocks"], w["block_len_log2"],
                                          w["receivers"], w["n_tx"], w["snr_db"])
        lens = [x.size for x, _ in blocks]
        xds = [torch.from_numpy(x).to(dev) for x, _ in blocks]
        plan = Plan(chips, spc, fs, max_block_len=max(lens), fft_len=fft_len, tag_tile=args.tag_tile,
                    precision=prec, refine_radius=w.get("refine_radius", 1), max_batch_blocks=len(lens),
                    max_batch_samples=sum(lens), graph=args.graph, **bins)
        x = blocks[0][0]
        run = lambda: len(plan.detect_batch(xds))      # noqa: E731
    elif tracking:
        fft_len = args.fft_len or w["fft_len"]
        L0 = C * spc
        n_task = int(math.floor(w["block_factor"] * L0))
        freqs = bin_frequencies(chips=chips, spc=spc, fs_hz=fs, max_block_len=n_task, fft_len=fft_len, **bins)
        log(f"[bench] generating {w['num_tasks']} tracking tasks")
        batch = siggen.make_tracking_batch(seed, chips, spc, fs, freqs, w["num_tasks"], w["block_factor"],
                                           w["p_present"], w["n_other"], w["snr_db"])
        lens = [xb.size for xb, _, _ in batch]
        tasks = [(torch.from_numpy(xb).to(dev), tag) for xb, tag, _ in batch]
        plan = Plan(chips, spc, fs, max_block_len=max(lens), fft_len=fft_len, precision=prec,
                    refine_radius=w.get("refine_radius", 1), max_batch_blocks=len(lens),
                    max_batch_samples=sum(lens), graph=args.graph, **bins)
        x = batch[0][0]
        task_arr = plan.task_array(tasks)
        run = lambda: plan.track_raw(task_arr)         # noqa: E731
    else:
        N = w["block_len"]
        fft_len = args.fft_len or w["fft_len"]
        plan = Plan(chips, spc, fs, max_block_len=N, fft_len=fft_len, tag_tile=args.tag_tile, precision=prec,
                    refine_radius=w.get("refine_radius", 1), **bins)
        freqs = plan.freqs_hz
        x, txs = siggen.make_block(seed, N, chips, spc, fs, freqs, w["n_tx"], snr_db=w["snr_db"])
        xd = torch.from_numpy(x).to(dev)
        lens = [N]
        run = lambda: plan.detect_raw(xd)              # noqa: E731
    g = plan.geometry
    M, V = g["fft_len"], g["valid_per_segment"]
    S = sum(-(-(n - L + 1) // V) for n in lens if n >= L)
    samples = sum(lens)
    if tracking:
        args.tune = False                              # tag tiles do not apply: one tag per task
        T_eff = 1
    else:
        T_eff = T
    if args.tune:
        table = plan.tune(xds[int(np.argmax(lens))] if batched else xd, reps=3)
        log(f"[bench] tuning table {table} -> {plan.tuning}")
    log(f"[bench] workload={args.workload} T={T} K={K} blocks={len(lens)} samples={samples} L={L} "
        f"M={M} V={V} S={S} tuning={plan.tuning}")

    for _ in range(args.warmup):
        run()
    # the FP32 detections the mixed-precision leg compares with (untimed)
    legs_req = [l for l in args.legs.split(",") if l and l != "none"] if args.workload == "tagbank_fp32" else []
    ref_dets = plan.detect(xd) if "mixed" in legs_req else None
    # one untimed step with every kernel timed gives the per-kernel figures for
    # the log; the timed steps record events around the correlation kernel
    # only (two per step)
    profiled = not ((batched or tracking) and args.graph)
    if profiled:
        plan.set_profiling(True)
        run()
        kt_all = plan.last_kernel_times()
    plan.set_profiling(profiled, correlate_only=True)
    corr_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ndet = 0
    for _ in range(args.steps):
        ndet = run()
        if profiled:
            corr_ms.append(plan.last_kernel_times()["correlate"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_profiling(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = T_eff * K * samples / (ms_per_step * 1e-3) / 1e6
    flops = correlate_flops(T_eff, K, S, M, V)
    if profiled:
        corr_avg = float(np.mean(corr_ms))
        achieved = flops / (corr_avg * 1e-3) / 1e12
        log(f"[bench] {ms_per_step:.3f} ms/step, correlate {corr_avg:.3f} ms (min {min(corr_ms):.3f}), "
            f"forward {kt_all['forward']:.3f} ms, kernels {sum(kt_all.values()):.3f} ms (one step, every kernel "
            f"timed), detections {ndet}")
        if tracking:
            log(f"[bench] {len(lens) / (ms_per_step * 1e-3):.0f} tracking tasks/s")
    else:
        corr_avg, achieved = None, None
        log(f"[bench] {ms_per_step:.3f} ms/step (graph replays, no per-kernel events), detections {ndet}")

    out = {
        "metric": "acquisition tag*freq*Msample/s",
        "value": value,
        "unit": "tag*freq*Msample/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else f"f32 ({prec} storage)",
        "data": "synthetic (seeded BPSK tags in AWGN)",
        "config": {"workload": args.workload, "tags": T, "bins": K, "blocks": len(lens), "samples": samples,
                   "tags_per_block": T_eff,
                   "template_len": L, "fft_len": M, "segments": S, "precision": prec, "tuning": plan.tuning,
                   "graph": bool((batched or tracking) and args.graph), "parallelism": "single GPU"},
        "roofline": roofline(achieved, corr_avg, flops, traffic_per_launch(args.workload)),
        "device": device_info(),
    }
    if corr_ms:
        out["roofline"]["kernel_ms_stats"] = {"min": float(np.min(corr_ms)), "median": float(np.median(corr_ms)),
                                              "max": float(np.max(corr_ms)), "launches": len(corr_ms)}
    plan.close()
    if args.workload == "tagbank_fp32":
        legs = legs_req
        if "mixed" in legs:
            out["mixed"] = mixed_leg(args, dev, xd, chips, ref_dets)
        legs = [l for l in legs if l != "mixed"]
        if legs:
            out.update(bench_stream_legs(args, legs, dev))
    if args.cpu_budget > 0:
        log("[bench] cpu baseline ...")
        if tracking:
            out["cpu_baseline"] = cpu_baseline_tasks([(xb, tag) for xb, tag, _ in batch], chips, spc, freqs, fs,
                                                     args.cpu_budget)
        else:
            out["cpu_baseline"] = cpu_baseline(x, chips, spc, freqs, fs, args.cpu_budget)
            log("[bench] cpu baseline, one core ...")
            out["cpu_baseline"]["one_core"] = cpu_baseline_one_core(x, chips, spc, freqs, fs, 0.5 * args.cpu_budget)
    print(json.dumps(out), flush=True)


def roofline(achieved, kernel_ms, flops, traffic):
    """Roofline record of the correlation kernel: FP32 vector peak, plus the fraction of
    the rate the kernel's unpacked FP32 arithmetic can reach (one FMA per lane per cycle,
    half the packed peak) and the HBM fraction of its counted traffic."""
    hbm = traffic / (kernel_ms * 1e-3) / 1e9 if traffic and kernel_ms else None
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS if achieved else None, "traffic": traffic,
            "kernel": "k_correlate", "kernel_ms": kernel_ms, "flops_per_launch": flops,
            "frac_unpacked_peak": achieved / (0.5 * PEAK_FP32_TFLOPS) if achieved else None,
            "hbm_gbs": hbm, "hbm_frac": hbm / PEAK_HBM_GBS if hbm else None}


def device_info():
    """The GPU and the ROCm build the numbers were taken on."""
    import torch
    props = torch.cuda.get_device_properties(0)
    return {"name": torch.cuda.get_device_name(0), "arch": getattr(props, "gcnArchName", None),
            "compute_units": props.multi_processor_count, "hbm_gib": round(props.total_memory / 2**30, 1),
            "hip": torch.version.hip, "torch": torch.__version__}


def _gpu_ms(fn, steps):
    """Mean wall time (ms) of fn over `steps` calls after one untimed call, each call
    bracketed by device synchronisations; returns (ms, last result)."""
    import torch
    r = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, r


def mixed_leg(args, dev, xd, chips, ref_dets):
    """The tag-bank block with spectra and replicas stored in FP16 and in BF16 (FP32
    arithmetic, FP64 refinement over +/-8 lags): time per step, the correlation
    kernel's rate, and the detections against those of the FP32 plan."""
    import numpy as np
    import siggen
    from paper_2005_10445_amd import Plan
    res = {}
    for name in ("tagbank_fp16", "tagbank_bf16"):
        w = siggen.workload(name)
        bins = dict(num_bins=w["num_bins"], bin_center_hz=w["bin_center_hz"], bin_step_hz=w["bin_step_hz"])
        N, M = w["block_len"], w["fft_len"]
        L = w["num_chips"] * w["spc"]
        with Plan(chips, w["spc"], w["fs_hz"], max_block_len=N, fft_len=M, precision=w["precision"],
                  refine_radius=w["refine_radius"], **bins) as plan:
            plan.tune(xd, reps=3)
            for _ in range(args.warmup):
                plan.detect_raw(xd)
            plan.set_profiling(True, correlate_only=True)
            corr = []
            torch_sync()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                plan.detect_raw(xd)
                corr.append(plan.last_kernel_times()["correlate"])
            torch_sync()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            plan.set_profiling(False)
            dets = plan.detect(xd)
            g = plan.geometry
        V = g["valid_per_segment"]
        S = -(-(N - L + 1) // V)
        T, K = chips.shape[0], w["num_bins"]
        flops = correlate_flops(T, K, S, M, V)
        corr_ms = float(np.mean(corr))
        same = [(d.tag, d.bin, d.lag) for d in dets] == [(d.tag, d.bin, d.lag) for d in ref_dets]
        res[w["precision"]] = {
            "ms_per_step": ms, "value": T * K * N / (ms * 1e-3) / 1e6, "unit": "tag*freq*Msample/s",
            "refine_radius": w["refine_radius"],
            "roofline": roofline(flops / (corr_ms * 1e-3) / 1e12, corr_ms, flops, traffic_per_launch(name)),
            "detections": len(dets), "same_detections_as_fp32": same,
            "max_toa_diff_vs_fp32": (max(abs(a.toa - b.toa) for a, b in zip(dets, ref_dets)) if same and dets
                                     else None),
        }
        log(f"[bench] {w['precision']}: {ms:.3f} ms/step, correlate {corr_ms:.3f} ms, {len(dets)} detections, "
            f"same as FP32: {same}")
    return res


def torch_sync():
    import torch
    torch.cuda.synchronize()


def bench_stream_legs(args, legs, dev):
    """Extra legs on the batched stream (64 resident blocks of log-uniform length in
    [2^18, 2^21], 256 tags x 21 bins, 0-20 transmissions each): the exhaustive batch
    search eagerly (per-kernel events) and as a replayed hipGraph, and the trained
    proposal network's batch search on the same blocks against it."""
    import numpy as np
    import torch
    import siggen
    from paper_2005_10445_amd import Plan, bin_frequencies
    w = siggen.workload("batched_stream")
    T, C, spc, K, fs = w["num_tags"], w["num_chips"], w["spc"], w["num_bins"], w["fs_hz"]
    seed = w["seeds"][0]
    chips = siggen.make_codes(seed, T, C)
    bins = dict(num_bins=K, bin_center_hz=w["bin_center_hz"], bin_step_hz=w["bin_step_hz"])
    fft_len = args.fft_len or w["fft_len"] or (1 << 15)
    freqs = bin_frequencies(chips=chips, spc=spc, fs_hz=fs, max_block_len=1 << 21, fft_len=fft_len, **bins)
    log(f"[bench] stream leg: generating {w['num_blocks']} blocks")
    blocks = siggen.make_stream_batch(seed, chips, spc, fs, freqs, w["num_blocks"], w["block_len_log2"],
                                      w["receivers"], w["n_tx"], w["snr_db"])
    lens = [x.size for x, _ in blocks]
    xds = [torch.from_numpy(x).to(dev) for x, _ in blocks]
    samples = sum(lens)
    kw = dict(max_block_len=max(lens), fft_len=fft_len, max_batch_blocks=len(lens), max_batch_samples=samples,
              **bins)
    out = {}
    eager = Plan(chips, spc, fs, **kw)
    table = eager.tune(xds[int(np.argmax(lens))], reps=2)
    tuning = eager.tuning
    log(f"[bench] stream tuning {table} -> {tuning}")
    g = eager.geometry
    L, M, V = C * spc, g["fft_len"], g["valid_per_segment"]
    S = sum(-(-(n - L + 1) // V) for n in lens if n >= L)
    eager.detect_batch(xds)
    eager.set_profiling(True)
    corr = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.leg_steps):
        full = eager.detect_batch(xds)
        corr.append(eager.last_kernel_times()["correlate"])
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / args.leg_steps
    eager.set_profiling(False)
    flops = correlate_flops(T, K, S, M, V)
    corr_ms = float(np.mean(corr))
    with Plan(chips, spc, fs, graph=True, **kw) as gp:
        gp.set_tuning(**tuning)
        ms_graph, gdets = _gpu_ms(lambda: gp.detect_batch(xds), args.leg_steps)
    key = lambda d: (d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power)   # noqa: E731
    assert sorted(map(key, gdets)) == sorted(map(key, full)), "graph replay differs from the eager batch"
    if "stream" in legs:
        out["stream"] = {
            "workload": "batched_stream", "tags": T, "bins": K, "blocks": len(lens), "samples": samples,
            "fft_len": M, "segments": S, "tuning": tuning,
            "ms_per_batch_eager": ms_eager, "ms_per_batch_graph": ms_graph,
            "value_graph": T * K * samples / (ms_graph * 1e-3) / 1e6,
            "value_eager": T * K * samples / (ms_eager * 1e-3) / 1e6, "unit": "tag*freq*Msample/s",
            "detections": len(full),
            "roofline": roofline(flops / (corr_ms * 1e-3) / 1e12, corr_ms, flops,
                                 traffic_per_launch("batched_stream")),
        }
        log(f"[bench] stream: eager {ms_eager:.1f} ms, graph {ms_graph:.1f} ms per batch, "
            f"correlate {corr_ms:.1f} ms, {len(full)} detections")
    if "learned" in legs:
        out["learned"] = learned_leg(args, eager, xds, blocks, full, ms_eager)
    eager.close()
    return out


def learned_leg(args, plan, xds, blocks, full, ms_exhaustive):
    """The committed trained network and its calibrated kappa on the stream batch:
    detections must be a subset of the exhaustive ones; recall is over the exhaustive
    detections of injected transmissions and over all of them."""
    import numpy as np
    from paper_2005_10445_amd.proposals import LearnedParams, Network, num_params
    wdir = os.path.join(ROOT, "paper_2005_10445_amd", "weights")
    params = np.load(os.path.join(wdir, "proposal_cnn.npy"), allow_pickle=False)
    with open(os.path.join(wdir, "proposal_cnn.json")) as f:
        kappa = float(json.load(f)["kappa"])
    assert params.size == num_params(256)
    lp = LearnedParams(kappa=kappa, max_fraction=args.max_fraction, floor_db=args.floor_db)
    with Network("bf16", 256, max_rows=1 << 15, max_block_len=1 << 21) as net:
        net.set_params(params)
        ms, (dets, reps) = _gpu_ms(lambda: net.detect_batch(plan, xds, lp), args.leg_steps)
    key = lambda d: (d.block, d.tag, d.bin, d.lag, d.toa, d.peak_power, d.z)   # noqa: E731
    fk, lk = {key(d) for d in full}, {key(d) for d in dets}

    def injected(d):
        return any(d.tag == t.tag and d.bin == t.bin and abs(d.lag - t.delay) <= 2 for t in blocks[d.block][1])
    inj = [key(d) for d in full if injected(d)]
    out = {"workload": "batched_stream + proposals", "network": "4 conv1d x 64 channels, k=5, bf16",
           "kappa": kappa, "max_fraction": args.max_fraction, "floor_db": args.floor_db,
           "ms_per_batch_learned": ms, "ms_per_batch_exhaustive": ms_exhaustive,
           "speedup": ms_exhaustive / ms,
           "recall_injected": sum(k in lk for k in inj) / max(len(inj), 1), "injected_detections": len(inj),
           "recall_all": len(lk & fk) / max(len(fk), 1), "exhaustive_detections": len(fk),
           "not_in_exhaustive": len(lk - fk),
           "segments_searched": sum(r.segments for r in reps) / max(sum(r.total_segments for r in reps), 1),
           "fallbacks": sum(r.fallback != 0 for r in reps), "blocks": len(reps)}
    log(f"[bench] learned: {ms:.1f} ms vs {ms_exhaustive:.1f} ms exhaustive, recall {out['recall_injected']:.4f} "
        f"(injected) {out['recall_all']:.4f} (all), segments {out['segments_searched']:.3f}, "
        f"fallbacks {out['fallbacks']}/{len(reps)}")
    return out


def bench_fsk(args, w):
    """The FSK searching task: one acq_fsk_detect per step on a resident window."""
    import numpy as np
    import torch
    import siggen
    from paper_2005_10445_amd.fsk import FskPlan
    T, fs, N = w["num_tags"], w["fs_hz"], w["block_len"]
    seed = w["seeds"][0]
    bits = siggen.make_fsk_bits(seed, T, w["num_bits"])
    bp = siggen.fsk_bandpass(w["bp_taps"], w["bp_cutoff_hz"], fs)
    tracking = "num_tasks" in w
    if tracking:
        rng = np.random.default_rng(seed)
        tasks, txs_all = [], []
        for i in range(w["num_tasks"]):
            tag = int(rng.integers(0, T))
            present = bool(rng.random() < w["p_present"])
            iq_i, txs_i = siggen.make_fsk_block(seed + 1 + i, N, bits, w["sps"], fs, w["f1_hz"], w["f0_hz"],
                                                w["lo_hz"], 1 if present else 0, snr_db=w["snr_db"],
                                                noise_rms=w["noise_rms"], tags=[tag] if present else None)
            tasks.append((torch.from_numpy(iq_i).to("cuda:0"), tag))
            txs_all.append(txs_i)
        iq = None
        plan = FskPlan(bits, fs, w["lo_hz"], w["f1_hz"], w["f0_hz"], bp, w["sps"], N * len(tasks),
                       max_track_tasks=len(tasks))
        task_arr = plan.task_array(tasks)
        run = lambda: plan.track_raw(task_arr)         # noqa: E731
        total_samples = N * len(tasks)
    else:
        iq, txs = siggen.make_fsk_block(seed + 1, N, bits, w["sps"], fs, w["f1_hz"], w["f0_hz"], w["lo_hz"],
                                        w["n_tx"], snr_db=w["snr_db"], noise_rms=w["noise_rms"])
        x = torch.from_numpy(iq).to("cuda:0")
        plan = FskPlan(bits, fs, w["lo_hz"], w["f1_hz"], w["f0_hz"], bp, w["sps"], N)
        run = lambda: plan.detect_raw(x)               # noqa: E731
        total_samples = N
    g = plan.geometry
    M, V, n_t = g["fft_len"], g["valid_per_segment"], g["template_len"]
    S = -(-(N - n_t + 1) // V)
    slots = -(-S // 2)
    if tracking:
        slots *= len(tasks)
    log(f"[bench] workload={args.workload} codes={T} N={N} n_t={n_t} M={M} V={V} segments={S} slots={slots}")
    for _ in range(args.warmup):
        run()
    plan.set_profiling(True)
    corr_ms, kern_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
        kt = plan.last_kernel_times()
        corr_ms.append(kt["correlate"])
        kern_ms.append(kt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_profiling(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # codes x samples searched per second (tracking: one code per task)
    value = (total_samples if tracking else T * N) / (ms_per_step * 1e-3) / 1e6
    # per code and pair of segments: one M-point inverse transform + spectrum product + |c| per valid lag
    flops = float(1 if tracking else T) * slots * (5.0 * M * math.log2(M) + 6.0 * M + 4.0 * V)
    corr_avg = float(np.mean(corr_ms))
    achieved = flops / (corr_avg * 1e-3) / 1e12
    window_s = N / fs
    codes_rt = 0.5 * window_s / (ms_per_step * 1e-3 / T)      # the paper's throughput: 50% of the time searching
    mean = {k: float(np.mean([m[k] for m in kern_ms])) for k in kern_ms[0]}
    if tracking:
        found = {d.block: d for d in plan.track(tasks)}
        want = [(i, tx[0][1]) for i, tx in enumerate(txs_all) if tx]
        hits = sum(1 for i, D in want if i in found and abs(found[i].lag - D) <= 1)
        log(f"[bench] {ms_per_step:.3f} ms per {len(tasks)} tasks ({len(tasks) / (ms_per_step * 1e-3):.0f} tasks/s), "
            f"kernels {mean}, {hits}/{len(want)} packets found")
    else:
        found = plan.detect(x)
        hits = sum(1 for t, D, _ in txs if abs(found[t].lag - D) <= 1 and found[t].z > 0.02)
        log(f"[bench] {ms_per_step:.3f} ms per window, kernels {mean}, {hits}/{len(txs)} packets found, "
            f"{codes_rt:.0f} codes searchable in real time at 50% duty")
    out = {
        "metric": "acquisition tag*freq*Msample/s",
        "value": value,
        "unit": "tag*freq*Msample/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded CPFSK packets in AWGN, int16)",
        "config": {"workload": args.workload, "codes": T, "bits": w["num_bits"], "samples_per_bit": w["sps"],
                   "window_samples": N, "template_len": n_t, "fft_len": M, "segments": S,
                   "tasks": len(tasks) if tracking else None,
                   "codes_realtime_half_duty": None if tracking else codes_rt, "parallelism": "single GPU"},
        "roofline": dict(roofline(achieved, corr_avg, flops, traffic_per_launch(args.workload)),
                         kernel="k_fsk_correlate"),
        "device": device_info(),
    }
    if args.cpu_budget > 0 and not tracking:
        log("[bench] cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline_fsk(iq, bits, w, args.cpu_budget)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
