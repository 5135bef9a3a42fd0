"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2005_10445_amd.profiling trace  <trace_dir> <out.txt> --cmd "<command>" [--last N]
  python -m paper_2005_10445_amd.profiling traffic <fetch_dir> <write_dir> <copy_fetch_dir>
         <copy_write_dir> <out.json> --kernel k_correlate --copy-bytes 268435456 --cmd "<command>"
  python -m paper_2005_10445_amd.profiling issue <pmc_dir> <out.txt> --kernel k_correlate --cmd "<command>"
  python -m paper_2005_10445_amd.profiling lds <pmc_dir> <out.txt> --cmd "<command>"

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for a plain device copy of known size, so that the reported
figure is HBM bytes per launch of the kernel.

`issue` turns SQ instruction counts (wave instructions per dispatch) into the
time the vector ALUs need to issue them: without packed FP32, a SIMD retires
16 lanes of an FP32 operation per clock, so one wave-64 VALU instruction
occupies its SIMD for 4 clocks; 256 CUs x 4 SIMDs at 2.4 GHz.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_10445_amd", "csrc")
# the correlation kernel and everything it includes from the library
KERNEL_SOURCES = ("correlate.hip", "device_common.h", "device_fft.h", "fft14.h", "storage.h", "kernels.h")
# the FSK pipeline's kernels
FSK_SOURCES = ("fsk.hip", "device_common.h", "device_fft.h", "fft14.h", "storage.h", "kernels.h")


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def counters(d: str):
    """{kernel name: {counter: [value per dispatch, in dispatch order]}} from a --pmc run."""
    out = defaultdict(lambda: defaultdict(list))
    with open(_find(d, "counter_collection.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def _pick(table, substr):
    names = [k for k in table if substr in k]
    if not names:
        raise KeyError(substr)
    return names[0]


def mean_counter(d: str, kernel_substr: str, counter: str, last: int = 0) -> float:
    """Mean of a counter over the kernel's dispatches (the last `last` ones if
    > 0: the timed steps of a run whose plan-time tuning launched others)."""
    t = counters(d)
    vals = t[_pick(t, kernel_substr)][counter]
    if last > 0:
        vals = vals[-last:]
    return sum(vals) / len(vals)


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel, copy_bytes, cmd, sources=KERNEL_SOURCES,
            last: int = 0):
    copy_name = "copyBuffer"
    f_copy = mean_counter(copy_fetch_dir, copy_name, "FETCH_SIZE")
    w_copy = mean_counter(copy_write_dir, copy_name, "WRITE_SIZE")
    f_scale = copy_bytes / f_copy          # bytes per counted KiB
    w_scale = copy_bytes / w_copy
    f_k = mean_counter(fetch_dir, kernel, "FETCH_SIZE", last)
    w_k = mean_counter(write_dir, kernel, "WRITE_SIZE", last)
    return {
        "kernel": kernel,
        "fetch_kib_counted": f_k, "write_kib_counted": w_k,
        "copy_bytes": copy_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
        "fetch_scale_bytes_per_kib": f_scale, "write_scale_bytes_per_kib": w_scale,
        "bytes_read_per_launch": f_k * f_scale, "bytes_written_per_launch": w_k * w_scale,
        "bytes_per_launch": f_k * f_scale + w_k * w_scale,
        "kernel_source_hash": kernel_source_hash(sources),
        "kernel_sources": list(sources),
        "dispatches": f"last {last}" if last > 0 else "all",
        "command": cmd,
    }


NUM_SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
VALU_CLOCKS = 4


def issue_summary(pmc_dir: str, kernel: str, cmd: str, sources=KERNEL_SOURCES, last: int = 0) -> str:
    t = counters(pmc_dir)
    name = _pick(t, kernel)
    series = {c: (v[-last:] if last > 0 else v) for c, v in sorted(t[name].items())}
    means = {c: sum(v) / len(v) for c, v in series.items()}
    n = len(next(iter(series.values())))
    lines = ["# rocprofv3 instruction counts per dispatch", f"# command: {cmd}",
             f"# kernel source hash: {kernel_source_hash(sources)} ({', '.join(sources)})",
             f"# kernel: {name.replace('void ', '')[:100]}",
             f"# dispatches: {n}" + (f" (the last {last})" if last > 0 else ""), ""]
    lines += [f"{c:24s} {v:18.0f}" for c, v in means.items()]
    if "SQ_INSTS_VALU" in means:
        ms = means["SQ_INSTS_VALU"] * VALU_CLOCKS / (NUM_SIMDS * CLOCK_HZ) * 1e3
        lines += ["", f"VALU issue time at {CLOCK_HZ / 1e9:.1f} GHz, {VALU_CLOCKS} clocks per wave instruction, "
                      f"{NUM_SIMDS} SIMDs: {ms:.3f} ms per dispatch"]
    return "\n".join(lines) + "\n"


LDS_COUNTERS = ("SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_ADDR_CONFLICT", "SQ_LDS_UNALIGNED_STALL",
                "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_LDS")


def lds_summary(pmc_dir: str, cmd: str, sources=KERNEL_SOURCES, top: int = 10) -> str:
    """Per-dispatch means of the LDS counters of every kernel that issues LDS
    instructions (the `top` with the most): instructions, cycles stalled on
    bank conflicts, on address conflicts and on unaligned accesses, and the
    cycles waves spend issuing LDS instructions, with the share of those that
    the bank conflicts add."""
    t = counters(pmc_dir)
    rows = []
    for name, cs in t.items():
        if "SQ_INSTS_LDS" not in cs or not cs["SQ_INSTS_LDS"]:
            continue
        means = {c: sum(cs[c]) / len(cs[c]) for c in LDS_COUNTERS if c in cs and cs[c]}
        if means.get("SQ_INSTS_LDS", 0.0) <= 0.0:
            continue
        short = _short(name).replace("(anonymous namespace)::", "").split("(")[0]
        rows.append((short, len(cs["SQ_INSTS_LDS"]), means))
    rows.sort(key=lambda r: -r[2]["SQ_INSTS_LDS"])
    lines = ["# rocprofv3 LDS counters per dispatch (means over each kernel's dispatches)", f"# command: {cmd}",
             f"# kernel source hash: {kernel_source_hash(sources)} ({', '.join(sources)})",
             "# columns: LDS instructions; cycles stalled on bank conflicts, address conflicts and unaligned",
             "# accesses; cycles waves spend issuing LDS instructions; bank-conflict cycles / LDS issue cycles", "",
             f"{'kernel':40s} {'disp':>5s} {'LDS inst':>11s} {'bank cfl':>11s} {'addr cfl':>10s} {'unalgn':>8s} "
             f"{'LDS issue':>12s} {'cfl/issue':>9s}"]
    for name, n, m in rows[:top]:
        act = m.get("SQ_ACTIVE_INST_LDS", 0.0)
        bank = m.get("SQ_LDS_BANK_CONFLICT", 0.0)
        share = f"{bank / act:9.3f}" if act > 0 else f"{'-':>9s}"
        lines.append(f"{name[:40]:40s} {n:5d} {m['SQ_INSTS_LDS']:11.4g} {bank:11.4g} "
                     f"{m.get('SQ_LDS_ADDR_CONFLICT', 0.0):10.4g} {m.get('SQ_LDS_UNALIGNED_STALL', 0.0):8.4g} "
                     f"{act:12.4g} {share}")
    return "\n".join(lines) + "\n"


def timed_dispatches(trace_dir: str, skip_steps: int, steps_total: int):
    """{kernel: [duration ns]} of the dispatches of the timed steps: a kernel
    launched c times over steps_total steps runs c // steps_total times per step,
    so its first skip_steps * (c // steps_total) dispatches are the warm-up."""
    with open(_find(trace_dir, "kernel_trace.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    calls = defaultdict(int)
    for r in rows:
        calls[r["Kernel_Name"]] += 1
    out = defaultdict(list)
    seen = defaultdict(int)
    for r in rows:
        name = r["Kernel_Name"]
        if calls[name] < steps_total:
            continue                                  # plan-time or occasional kernels
        seen[name] += 1
        if seen[name] > skip_steps * (calls[name] // steps_total):
            out[name].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def last_dispatches(trace_dir: str, n: int, anchor: str = "k_correlate"):
    """{kernel: [duration ns]} of the dispatches in the timed steps of a run
    whose plan-time tuning launched the same kernels before them: the window
    opens at the n-th last dispatch of the anchor kernel (of the kernels whose
    name contains `anchor`, the one launched last) and runs to the end."""
    with open(_find(trace_dir, "kernel_trace.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    starts = defaultdict(list)
    for r in rows:
        starts[r["Kernel_Name"]].append(int(r["Start_Timestamp"]))
    cands = [k for k in starts if anchor in k and len(starts[k]) >= n]
    if not cands:
        raise KeyError(anchor)
    key = max(cands, key=lambda k: starts[k][-1])
    t0 = starts[key][-n]
    out = defaultdict(list)
    for r in rows:
        if int(r["Start_Timestamp"]) >= t0:
            out[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def _short(name: str) -> str:
    return name.replace("void ", "").replace("acq::(anonymous namespace)::", "").replace("acq::", "")


def trace_summary(trace_dir: str, cmd: str, top: int = 12, sources=KERNEL_SOURCES, skip: int = 0,
                  steps_total: int = 0, last: int = 0) -> str:
    path = _find(trace_dir, "kernel_stats.csv")
    with open(path) as f:
        rows = list(csv.DictReader(f))
    lines = [f"# rocprofv3 kernel trace summary", f"# command: {cmd}",
             f"# kernel source hash: {kernel_source_hash(sources)} ({', '.join(sources)})", "",
             f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    for r in rows[:top]:
        name = _short(r["Name"])[:60]
        lines.append(f"{name:60s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):6.2f}")
    if last > 0:
        timed = last_dispatches(trace_dir, last)
        lines += ["", f"# timed steps only: from the {last}-th last dispatch of the correlation kernel on",
                  f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}"]
        for name, d in sorted(timed.items(), key=lambda kv: -sum(kv[1]))[:top]:
            lines.append(f"{_short(name)[:60]:60s} {len(d):6d} {sum(d) / len(d) / 1e3:10.2f} "
                         f"{min(d) / 1e3:10.2f} {max(d) / 1e3:10.2f}")
    elif skip > 0 and steps_total > skip:
        timed = timed_dispatches(trace_dir, skip, steps_total)
        lines += ["", f"# timed steps only: {steps_total - skip} of {steps_total} steps, the first {skip} "
                      f"(warm-up) left out",
                  f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}"]
        for name, d in sorted(timed.items(), key=lambda kv: -sum(kv[1]))[:top]:
            lines.append(f"{_short(name)[:60]:60s} {len(d):6d} {sum(d) / len(d) / 1e3:10.2f} "
                         f"{min(d) / 1e3:10.2f} {max(d) / 1e3:10.2f}")
    return "\n".join(lines) + "\n"


PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP32_VALU_TFLOPS = 157.3


def learned_summary(trace_dir: str, cmd: str, batch: int, block_len: int, steps_total: int, warmup: int) -> str:
    """Per-step kernel times of proposal-network training steps (the timed steps
    after `warmup`) with algorithmic FLOP rates: convolutions (4 layers, 5 taps,
    256 -> 64 -> 64 -> 64 -> 64 channels) against the bf16 MFMA peak, the STFT
    (256-point transform per frame, 5 N log2 N) against the FP32 vector peak."""
    frames = (block_len - 256) // 128 + 1
    rows = batch * frames
    conv_macs = rows * 64 * 5 * (256 + 3 * 64)          # all layers, forward
    flops = {
        "k_conv_tile<true>": (2.0 * conv_macs, PEAK_BF16_MFMA_TFLOPS, "forward, 4 layers"),
        "k_conv_tile<false>": (2.0 * rows * 64 * 5 * 64 * 3, PEAK_BF16_MFMA_TFLOPS, "input gradient, layers 1-3"),
        "k_conv_dw_taps<1>": (2.0 * rows * 64 * 5 * 256, PEAK_BF16_MFMA_TFLOPS, "weight gradient, layer 0 (d = 1)"),
        "k_conv_dw_taps<2>": (2.0 * rows * 64 * 5 * 64, PEAK_BF16_MFMA_TFLOPS, "weight gradient, layer 1 (d = 2)"),
        "k_conv_dw_taps<4>": (2.0 * rows * 64 * 5 * 64, PEAK_BF16_MFMA_TFLOPS, "weight gradient, layer 2 (d = 4)"),
        "k_conv_dw_taps<8>": (2.0 * rows * 64 * 5 * 64, PEAK_BF16_MFMA_TFLOPS, "weight gradient, layer 3 (d = 8)"),
        "k_head": (6.0 * rows * 64, PEAK_FP32_VALU_TFLOPS, "head forward + backward"),
        "k_stft": (rows * (5.0 * 256 * 8 + 8.0 * 256), PEAK_FP32_VALU_TFLOPS, "generator + window + 256-point FFT + |X|^2"),
    }
    timed = timed_dispatches(trace_dir, warmup, steps_total)
    steps = steps_total - warmup
    per_step = {name: sum(d) / steps / 1e3 for name, d in timed.items()}       # microseconds
    total = sum(per_step.values())
    lines = ["# rocprofv3 kernel trace of proposal-network training (per step, timed steps only)",
             f"# command: {cmd}",
             f"# kernel source hash: {kernel_source_hash(('learned_kernels.hip', 'learned.h', 'cnn.hip'))} "
             f"(learned_kernels.hip, learned.h, cnn.hip)",
             f"# batch {batch} blocks of {block_len} samples: {frames} frames each, {rows} rows per step; "
             f"{steps} timed steps after {warmup} warm-up",
             "", f"{'kernel':44s} {'calls/step':>10s} {'us/step':>9s} {'share':>6s} {'GFLOP':>8s} {'TFLOP/s':>8s} "
             f"{'of peak':>8s}  work"]
    for name, us in sorted(per_step.items(), key=lambda kv: -kv[1]):
        short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1]
        calls = len(timed[name]) / steps
        f = next((v for k, v in flops.items() if short.startswith(k)), None)
        if f:
            tf = f[0] / (us * 1e-6) / 1e12
            lines.append(f"{short:44s} {calls:10.0f} {us:9.1f} {us / total:6.1%} {f[0] / 1e9:8.2f} "
                         f"{tf:8.1f} {tf / f[1]:8.2%}  {f[2]} (peak {f[1]:.0f} TFLOP/s)")
        else:
            lines.append(f"{short:44s} {calls:10.0f} {us:9.1f} {us / total:6.1%}")
    lines.append(f"{'total':44s} {'':10s} {total:9.1f}")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("trace_dir")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    t.add_argument("--fsk", action="store_true", help="hash the FSK pipeline's sources")
    t.add_argument("--warmup", type=int, default=0, help="warm-up steps of the profiled run")
    t.add_argument("--steps-total", type=int, default=0, help="warm-up plus timed steps of the profiled run")
    t.add_argument("--last", type=int, default=0, help="also list each kernel's last N dispatches (timed steps "
                                                       "after plan-time tuning)")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("copy_fetch_dir")
    c.add_argument("copy_write_dir")
    c.add_argument("out")
    c.add_argument("--kernel", default="k_correlate")
    c.add_argument("--copy-bytes", type=int, default=256 << 20)
    c.add_argument("--cmd", required=True)
    c.add_argument("--fsk", action="store_true", help="hash the FSK pipeline's sources")
    c.add_argument("--last", type=int, default=0, help="average only the kernel's last N dispatches")
    i = sub.add_parser("issue")
    i.add_argument("pmc_dir")
    i.add_argument("out")
    i.add_argument("--kernel", default="k_correlate")
    i.add_argument("--cmd", required=True)
    i.add_argument("--fsk", action="store_true", help="hash the FSK pipeline's sources")
    i.add_argument("--last", type=int, default=0, help="average only the kernel's last N dispatches")
    ld = sub.add_parser("lds")
    ld.add_argument("pmc_dir")
    ld.add_argument("out")
    ld.add_argument("--cmd", required=True)
    ld.add_argument("--fsk", action="store_true", help="hash the FSK pipeline's sources")
    ls = sub.add_parser("learned")
    ls.add_argument("trace_dir")
    ls.add_argument("out")
    ls.add_argument("--cmd", required=True)
    ls.add_argument("--batch", type=int, default=8)
    ls.add_argument("--block-len", type=int, default=1 << 20)
    ls.add_argument("--warmup", type=int, default=10)
    ls.add_argument("--steps-total", type=int, default=100)
    a = ap.parse_args(argv)
    if a.what == "lds":
        with open(a.out, "w") as f:
            f.write(lds_summary(a.pmc_dir, a.cmd, sources=FSK_SOURCES if a.fsk else KERNEL_SOURCES))
        print(open(a.out).read())
        return
    if a.what == "learned":
        with open(a.out, "w") as f:
            f.write(learned_summary(a.trace_dir, a.cmd, a.batch, a.block_len, a.steps_total, a.warmup))
        print(open(a.out).read())
        return
    if a.what == "issue":
        with open(a.out, "w") as f:
            f.write(issue_summary(a.pmc_dir, a.kernel, a.cmd, sources=FSK_SOURCES if a.fsk else KERNEL_SOURCES,
                                  last=a.last))
    elif a.what == "trace":
        with open(a.out, "w") as f:
            f.write(trace_summary(a.trace_dir, a.cmd, sources=FSK_SOURCES if a.fsk else KERNEL_SOURCES,
                                  skip=a.warmup, steps_total=a.steps_total, last=a.last))
    else:
        res = traffic(a.fetch_dir, a.write_dir, a.copy_fetch_dir, a.copy_write_dir, a.kernel,
                      a.copy_bytes, a.cmd, sources=FSK_SOURCES if a.fsk else KERNEL_SOURCES, last=a.last)
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
            f.write("\n")
    print(open(a.out).read())


if __name__ == "__main__":
    main()
