"""bench.py's output contract: one JSON line with the metric, the whole-job
value, the timing fields, the roofline record of the dominant kernel and the
CPU oracle baseline; and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2", timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_json_line_contract():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = _run("--steps", "3", "--warmup", "1", "--legs", "none", "--cpu-budget", "0.5")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert d["metric"] == "acquisition tag*freq*Msample/s" and d["unit"] == "tag*freq*Msample/s"
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["scaling"] == "weak" and d["vs_baseline"] is None
    assert d["dtype"] == "f32" and d["data"].startswith("synthetic")
    assert d["config"]["workload"] == "tagbank_fp32"
    # value: tags x bins x samples per step over the step time
    c = d["config"]
    expect = c["tags"] * c["bins"] * c["samples"] / (d["ms_per_step"] * 1e-3) / 1e6
    assert abs(d["value"] - expect) <= 1e-9 * expect
    rf = d["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 157.3
    assert rf["kernel"] == "k_correlate" and 0.0 < rf["frac"] < 1.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-12
    assert abs(rf["achieved"] - rf["flops_per_launch"] / (rf["kernel_ms"] * 1e-3) / 1e12) <= 1e-9 * rf["achieved"]
    assert rf["kernel_ms"] < d["ms_per_step"]
    assert rf["traffic"] is None or rf["traffic"] > 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == d["unit"] and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["one_core"]["cores"] == 1 and cb["one_core"]["value"] > 0
    assert "device" in d and d["device"]["compute_units"] > 0
