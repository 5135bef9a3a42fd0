"""Autotuning cache for acquisition plans.

`acq_tune` (in the library) times every candidate launch configuration of the
correlation kernel -- transform engine and tags per work item -- on a sample
block and keeps the fastest.  This module remembers the winner per shape and
device in a JSON file (ACQ_TUNE_CACHE, default ~/.cache/acq_tune.json) so that
later plans of the same shape skip the timing runs.  Tuning never changes
results: every candidate computes the same correlation.
"""
from __future__ import annotations

import json
import os
from typing import Optional


def cache_path() -> str:
    return os.environ.get("ACQ_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "acq_tune.json")


def shape_key(plan) -> str:
    import torch
    g = plan.geometry
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return (f"T{plan.num_tags}_C{plan.num_chips}_spc{plan.spc}_K{plan.num_bins}_M{g['fft_len']}"
            f"_{plan.precision}_{dev}_hip{torch.version.hip}")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(plan, sample_block, reps: int = 3, path: Optional[str] = None, force: bool = False) -> dict:
    """Apply the cached tuning for the plan's shape, or measure, apply and cache it."""
    path = path or cache_path()
    key = shape_key(plan)
    cache = _load(path)
    if not force and key in cache:
        t = cache[key]
        plan.set_tuning(t["engine"], t["tag_tile"], t.get("batch_launch", 0))
        return {"key": key, "cached": True, **t}
    table = plan.tune(sample_block, reps=reps)
    best = plan.tuning
    entry = {**best, "table": table}
    cache[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    return {"key": key, "cached": False, **entry}
