"""Autotuned far-field launch shape with a JSON cache.

The library's mhlp_plan_autotune times the far-field evaluation of a plan for
several source-split counts and keeps the fastest.  This module caches the
choice per (device, plan shape, layers, precision) in a JSON file so later
plans of the same shape skip the timing.  The cache path is
$MHLP_TUNE_CACHE, else ~/.cache/mhlp/far_tuning.json.
"""
from __future__ import annotations

import json
import os

import torch

from . import mhlp

LAYERS = {"slp": 1, "dlp": 2, "both": 3, "bie": 4, "grad": 5, "stokes": 6, "stokes_grad": 7}


def cache_path() -> str:
    return os.environ.get("MHLP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mhlp",
                                                           "far_tuning.json"))


def _key(plan: mhlp.Plan, layers: str, precision: int) -> str:
    # the compute-unit count identifies the part (the marketing name is not
    # reported reliably, e.g. under a profiler)
    dev = f"cu{torch.cuda.get_device_properties(plan.geom.device).multi_processor_count}"
    kind = "onsurf" if plan.onsurface else "targets"
    return f"{dev}|{kind}|M={plan.n_targets}|N={plan.n_sources}|alpha={plan.alpha:g}|{layers}|prec={precision}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(plan: mhlp.Plan, layers: str = "both", precision: int = mhlp.FP64, reps: int = 5,
         use_cache: bool = True, path: str | None = None, write: bool = True) -> dict:
    """Set the plan's split count from the cache or by timing; returns the record.
    path: cache file (default cache_path()); write=False never modifies it."""
    path = path or cache_path()
    key = _key(plan, layers, precision)
    cache = _load(path) if use_cache else {}
    if key in cache:
        plan.set_split(cache[key]["nsplit"])
        return dict(cache[key], cached=True)
    best, ms, table = plan.autotune(LAYERS[layers], precision, reps)
    rec = {"nsplit": best, "ms": ms, "candidates": {str(k): v for k, v in table.items()}}
    if use_cache and write:
        cache = _load(path)
        cache[key] = rec
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(rec, cached=False)
