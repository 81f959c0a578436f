"""Autotuner for the sweep's execution tiling.

Candidates: for single systems the stage pipeline ("stage", one kernel per
stage) and the batched stage pipeline ("batch", 2, 3, 4, 8 or 16 stages
tried per kernel); for all, the graph-captured persistent launch with 1, 2,
4 or 8 active cells per 16-lane trial group per stage (which sets the number
of workgroups per replica).  Results do not depend on the choice: every
candidate produces the same chain, so the sweeps made while tuning are real
sweeps of the chain.  The winner is cached in a JSON file keyed by the GPU
architecture, the problem shape (replicas, sites and active cells per stage,
bucketed to powers of two) and the operating point the caller names: the
batched pipeline's cost depends on how often stages are accepted, which
depends on (dmu0, kappa, cbar, T).
"""
from __future__ import annotations

import json
import math
import os

CACHE = os.environ.get("VCSGC_TUNING_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "vcsgc_tuning.json"))
TPG = (1, 2, 4, 8)
BATCH = (2, 3, 4, 8, 16)


def cache_key(arch, n_rep, n_sites, cells_per_stage, op=None):
    """The cache key: architecture, replicas, sites and active cells per
    stage bucketed to powers of two, and the operating point (6 significant
    digits each) when given."""
    b = lambda v: int(2 ** round(math.log2(max(1, v))))  # noqa: E731
    key = f"{arch}|R{n_rep}|N{b(n_sites)}|C{b(cells_per_stage)}"
    if op is not None:
        key += "|op" + ",".join(f"{float(v):.6g}" for v in op)
    return key


def _key(ctx, op):
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    info = ctx.info()
    ncpc = int(info["n_cells"][0] * info["n_cells"][1] * info["n_cells"][2]) // 8
    return cache_key(arch, getattr(ctx, "n_rep", 1), ctx.n, ncpc, op)


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(tab):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(tab, f, indent=1)
    except OSError:
        pass


def tune(ctx, sweep_fn, op=None, sweeps_per_candidate=4, use_cache=True):
    """Pick the fastest tiling for ctx.  sweep_fn(n) runs n sweeps on ctx with
    the caller's parameters (and no statistics read-back); op names the
    operating point for the cache key (e.g. (dmu0, kappa, cbar, T); None: not
    keyed).  Returns {"choice": (strategy, tpg), "times_ms": {...},
    "cached": bool}."""
    import torch
    key = _key(ctx, op)
    tab = _load() if use_cache else {}
    if key in tab:
        s, t = tab[key]["choice"]
        ctx.set_tuning(s, t)
        return {"choice": (s, t), "times_ms": tab[key]["times_ms"], "cached": True, "key": key}
    cands = [("graph", t) for t in TPG]
    if getattr(ctx, "n_rep", 1) == 1:
        cands = [("stage", 1)] + [("batch", b) for b in BATCH] + cands
    times = {}
    for s, t in cands:
        ctx.set_tuning(s, t)
        sweep_fn(1)  # first use builds the graph
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        sweep_fn(sweeps_per_candidate)
        b.record()
        torch.cuda.synchronize()
        times[f"{s}:{t}"] = a.elapsed_time(b) / sweeps_per_candidate
    best = min(times, key=times.get)
    s, t = best.split(":")
    ctx.set_tuning(s, int(t))
    if use_cache:
        tab[key] = {"choice": [s, int(t)], "times_ms": times}
        _store(tab)
    return {"choice": (s, int(t)), "times_ms": times, "cached": False, "key": key}
