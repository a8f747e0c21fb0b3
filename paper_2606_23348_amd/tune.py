"""Packing autotuner for batched pools.

For a pool's mix of shapes and modes it times every candidate packing
(envs per workgroup, persistent grid size, work order) on a scratch copy of
the pool and keeps the fastest.  A candidate is accepted only if, from the
same reset, a few steps under it leave the state, observations, actions,
rewards and done flags bit-identical to the default packing.  Results are
cached per (GPU architecture, pool signature) in a JSON file.

    best, table = tune(specs, common, seed=4, actor_seed=1004)
    pool.set_tuning(**best)

tune_buckets() then chooses a packing per size bucket (players, 64-cell
words): envs per workgroup and one or two waves per env, each bucket's
choice timed on the whole pool, verified the same way:

    buckets, report = tune_buckets(specs, common, seed=4, actor_seed=1004, base=best)
    pool.set_buckets(buckets)
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import GenError, Pool, SPEC_FIELDS

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2606_23348_amd", "pool_tuning.json")


def candidates(n_cus: int) -> list:
    out = []
    for order in (0, 1):
        for wpg in (1, 2, 4):
            for grid in (0, 4 * n_cus, 8 * n_cus, 16 * n_cus):
                out.append({"waves_per_group": wpg, "grid": grid, "order": order})
    return out


def signature(specs: dict) -> str:
    """Histogram of (H, W, mode, P, cities, spawn distance) buckets."""
    rows = np.stack([np.asarray(specs[k], np.int64) for k in SPEC_FIELDS], axis=1)
    uniq, counts = np.unique(rows, axis=0, return_counts=True)
    h = hashlib.sha256(uniq.tobytes() + counts.tobytes()).hexdigest()[:16]
    return f"n{rows.shape[0]}-{h}"


def _run_from_reset(pool: Pool, actor_seed: int, steps: int, stream):
    pool.reset(actor_seed=actor_seed, stream=stream)
    for _ in range(steps):
        pool.step(actor_seed=actor_seed, stream=stream)


def tune(specs: dict, common=None, seed: int = 0, actor_seed: int = 1, steps: int = 10, warmup: int = 2,
         verify_steps: int = 3, cache_path: str | None = DEFAULT_CACHE, force: bool = False,
         cands: list | None = None, progress=None):
    """Returns (best tuning dict, {candidate: mean step microseconds or None}).
    progress: optional callable taking a one-line message per candidate."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    sig = signature(specs)
    key = f"{arch}/{sig}"
    if cache_path and not force and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"], cache[key]["table"]
    n_cus = torch.cuda.get_device_properties(0).multi_processor_count
    cands = cands or candidates(n_cus)
    stream = torch.cuda.current_stream()
    pool = Pool(specs, common, seed=seed)
    _run_from_reset(pool, actor_seed, verify_steps, stream)
    ref = pool.digest()
    table = {}
    best, best_us = None, float("inf")
    for c in cands:
        name = json.dumps(c, sort_keys=True)
        try:
            pool.set_tuning(**c, stream=stream)
        except GenError:
            table[name] = None                       # does not fit (LDS)
            continue
        _run_from_reset(pool, actor_seed, verify_steps, stream)
        if pool.digest() != ref:
            raise RuntimeError(f"packing {c} changed the results")
        for _ in range(warmup):
            pool.step(actor_seed=actor_seed, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            pool.step(actor_seed=actor_seed, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        table[name] = us
        if progress is not None:
            progress(f"tune {name}: {us:.1f} us")
        if us < best_us:
            best, best_us = c, us
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {"best": best, "table": table, "best_us": best_us}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best, table


BUCKET_CANDIDATES = ({"waves_per_group": 1, "waves_per_env": 1}, {"waves_per_group": 2, "waves_per_env": 1},
                     {"waves_per_group": 4, "waves_per_env": 1}, {"waves_per_group": 1, "waves_per_env": 2})


def _time_steps(pool: Pool, actor_seed: int, steps: int, warmup: int, stream) -> float:
    import torch
    for _ in range(warmup):
        pool.step(actor_seed=actor_seed, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        pool.step(actor_seed=actor_seed, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / steps


def tune_buckets(specs: dict, common=None, seed: int = 0, actor_seed: int = 1, base: dict | None = None,
                 steps: int = 20, warmup: int = 3, verify_steps: int = 3, min_envs: int = 2048,
                 min_gain: float = 0.005, cache_path: str | None = DEFAULT_CACHE, force: bool = False,
                 progress=None):
    """Per-bucket packing, chosen greedily on the whole pool: starting from
    the pool-wide packing `base`, the buckets (players, 64-cell words) with
    at least min_envs envs are visited largest first, and each keeps the
    candidate of BUCKET_CANDIDATES (envs per workgroup, one or two waves per
    env) that makes a step of the whole pool fastest, if it beats the
    current table by more than min_gain (a bucket whose packing differs from
    the others' takes a launch of its own, so the whole pool is what is
    timed).  The table is accepted only if the pool, from the same reset,
    gives bit-identical results under it and under `base`.  Returns (table,
    report) where report holds every trial's step time.  Cached per
    (architecture, pool signature, base)."""
    import torch
    base = dict(base or {"waves_per_group": 1, "grid": 0, "order": 0})
    arch = torch.cuda.get_device_properties(0).gcnArchName
    key = f"{arch}/{signature(specs)}/buckets/{json.dumps(base, sort_keys=True)}"
    if cache_path and not force and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["table"], cache[key]["report"]
    stream = torch.cuda.current_stream()
    full = Pool(specs, common, seed=seed)
    full.set_tuning(**base, stream=stream)
    full.reset(actor_seed=actor_seed, stream=stream)

    def step_us(table):
        full.set_buckets(table, stream=stream)
        return _time_steps(full, actor_seed, steps, warmup, stream)

    table = []
    cur = step_us(table)
    report = {"base": cur}
    default = {"waves_per_group": int(base["waves_per_group"]), "waves_per_env": 1}
    for b in sorted(full.buckets(), key=lambda x: -x["n_envs"]):
        if b["n_envs"] < min_envs:
            continue
        name = f"P{b['n_players']}-w{b['words']}"
        best, best_us = None, cur
        for c in BUCKET_CANDIDATES:
            if c == default:
                continue
            trial = table + [dict(n_players=b["n_players"], words=b["words"], **c)]
            try:
                us = step_us(trial)
            except GenError:
                us = None                               # does not fit (LDS)
            report[f"{name} {json.dumps(c, sort_keys=True)}"] = us
            if us is not None and us < best_us * (1.0 - min_gain):
                best, best_us = trial, us
        if best is not None:
            table, cur = best, best_us
        if progress is not None:
            progress(f"tune bucket {name} ({b['n_envs']} envs): {'kept ' + json.dumps(table[-1]) if best else 'pool-wide'}"
                     f", step {cur:.1f} us")
    report["table"] = cur
    # the table must not change any result
    full.set_buckets([], stream=stream)
    _run_from_reset(full, actor_seed, verify_steps, stream)
    ref = full.digest()
    full.set_buckets(table, stream=stream)
    _run_from_reset(full, actor_seed, verify_steps, stream)
    if full.digest() != ref:
        raise RuntimeError("the per-bucket packing changed the results")
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {"table": table, "report": report}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return table, report
