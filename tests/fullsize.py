"""Whole-workload parity at the benchmark's sizes.

The oracle runs as independent shards on several host threads: each shard
is an oracle batch keyed by its envs' global ids, and the C oracle releases
the GIL inside every ctypes call, so the shards step in parallel while each
one stays the plain single-threaded simulator.  Nothing the GPU produced is
fed to the oracle; the GPU's outputs are only compared with the oracle's.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

KEYS = ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")


def host_threads() -> int:
    """Oracle threads: the host cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - non-Linux
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def first_mismatch(got: np.ndarray, want: np.ndarray) -> str | None:
    """None if equal, else where and how the arrays first differ."""
    if got.shape != want.shape:
        return f"shape {got.shape} != {want.shape}"
    if np.array_equal(got, want):
        return None
    bad = np.argwhere(got != want)
    i = tuple(bad[0])
    return f"{len(bad)} elements differ, first at {list(i)} (gpu {got[i]}, oracle {want[i]})"


class PlainShards:
    """E envs of one plain batch as contiguous oracle shards (env_base = the
    shard's first env), stepped in parallel; compares against the GPU's
    full host-format state, observation, rewards, dones and actions."""

    def __init__(self, cfg_kw: dict, E: int, pool: ThreadPoolExecutor, n_shards: int | None = None,
                 plane_stride: int | None = None):
        n = n_shards or 4 * pool._max_workers
        self.HW = cfg_kw["H"] * cfg_kw["W"]
        self.PS = plane_stride or self.HW      # GPU observation planes of PS bytes (padded if > H*W)
        self.bounds = np.linspace(0, E, min(n, E) + 1).astype(np.int64)
        self.pool = pool
        self.cfgs = [oracle.Config(env_base=int(lo), **cfg_kw) for lo in self.bounds[:-1]]
        sizes = np.diff(self.bounds)
        self.states = list(pool.map(lambda c, k: oracle.reset(c, int(k))[0], self.cfgs, sizes))
        self.next_act: list[np.ndarray | None] = [None] * len(self.cfgs)

    def _each(self, fn):
        errs = [e for e in self.pool.map(fn, range(len(self.cfgs))) if e]
        if errs:
            raise AssertionError(errs[0])

    def check_state(self, got: dict, where: str):
        def one(i):
            lo, hi = self.bounds[i], self.bounds[i + 1]
            for k in KEYS:
                m = first_mismatch(got[k][lo:hi], self.states[i][k])
                if m:
                    return f"{where}: envs {lo}..{hi - 1} field {k}: {m}"
            return None
        self._each(one)

    def _obs_mismatch(self, got_obs: np.ndarray, i: int) -> str | None:
        """Shard i's observation against the oracle's ([E, P, 8, H, W] on the
        GPU side, or [E, P, 8, PS] with zero padding after each plane)."""
        lo, hi = self.bounds[i], self.bounds[i + 1]
        want = oracle.observe(self.cfgs[i], self.states[i])
        g = got_obs[lo:hi]
        if self.PS != self.HW:
            if g[..., self.HW:].any():
                return "nonzero plane padding"
            g = np.ascontiguousarray(g[..., :self.HW]).reshape(want.shape)
        return first_mismatch(g, want)

    def check_obs(self, got_obs: np.ndarray, where: str):
        def one(i):
            lo, hi = self.bounds[i], self.bounds[i + 1]
            m = self._obs_mismatch(got_obs, i)
            return f"{where}: observation of envs {lo}..{hi - 1}: {m}" if m else None
        self._each(one)

    def sample(self, actor_seed: int, t: int, got_actions: np.ndarray | None, where: str):
        """The oracle's draws for step t (kept as the actions of that step);
        compared with the GPU's if given."""
        def one(i):
            lo, hi = self.bounds[i], self.bounds[i + 1]
            a = oracle.sample(self.cfgs[i], self.states[i], actor_seed, t)
            self.next_act[i] = a
            if got_actions is not None:
                m = first_mismatch(got_actions[lo:hi], a)
                if m:
                    return f"{where}: actions of step {t}, envs {lo}..{hi - 1}: {m}"
            return None
        self._each(one)

    def step(self, got_rew: np.ndarray, got_done: np.ndarray, got_obs: np.ndarray, where: str):
        """One oracle step of every shard with its own draws, then the
        rewards, dones and observation compared."""
        def one(i):
            lo, hi = self.bounds[i], self.bounds[i + 1]
            r, d = oracle.step(self.cfgs[i], self.states[i], self.next_act[i])
            for name, g, w in (("rewards", got_rew[lo:hi], r), ("dones", got_done[lo:hi], d)):
                m = first_mismatch(g, w)
                if m:
                    return f"{where}: {name} of envs {lo}..{hi - 1}: {m}"
            m = self._obs_mismatch(got_obs, i)
            if m:
                return f"{where}: observation of envs {lo}..{hi - 1}: {m}"
            return None
        self._each(one)

    def n_done_episodes(self) -> int:
        return int(sum(int(s["episode"].astype(np.int64).sum()) for s in self.states))

    def env_state(self, e: int) -> dict:
        """A copy of env e's oracle state (one-env host format)."""
        i = int(np.searchsorted(self.bounds, e, side="right") - 1)
        j = e - int(self.bounds[i])
        return {k: v[j:j + 1].copy() for k, v in self.states[i].items()}


class PoolBuckets:
    """The envs of a mixed pool grouped by identical spec into oracle
    batches whose envs keep their global ids (env_base + index), stepped in
    parallel; compares against the pool's ragged outputs."""

    SPEC = ("H", "W", "mode", "P", "cities_min", "cities_max", "min_general_dist")

    def __init__(self, specs: dict, common_kw: dict, seed: int, env_base: int, obs_off: np.ndarray,
                 act_off: np.ndarray, pool: ThreadPoolExecutor):
        self.pool = pool
        keys = np.stack([np.asarray(specs[k], np.int64) for k in self.SPEC], 1)
        uniq, inv = np.unique(keys, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        HW = np.asarray(specs["H"], np.int64) * np.asarray(specs["W"], np.int64)
        cell_off = np.concatenate([[0], np.cumsum(HW)[:-1]])
        self.buckets = []
        for b, u in enumerate(uniq):
            idx = np.flatnonzero(inv == b)
            H, W, mode, P, cmin, cmax, dmin = (int(x) for x in u)
            cfg = oracle.Config(H=H, W=W, mode=mode, P=P, cities_min=cmin, cities_max=cmax, min_general_dist=dmin,
                                seed=seed, env_ids=(np.uint64(env_base) + idx.astype(np.uint64)), **common_kw)
            self.buckets.append({"idx": idx, "cfg": cfg, "cells": cell_off[idx], "obs": obs_off[idx].astype(np.int64),
                                 "act": act_off[idx].astype(np.int64), "HW": H * W, "PS": (H * W + 63) & ~63 if P > 2 else (H * W + 31) & ~31, "P": P})
        self.states = list(pool.map(lambda bk: oracle.reset(bk["cfg"], len(bk["idx"]))[0], self.buckets))
        self.next_act: list[np.ndarray | None] = [None] * len(self.buckets)

    def _each(self, fn):
        errs = [e for e in self.pool.map(fn, range(len(self.buckets))) if e]
        if errs:
            raise AssertionError(errs[0])

    @staticmethod
    def _rows(flat: np.ndarray, starts: np.ndarray, n: int) -> np.ndarray:
        return np.take(flat, np.add.outer(starts, np.arange(n, dtype=np.int64)))

    def _where(self, b: int) -> str:
        bk = self.buckets[b]
        c = bk["cfg"]
        return f"bucket {c.H}x{c.W} mode {c.mode} P {c.P} (envs {bk['idx'][:4].tolist()}...)"

    def check_state(self, got: dict, where: str):
        def one(b):
            bk, st = self.buckets[b], self.states[b]
            for k in ("owner", "army", "type"):
                m = first_mismatch(self._rows(got[k], bk["cells"], bk["HW"]), st[k])
                if m:
                    return f"{where}: {self._where(b)} field {k}: {m}"
            for k in ("turn", "episode", "alive", "finished"):
                m = first_mismatch(got[k][bk["idx"]], st[k])
                if m:
                    return f"{where}: {self._where(b)} field {k}: {m}"
            m = first_mismatch(got["gpos"][bk["idx"], :bk["P"]], st["gpos"])
            if m:
                return f"{where}: {self._where(b)} field gpos: {m}"
            return None
        self._each(one)

    def _obs_check(self, b: int, got_obs: np.ndarray) -> str | None:
        """Bucket b's observations: each env's block is [P][8] planes of PS
        bytes, the map's H*W bytes then zero padding."""
        bk = self.buckets[b]
        n, P, HW, PS = len(bk["idx"]), bk["P"], bk["HW"], bk["PS"]
        got = self._rows(got_obs, bk["obs"], P * 8 * PS).reshape(n, P * 8, PS)
        want = oracle.observe(bk["cfg"], self.states[b]).reshape(n, P * 8, HW)
        m = first_mismatch(got[:, :, :HW], want)
        if m:
            return f"{self._where(b)} observation: {m}"
        if PS > HW and got[:, :, HW:].any():
            return f"{self._where(b)} observation: nonzero plane padding"
        return None

    def check_obs(self, got_obs: np.ndarray, where: str):
        def one(b):
            m = self._obs_check(b, got_obs)
            return f"{where}: {m}" if m else None
        self._each(one)

    def env_state(self, e: int) -> tuple:
        """(bucket config for env e alone, a copy of its oracle state)."""
        for b, bk in enumerate(self.buckets):
            j = np.flatnonzero(bk["idx"] == e)
            if len(j):
                c = bk["cfg"]
                one = oracle.Config(**{**c.__dict__, "env_ids": c.env_ids[j[0]:j[0] + 1].copy()})
                return one, {k: v[j[0]:j[0] + 1].copy() for k, v in self.states[b].items()}
        raise KeyError(e)

    def sample(self, actor_seed: int, t: int, got_actions: np.ndarray | None, where: str):
        def one(b):
            bk = self.buckets[b]
            a = oracle.sample(bk["cfg"], self.states[b], actor_seed, t)
            self.next_act[b] = a
            if got_actions is not None:
                m = first_mismatch(self._rows(got_actions, bk["act"], bk["P"]), a)
                if m:
                    return f"{where}: {self._where(b)} actions of step {t}: {m}"
            return None
        self._each(one)

    def step(self, got_rew: np.ndarray, got_done: np.ndarray, got_obs: np.ndarray, where: str):
        def one(b):
            bk, st = self.buckets[b], self.states[b]
            r, d = oracle.step(bk["cfg"], st, self.next_act[b])
            m = first_mismatch(self._rows(got_rew, bk["act"], bk["P"]), r) or first_mismatch(got_done[bk["idx"]], d)
            if m:
                return f"{where}: {self._where(b)} rewards/dones: {m}"
            m = self._obs_check(b, got_obs)
            return f"{where}: {m}" if m else None
        self._each(one)

    def n_done_episodes(self) -> int:
        return int(sum(int(s["episode"].astype(np.int64).sum()) for s in self.states))
