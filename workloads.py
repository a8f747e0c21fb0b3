"""Seeded synthetic workloads for the Generals.io environment step.

This module only holds parameters and seeded input generators: map-generator
settings, seeds, and the per-env shape/mode mix of the pooled and served
workloads.  It contains none of the game's arithmetic, so both the CPU oracle
(tests) and the GPU library (tests, bench) can take their inputs from it.

Seeds follow one convention: map seed = workload number, actor seed =
1000 + workload number, arrival seed = 2000 + workload number.

The paper's own generator (Section IV-A) fills 20% of cells with mountains
and places 9-11 neutral castles holding 40-50 units; the workloads below use
that generator family with the densities, city counts and spawn distances
listed per workload.  No public benchmark or dataset is involved.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MODE_1V1, MODE_2V2, MODE_FFA = 0, 1, 2


def mountain_thresh(num: int, den: int) -> int:
    """32-bit threshold t such that a uniform 32-bit draw r is a mountain iff r < t."""
    return (2 ** 32 * num) // den


def players(mode: int, n_players: int = 0) -> int:
    if mode == MODE_1V1:
        return 2
    if mode == MODE_2V2:
        return 4
    return n_players


@dataclass
class Workload:
    name: str
    H: int
    W: int
    mode: int
    P: int
    n_envs: int
    steps: int
    density: tuple = (1, 5)
    cities_min: int = 9
    cities_max: int = 11
    city_army_min: int = 40
    city_army_max: int = 50
    min_general_dist: int = 9
    auto_reset: int = 1
    pregrow: int = 0
    seed: int = 0
    actor_seed: int = 0

    @property
    def thresh(self) -> int:
        return mountain_thresh(*self.density)

    def params(self) -> dict:
        """Generator parameters as keyword arguments (same names on both sides)."""
        return dict(mountain_thresh=self.thresh, cities_min=self.cities_min,
                    cities_max=self.cities_max, city_army_min=self.city_army_min,
                    city_army_max=self.city_army_max, min_general_dist=self.min_general_dist,
                    auto_reset=self.auto_reset, pregrow=self.pregrow)


# Plain step, 1v1, 16 envs on 10x10: 20% mountains, exactly 4 cities (40-50),
# generals >= 9 apart; 1,000 steps.  Small enough for the oracle in seconds.
C1 = Workload("plain-1v1-10x10-16env", 10, 10, MODE_1V1, 2, 16, 1000, (1, 5), 4, 4, 40, 50, 9,
              seed=1, actor_seed=1001)
# Plain step, 1v1, 24x24, 65,536 envs, 8-12 cities; 10,000 steps.  Headline.
C2 = Workload("plain-1v1-24x24-65536env", 24, 24, MODE_1V1, 2, 65536, 10000, (1, 5), 8, 12, 40, 50, 9,
              seed=2, actor_seed=1002)
# Plain step, FFA-8 on 25x25, 16,384 envs, 25% mountains, 12-16 cities,
# generals pairwise >= 7 apart, pre-grown generals on every 4th env; 5,000 steps.
C3 = Workload("plain-ffa8-25x25-16384env", 25, 25, MODE_FFA, 8, 16384, 5000, (1, 4), 12, 16, 40, 50, 7,
              pregrow=1, seed=3, actor_seed=1003)

PLAIN = {"c1": C1, "c2": C2, "c3": C3}


@dataclass
class EnvSpec:
    """Shape and mode of one env of a mixed pool."""
    H: int
    W: int
    mode: int
    P: int
    cities_min: int
    cities_max: int
    min_general_dist: int


@dataclass
class MixedPool:
    name: str
    n_envs: int
    steps: int
    seed: int
    actor_seed: int
    density: tuple = (1, 5)
    city_army_min: int = 40
    city_army_max: int = 50
    auto_reset: int = 1
    specs: list = field(default_factory=list)

    @property
    def thresh(self) -> int:
        return mountain_thresh(*self.density)


def mixed_specs(n_envs: int, seed: int) -> dict:
    """Per-env (H, W, mode) of the mixed pool: H, W uniform in 10..25; mode 1v1
    with probability 0.60, 2v2 0.25, FFA-4 0.15.  City count range
    floor(HW/72)..floor(HW/48) (8-12 at 24x24); spawn distance 9 for two
    players, 6 for four.  Drawn with numpy's Philox generator."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 4], np.uint64)))
    H = rng.integers(10, 26, size=n_envs, dtype=np.int32)
    W = rng.integers(10, 26, size=n_envs, dtype=np.int32)
    u = rng.integers(0, 100, size=n_envs, dtype=np.int32)
    mode = np.where(u < 60, MODE_1V1, np.where(u < 85, MODE_2V2, MODE_FFA)).astype(np.int32)
    P = np.where(mode == MODE_1V1, 2, 4).astype(np.int32)
    HW = H * W
    return {
        "H": H, "W": W, "mode": mode, "P": P,
        "cities_min": (HW // 72).astype(np.int32),
        "cities_max": (HW // 48).astype(np.int32),
        "min_general_dist": np.where(P == 2, 9, 6).astype(np.int32),
    }


# Batched persistent step over a mixed pool of 131,072 envs.
C4 = MixedPool("pool-mixed-10to25-131072env", 131072, 100, seed=4, actor_seed=1004)


@dataclass
class Served:
    name: str = "served-mixed-256streams"
    n_streams: int = 256
    groups_per_stream: int = 8
    rate_per_stream: float = 4000.0     # requests per second (Poisson)
    batch_min: int = 64
    batch_max: int = 2048
    steps_per_group: int = 1000
    hbm_budget: int = 200 * 10 ** 9
    seed: int = 5
    actor_seed: int = 1005
    arrival_seed: int = 2005


C5 = Served()


def arrival_gaps(seed: int, stream: int, n: int, rate: float) -> np.ndarray:
    """Exponential inter-arrival gaps (seconds) of one actor stream."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, stream], np.uint64)))
    return rng.exponential(1.0 / rate, size=n)


def group_sizes(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 6], np.uint64)))
    return rng.integers(lo, hi + 1, size=n, dtype=np.int32)
