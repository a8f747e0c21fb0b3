"""Pins of the oracle's official map generator (Section IV-A) and the
spawn-distance cap of the curriculum (Section V-C), reading R18.

Distances are recomputed independently with scipy's graph shortest paths
over the 4-connected non-mountain cells; the first two generator steps are
re-derived from numpy's Philox; bounds are checked for tightness over many
maps so that an off-by-one in either direction shows.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import workloads
from tests.test_oracle_pins import _numpy_block


def grid_graph(typ, H, W):
    passable = (typ.reshape(H, W) != oracle.T_MOUNTAIN)
    rows, cols = [], []
    for r in range(H):
        for c in range(W):
            if not passable[r, c]:
                continue
            for dr, dc in ((1, 0), (0, 1)):
                nr, nc = r + dr, c + dc
                if nr < H and nc < W and passable[nr, nc]:
                    rows += [r * W + c, nr * W + nc]
                    cols += [nr * W + nc, r * W + c]
    n = H * W
    return coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)).tocsr()


def bfs_from(typ, H, W, srcs):
    d = shortest_path(grid_graph(typ, H, W), unweighted=True, indices=srcs)
    return np.where(np.isinf(d), -1, d).astype(np.int64)


def official(H, W, P=2, mode=0, dmin=17, dmax=0, radius=6, seed=6, cmin=9, cmax=11):
    return oracle.Config(H=H, W=W, mode=mode, P=P, mountain_thresh=workloads.mountain_thresh(1, 5),
                         cities_min=cmin, cities_max=cmax, city_army_min=40, city_army_max=50,
                         min_general_dist=dmin, auto_reset=1, seed=seed, generator=1, max_general_dist=dmax,
                         castle_radius=radius)


def check_maps(cfg, st, att):
    H, W, P = cfg.H, cfg.W, cfg.P
    dists, nearest = [], []
    for e in range(st["turn"].shape[0]):
        if att[e] == 128:                         # deterministic last resort: no constraints hold
            continue
        typ, owner, army, gpos = st["type"][e], st["owner"][e], st["army"][e], st["gpos"][e].astype(int)
        assert np.array_equal(np.flatnonzero(typ == oracle.T_GENERAL), np.sort(gpos))
        for i, g in enumerate(gpos):
            assert owner[g] == i and army[g] == 1
        cas = np.flatnonzero(typ == oracle.T_CASTLE)
        assert cfg.cities_min <= len(cas) <= max(cfg.cities_max, P)
        assert np.all((army[cas] >= 40) & (army[cas] <= 50)) and np.all(owner[cas] == -1)
        d = bfs_from(typ, H, W, gpos)
        for i in range(P):
            for k in range(i):
                assert d[k, gpos[i]] >= cfg.min_general_dist
                if cfg.max_general_dist:
                    assert d[k, gpos[i]] <= cfg.max_general_dist
                dists.append(d[k, gpos[i]])
            dc = d[i, cas]
            dc = dc[dc >= 0]
            assert len(dc) and dc.min() <= cfg.castle_radius, f"env {e}: no castle within radius of general {i}"
            nearest.append(dc.min())
    return np.array(dists), np.array(nearest)


def test_official_1v1_23x23_constraints_and_tightness():
    cfg = official(23, 23)
    st, att = oracle.reset(cfg, 300)
    dists, nearest = check_maps(cfg, st, att)
    assert (att < 128).all()
    assert dists.min() == 17                     # the lower bound is reached, never crossed
    assert nearest.max() == 6                    # so is the castle radius
    # 20% mountains (G1 unchanged) and 9..11 castles
    frac = (st["type"] == oracle.T_MOUNTAIN).mean()
    assert 0.17 < frac < 0.21


@pytest.mark.parametrize("cap", [4, 7])
def test_curriculum_cap(cap):
    cfg = official(16, 16, dmin=1, dmax=cap, seed=7)
    st, att = oracle.reset(cfg, 300)
    dists, _ = check_maps(cfg, st, att)
    assert dists.max() == cap and dists.min() >= 1


@pytest.mark.parametrize("mode,P", [(1, 4), (2, 5)])
def test_official_multiplayer(mode, P):
    cfg = official(20, 20, P=P, mode=mode, dmin=6, seed=8)
    st, att = oracle.reset(cfg, 120)
    dists, _ = check_maps(cfg, st, att)
    assert dists.min() == 6


def test_official_first_steps_match_numpy_philox():
    """G1 (mountains) and G2 (first general) are the synthetic generator's
    first draws, re-derived from numpy's Philox: key (seed, 1), counter
    (env, episode, attempt, block)."""
    cfg = official(12, 14, dmin=5, seed=99)
    st, att = oracle.reset(cfg, 20)
    HW = cfg.H * cfg.W
    checked = 0
    for e in np.flatnonzero(att == 0):
        w = []
        for blk in range((HW + 1 + 7) // 8):
            w += _numpy_block([int(e), 0, 0, blk], [cfg.seed, oracle.D_MAPGEN])
        draws = [x & 0xFFFFFFFF if j % 2 == 0 else x >> 32 for x in w for j in (0, 1)]
        mtn = np.array([draws[c] < cfg.mountain_thresh for c in range(HW)])
        assert np.array_equal(mtn, st["type"][e] == oracle.T_MOUNTAIN)
        free = np.flatnonzero(~mtn)
        assert st["gpos"][e][0] == free[(draws[HW] * len(free)) >> 32]
        checked += 1
    assert checked > 10


def test_official_regenerates_on_autoreset():
    """Maps made by auto-resets (episode > 0) obey the same constraints."""
    cfg = official(5, 5, dmin=3, radius=4, seed=3, cmin=1, cmax=2)
    st, _ = oracle.reset(cfg, 64)
    fresh = 0
    for t in range(300):
        oracle.step(cfg, st, oracle.sample(cfg, st, 2, t))
        new = np.flatnonzero((st["turn"] == 0) & (st["episode"] > 0))
        if len(new):
            sub = {k: v[new] for k, v in st.items()}
            check_maps(cfg, sub, np.zeros(len(new), int))
            fresh += len(new)
    assert fresh > 20
