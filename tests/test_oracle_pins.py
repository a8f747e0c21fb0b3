"""Pins of the CPU oracle against facts outside itself (no GPU needed).

Each test ties a part of the oracle to something the paper, a library routine
or plain mathematics fixes:
  * Philox4x64-10           -> numpy.random.Philox (library)
  * Philox4x32-10           -> the generator's published known-answer vectors
  * fog of war (Sec. IV-B)  -> scipy.ndimage.binary_dilation with a 3x3 block
  * map connectivity        -> scipy.ndimage.label with the 4-neighbour cross
  * rules (Sec. IV-C..E)    -> hand-worked scenarios in tests/golden/
  * growth (Sec. IV-C)      -> closed form under all-pass play
  * random actor            -> legality by trial application + chi-square
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
from scipy import stats

import oracle
import workloads
from tests import scenarios as scn

MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------- Philox
def _numpy_block(ctr, key):
    """numpy's Philox emits the block of counter+1 first, so start one below."""
    c = (ctr[0] | (ctr[1] << 64) | (ctr[2] << 128) | (ctr[3] << 192)) - 1
    c %= 1 << 256
    words = np.array([(c >> (64 * i)) & MASK64 for i in range(4)], np.uint64)
    g = np.random.Philox(key=np.array(key, np.uint64), counter=words)
    return [int(v) for v in g.random_raw(4)]


@pytest.mark.parametrize("seed", range(6))
def test_philox_matches_numpy(seed):
    rng = np.random.default_rng(seed)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 2 ** 63, 4, dtype=np.int64)]
        if seed == 0:
            ctr = [0, 0, 0, 0]
        key = [int(x) for x in rng.integers(0, 2 ** 63, 2, dtype=np.int64)]
        assert [int(v) for v in oracle.philox(ctr, key)] == _numpy_block(ctr, key)


def test_draw_word_order():
    """Draw j = 32-bit half (low first) of 64-bit word (j/2)%4 of block j/8."""
    seed, dom, c0, c1, c2 = 77, 1, 5, 6, 7
    for j in range(40):
        blk = _numpy_block([c0, c1, c2, j // 8], [seed, dom])
        w = blk[(j // 2) % 4]
        want = w & 0xFFFFFFFF if j % 2 == 0 else w >> 32
        assert oracle.draw(seed, dom, c0, c1, c2, j) == want


def test_philox4x32_known_answers():
    """Philox4x32-10 reproduces the published known-answer vectors
    (tests/golden/philox4x32_kat.json)."""
    import json
    import os
    kat = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert [int(x) for x in oracle.philox32(ctr, key)] == [int(x, 16) for x in v["out"]]


def test_actor_draw_layout():
    """Reading R15: player p's draw is word p mod 4 of the Philox4x32-10
    block keyed by the actor seed's halves, counter (step lo, step hi, env
    lo, env hi), the counter's top bit flipped for players 4..7."""
    rng = np.random.default_rng(3)
    for _ in range(30):
        seed, env, step = (int(x) for x in rng.integers(0, 2 ** 62, 3, dtype=np.int64))
        key = [seed & 0xFFFFFFFF, seed >> 32]
        lo = oracle.philox32([step & 0xFFFFFFFF, step >> 32, env & 0xFFFFFFFF, env >> 32], key)
        hi = oracle.philox32([step & 0xFFFFFFFF, step >> 32, env & 0xFFFFFFFF, (env >> 32) ^ 0x80000000], key)
        for p in range(8):
            want = int(lo[p]) if p < 4 else int(hi[p - 4])
            assert oracle.actor_draw(seed, env, step, p) == want
    # neighbouring envs and steps get different blocks
    d = {oracle.actor_draw(9, e, t, 0) for e in range(16) for t in range(16)}
    assert len(d) == 256


# ---------------------------------------------------------------- scenarios
def _cfg_for(sc, H, W):
    return oracle.Config(H=H, W=W, mode=sc["mode"], P=sc["P"], auto_reset=sc.get("auto_reset", 0),
                         seed=sc.get("seed", 7))


@pytest.mark.parametrize("sc", scn.load(), ids=lambda s: s["name"])
def test_hand_worked_scenario(sc):
    H, W = len(sc["grid"]), len(sc["grid"][0].split())
    cfg = _cfg_for(sc, H, W)
    st = scn.initial_state(sc)
    for k, stp in enumerate(sc["steps"]):
        acts = scn.encode_actions(stp, sc["P"])
        for _ in range(stp.get("repeat", 1)):
            rew, done = oracle.step(cfg, st, acts)
        exp = stp["expect"]
        assert scn.grid_of(st, H, W) == exp["grid"], f"step {k}"
        assert int(st["turn"][0]) == exp["turn"]
        assert rew[0].tolist() == exp["rewards"]
        assert int(done[0]) == exp["done"]
        assert int(st["alive"][0]) == exp["alive"]


def test_auto_reset_starts_next_episode():
    """R13: the capturing step returns the terminal rewards and done, and the
    env state is a fresh map of episode + 1."""
    sc = next(s for s in scn.load() if s["name"] == "H6_general_capture_1v1")
    cfg = oracle.Config(H=3, W=4, mode=0, P=2, auto_reset=1, seed=11, cities_min=1, cities_max=2,
                        min_general_dist=2)
    st = scn.initial_state(sc)
    rew, done = oracle.step(cfg, st, scn.encode_actions(sc["steps"][0], 2))
    assert rew[0].tolist() == [1, -1] and done[0] == 1
    assert st["episode"][0] == 1 and st["turn"][0] == 0 and st["alive"][0] == 3
    assert st["finished"][0] == 0
    # the new map is a valid map: two generals with army 1 at gpos
    for p in range(2):
        g = st["gpos"][0, p]
        assert st["type"][0, g] == oracle.T_GENERAL and st["owner"][0, g] == p and st["army"][0, g] == 1


# ---------------------------------------------------------------- growth closed form
@pytest.mark.parametrize("T", [1, 2, 49, 50, 51, 99, 100, 257])
def test_growth_closed_form(T):
    """All players pass for T steps from turn 0: a general holds 1 + T//2, an
    owned castle a0 + T//2, an owned plain cell a0 + T//50, neutral cells keep
    their army (Section IV-C)."""
    cfg = oracle.Config(H=10, W=10, P=2, cities_min=4, cities_max=4, seed=3, auto_reset=0)
    st, _ = oracle.reset(cfg, 8)
    rng = np.random.default_rng(T)
    # hand some plain cells and one city to player 0 or 1 with random armies
    for e in range(8):
        plain = np.flatnonzero(st["type"][e] == 0)
        pick = rng.choice(plain, 5, replace=False)
        st["owner"][e, pick] = rng.integers(0, 2, 5)
        st["army"][e, pick] = rng.integers(0, 1000, 5)
        city = np.flatnonzero(st["type"][e] == 2)[0]
        st["owner"][e, city] = 1
    before = {k: v.copy() for k, v in st.items()}
    for _ in range(T):
        oracle.step(cfg, st, np.zeros((8, 2), np.int32))
    own, typ, a0 = before["owner"], before["type"], before["army"].astype(np.int64)
    want = a0.copy()
    gen_or_castle = (own >= 0) & ((typ == 3) | (typ == 2))
    plain = (own >= 0) & (typ == 0)
    want[gen_or_castle] += T // 2
    want[plain] += T // 50
    assert (st["army"] == want).all()
    assert (st["owner"] == own).all() and (st["turn"] == T).all()


# ---------------------------------------------------------------- fog and observation
def _random_states(cfg, E, seed):
    st, _ = oracle.reset(cfg, E)
    rng = np.random.default_rng(seed)
    HW = cfg.H * cfg.W
    for e in range(E):
        passable = np.flatnonzero(st["type"][e] != 1)
        k = rng.integers(0, len(passable) + 1)
        cells = rng.choice(passable, k, replace=False)
        st["owner"][e, cells] = rng.integers(-1, cfg.P, k)
        st["army"][e, cells] = rng.integers(0, 400, k)
        gens = st["gpos"][e]
        st["owner"][e, gens] = np.arange(cfg.P)
        assert HW == st["owner"].shape[1]
    return st


@pytest.mark.parametrize("mode,P,H,W", [(0, 2, 10, 10), (1, 4, 13, 11), (2, 8, 25, 25), (2, 3, 7, 19)])
def test_fog_is_moore_dilation(mode, P, H, W):
    """Section IV-B: a player sees the cells they own and their 8-neighbourhood
    (2v2: the team's cells, R10)."""
    cfg = oracle.Config(H=H, W=W, mode=mode, P=P, cities_min=2, cities_max=3,
                        min_general_dist=3, seed=5)
    st = _random_states(cfg, 12, seed=H * W)
    obs = oracle.observe(cfg, st)
    for e in range(12):
        own = st["owner"][e].reshape(H, W)
        for p in range(P):
            team = (own == p)
            if mode == 1:
                team |= (own == (p ^ 2))
            vis = ndi.binary_dilation(team, structure=np.ones((3, 3), bool))
            assert (obs[e, p, 6] == (~vis)).all()
            # channels 1..5 are zero under fog, channel 7 too
            for ch in (1, 2, 3, 4, 5, 7):
                assert (obs[e, p, ch][~vis] == 0).all()


@pytest.mark.parametrize("mode,P", [(0, 2), (1, 4), (2, 5)])
def test_obs_channel_semantics(mode, P):
    cfg = oracle.Config(H=9, W=12, mode=mode, P=P, cities_min=2, cities_max=3, min_general_dist=3, seed=9)
    st = _random_states(cfg, 10, seed=P)
    obs = oracle.observe(cfg, st)
    for e in range(10):
        own = st["owner"][e].reshape(9, 12)
        typ = st["type"][e].reshape(9, 12)
        army = st["army"][e].reshape(9, 12)
        for p in range(P):
            o = obs[e, p]
            vis = o[6] == 0
            assert (o[0] == (own == p)).all()
            assert (o[0][~vis] == 0).all()            # own cells are always visible
            assert (o[3] == (vis & (typ == 1))).all()
            assert (o[4] == (vis & (typ == 2))).all()
            assert (o[5] == (vis & (typ == 3))).all()
            assert (o[7] == np.where(vis, np.minimum(army, 255), 0)).all()
            # owned / enemy / neutral partition the visible non-mountain cells
            # (in 2v2 the ally's cells are the fourth, unlabelled class)
            s = o[0].astype(int) + o[1] + o[2]
            ally = (own == (p ^ 2)) if mode == 1 else np.zeros_like(vis)
            assert (s[vis & (typ != 1) & ~ally] == 1).all()
            assert (s[~vis | (typ == 1) | ally] == 0).all()
            assert set(np.unique(o[:7])) <= {0, 1}


# ---------------------------------------------------------------- map generator
@pytest.mark.parametrize("wl", [workloads.C1, workloads.C2, workloads.C3], ids=lambda w: w.name)
def test_mapgen_invariants(wl):
    cfg = oracle.Config(H=wl.H, W=wl.W, mode=wl.mode, P=wl.P, **{k: v for k, v in wl.params().items()
                        if k not in ("n_players",)}, seed=wl.seed)
    E = 200
    st, att = oracle.reset(cfg, E)
    assert (att < 128).all()                       # last-resort placement never needed
    cross = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    for e in range(E):
        typ = st["type"][e].reshape(wl.H, wl.W)
        own = st["owner"][e].reshape(wl.H, wl.W)
        army = st["army"][e].reshape(wl.H, wl.W)
        g = st["gpos"][e]
        lab, _ = ndi.label(typ != 1, structure=cross)
        gl = [lab.flat[c] for c in g]
        assert len(set(gl)) == 1 and gl[0] > 0       # generals share one component
        rc = np.stack([g // wl.W, g % wl.W], 1)
        for i in range(wl.P):
            assert typ.flat[g[i]] == 3 and own.flat[g[i]] == i
            for j in range(i):
                assert np.abs(rc[i] - rc[j]).sum() >= wl.min_general_dist
        cities = typ == 2
        assert wl.cities_min <= cities.sum() <= wl.cities_max
        assert ((army[cities] >= 40) & (army[cities] <= 50)).all()
        assert (own[cities] == -1).all()
        assert (own[typ == 1] == -1).all() and (army[typ == 1] == 0).all()
        plain = typ == 0
        assert (own[plain] == -1).all() and (army[plain] == 0).all()
        if wl.pregrow and e % 4 == 0:
            assert ((army.flat[g] >= 100000) & (army.flat[g] <= 1000000)).all()
        else:
            assert (army.flat[g] == 1).all()
    assert (st["turn"] == 0).all() and (st["alive"] == (1 << wl.P) - 1).all()


def test_mapgen_first_attempt_uses_philox_cells():
    """G1 and G2 of R14 re-derived from numpy's Philox: the mountain mask is
    draw(cell) < T, the first general is the pick over non-mountain cells."""
    wl = workloads.C2
    cfg = oracle.Config(H=24, W=24, P=2, mountain_thresh=wl.thresh, cities_min=8, cities_max=12,
                        min_general_dist=9, seed=2)
    st, att = oracle.reset(cfg, 24)
    HW = 24 * 24
    checked = 0
    for e in range(24):
        if att[e] != 0:
            continue
        draws = []
        for blk in range((HW + 8) // 8 + 1):
            for w in _numpy_block([e, 0, 0, blk], [2, 1]):
                draws += [w & 0xFFFFFFFF, w >> 32]
        mtn = np.array(draws[:HW]) < wl.thresh
        assert ((st["type"][e] == 1) == mtn).all()
        free = np.flatnonzero(~mtn)
        g0 = free[(draws[HW] * len(free)) >> 32]
        assert st["gpos"][e, 0] == g0
        checked += 1
    assert checked >= 20


def test_mountain_density():
    cfg = oracle.Config(H=24, W=24, P=2, cities_min=8, cities_max=12, seed=2)
    st, att = oracle.reset(cfg, 400)
    n = (st["type"][att == 0] == 1).sum()
    N = (att == 0).sum() * 576
    # first-attempt maps are conditioned on success, so allow a small bias
    assert abs(n / N - 0.2) < 0.01


# ---------------------------------------------------------------- random actor
def _legal_set(cfg, st, e, p):
    """Actions of player p that change the state when applied alone (R4):
    found by trial application of every code, with everyone else passing."""
    HW = cfg.H * cfg.W
    E1 = HW * 9
    sub = {k: np.repeat(v[e:e + 1], E1, axis=0) for k, v in st.items()}
    acts = np.zeros((E1, cfg.P), np.int32)
    acts[:, p] = np.arange(E1)
    c2 = oracle.Config(**{**cfg.__dict__, "auto_reset": 0})
    oracle.step(c2, sub, acts)
    changed = (sub["army"] != st["army"][e]).any(1) | (sub["owner"] != st["owner"][e]).any(1)
    return set(np.flatnonzero(changed).tolist())


def test_actor_samples_only_legal_moves():
    cfg = oracle.Config(H=8, W=9, P=2, cities_min=2, cities_max=3, min_general_dist=4, seed=4)
    st = _random_states(cfg, 6, seed=1)
    for step_idx in range(40):
        acts = oracle.sample(cfg, st, 99, step_idx)
        for e in range(6):
            for p in range(2):
                a = int(acts[e, p])
                if a != 0:
                    assert a in _legal_set(cfg, st, e, p)


def test_actor_is_uniform_over_legal_plus_pass():
    cfg = oracle.Config(H=6, W=7, P=2, cities_min=1, cities_max=1, min_general_dist=4, seed=8)
    st = _random_states(cfg, 1, seed=3)
    st["army"][0, st["owner"][0] == 0] = 5
    L = sorted(_legal_set(cfg, st, 0, 0) | {0})
    assert len(L) > 10
    N = 20000
    counts = {a: 0 for a in L}
    for t in range(N):
        a = int(oracle.sample(cfg, st, 12345, t)[0, 0])
        counts[a] += 1                             # KeyError would mean an illegal pick
    chi2, pval = stats.chisquare(list(counts.values()))
    assert pval > 1e-4


def test_actor_dead_player_passes():
    cfg = oracle.Config(H=6, W=6, mode=2, P=3, cities_min=1, cities_max=1, min_general_dist=3, seed=8)
    st = _random_states(cfg, 4, seed=2)
    st["alive"][:] = 0b101
    for t in range(20):
        assert (oracle.sample(cfg, st, 5, t)[:, 1] == 0).all()


# ---------------------------------------------------------------- 3x3 brute force
def _case_table(own, army, typ, gpos, a):
    """Expected single-move outcome from the rule text (Section IV-D, R4/R6-R8)
    for player 0 moving and player 1 passing, 1v1, no growth on this step."""
    own, army, typ = own.copy(), army.copy(), typ.copy()
    alive, rew, done = 3, [0, 0], 0
    if a < 0 or a >= 81 or a % 9 == 0:
        return own, army, typ, alive, rew, done
    src, k = divmod(a, 9)
    d = (k - 1) % 4
    r, c = divmod(src, 3)
    r, c = [(r - 1, c), (r + 1, c), (r, c - 1), (r, c + 1)][d]
    if not (0 <= r < 3 and 0 <= c < 3):
        return own, army, typ, alive, rew, done
    dst = r * 3 + c
    if typ[dst] == 1 or own[src] != 0 or army[src] <= 1:
        return own, army, typ, alive, rew, done
    m = army[src] // 2 if k >= 5 else army[src] - 1
    army[src] -= m
    if own[dst] == 0:
        army[dst] += m
    elif m > army[dst]:
        army[dst] = m - army[dst]
        own[dst] = 0
        if typ[dst] == 3 and dst == gpos[1]:
            for i in range(9):
                if own[i] == 1:
                    own[i] = 0
                    army[i] //= 2
            typ[dst] = 2
            alive, rew, done = 1, [1, -1], 1
    else:
        army[dst] -= m
    return own, army, typ, alive, rew, done


def test_bruteforce_3x3_single_moves():
    rng = np.random.default_rng(2024)
    boards = []
    while len(boards) < 1500:
        typ = np.where(rng.random(9) < 0.2, 1, 0).astype(np.uint8)
        cells = rng.permutation(np.flatnonzero(typ == 0))
        if len(cells) < 2:
            continue
        g0, g1 = cells[:2]
        own = np.where(typ == 1, -1, rng.integers(-1, 2, 9)).astype(np.int8)
        army = np.where(typ == 1, 0, rng.integers(0, 4, 9)).astype(np.int32)
        typ[g0], typ[g1] = 3, 3
        own[g0], own[g1] = 0, 1
        boards.append((own, army, typ, np.array([g0, g1], np.int16)))
    E = len(boards) * 82
    cfg = oracle.Config(H=3, W=3, P=2, auto_reset=0, seed=1)
    st = oracle.empty_state(cfg, E)
    acts = np.zeros((E, 2), np.int32)
    for b, (own, army, typ, gp) in enumerate(boards):
        sl = slice(b * 82, (b + 1) * 82)
        st["owner"][sl], st["army"][sl], st["type"][sl], st["gpos"][sl] = own, army, typ, gp
        acts[sl, 0] = np.arange(-1, 81)
    st["turn"][:] = 2
    st["alive"][:] = 3
    rew, done = oracle.step(cfg, st, acts)
    for b, (own, army, typ, gp) in enumerate(boards):
        for j, a in enumerate(range(-1, 81)):
            e = b * 82 + j
            eo, ea, et, alive, r, d = _case_table(own, army, typ, gp, a)
            assert (st["owner"][e] == eo).all() and (st["army"][e] == ea).all() and (st["type"][e] == et).all()
            assert st["alive"][e] == alive and rew[e].tolist() == r and done[e] == d


def test_army_parity_invariant_under_random_play():
    """With no growth and no capture in a step, combat removes 2*min(m, d)
    units and merges conserve them, so the total army drops by an even,
    non-negative amount (Section IV-D)."""
    cfg = oracle.Config(H=10, W=10, mode=2, P=4, cities_min=3, cities_max=5, min_general_dist=5, seed=6,
                        auto_reset=0)
    st, _ = oracle.reset(cfg, 64)
    for t in range(300):
        before = st["army"].astype(np.int64).sum(1)
        alive0 = st["alive"].copy()
        acts = oracle.sample(cfg, st, 3, t)
        oracle.step(cfg, st, acts)
        after = st["army"].astype(np.int64).sum(1)
        no_growth = (st["turn"] % 2 == 1)
        quiet = no_growth & (st["alive"] == alive0) & (st["finished"] == 0)
        delta = before - after
        assert (delta[quiet] >= 0).all() and (delta[quiet] % 2 == 0).all()
        assert (st["army"] >= 0).all()
        assert (st["owner"][st["type"] == 1] == -1).all()


def test_capture_invariants_ffa():
    """Section IV-E: after a general falls the victim owns nothing, its general
    cell is a castle, and it stays eliminated."""
    cfg = oracle.Config(H=8, W=8, mode=2, P=6, cities_min=1, cities_max=2, min_general_dist=3, seed=12,
                        auto_reset=0)
    st, _ = oracle.reset(cfg, 256)
    seen = 0
    for t in range(400):
        alive0 = st["alive"].copy()
        oracle.step(cfg, st, oracle.sample(cfg, st, 77, t))
        for e in np.flatnonzero(alive0 != st["alive"]):
            lost = int(alive0[e]) & ~int(st["alive"][e])
            assert int(st["alive"][e]) & ~int(alive0[e]) == 0
            for v in range(6):
                if lost >> v & 1:
                    seen += 1
                    assert not (st["owner"][e] == v).any()
                    assert st["type"][e, st["gpos"][e, v]] == 2
    assert seen > 20


def test_env_ids_key_each_env():
    """A batch whose envs carry explicit global ids behaves as separate
    batches of one env at those ids (the pool parity checks group envs of
    one shape that are scattered over the pool)."""
    ids = np.array([5, 9, 2, 700], np.uint64)
    kw = dict(H=7, W=6, mode=2, P=3, cities_min=1, cities_max=3, min_general_dist=3, seed=12, auto_reset=1)
    grouped = oracle.Config(env_ids=ids, **kw)
    st, _ = oracle.reset(grouped, len(ids))
    singles = [(oracle.Config(env_base=int(e), **kw),) for e in ids]
    sts = [oracle.reset(c[0], 1)[0] for c in singles]
    for t in range(60):
        a = oracle.sample(grouped, st, 4, t)
        r, d = oracle.step(grouped, st, a)
        for j, (c,) in enumerate(singles):
            aj = oracle.sample(c, sts[j], 4, t)
            rj, dj = oracle.step(c, sts[j], aj)
            assert np.array_equal(a[j], aj[0]) and np.array_equal(r[j], rj[0]) and d[j] == dj[0]
            for k in st:
                assert np.array_equal(st[k][j], sts[j][k][0])
    with pytest.raises(ValueError):
        oracle.reset(grouped, 3)
