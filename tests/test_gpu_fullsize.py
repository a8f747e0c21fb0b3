"""Whole-workload parity at the benchmark's sizes, in the launch
configuration bench.py times, and exhaustive 3x3 move sets through the GPU.

Every env of the 1v1 24x24 workload (65,536 envs) is compared with the
oracle for its first 200 steps, every env of the FFA-8 25x25 workload
(16,384 envs) for 100 steps and every env of the mixed 131,072-env pool for
50 steps -- full state, observation, rewards, dones and the fused actor's
next actions, bit-exact -- and then a strided env subset for the steps
after that.  The oracle runs as independent shards on the host's cores
(tests/fullsize.py); nothing the GPU produced is fed to it.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads
from tests.fullsize import KEYS, PlainShards, PoolBuckets, first_mismatch, host_threads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gen():
    import torch
    import paper_2606_23348_amd as g
    assert torch.cuda.is_available()
    g.lib()
    return g


def _subset(E, seed):
    """Every 1,024th env plus 32 seeded picks."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(0, E, 1024), rng.choice(E, 32, replace=False)]))


def _progress(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("name,steps_all,steps_total,obs_layout",
                         [("c2", 200, 500, 0), ("c3", 100, 300, 1), ("c3", 30, 60, 0)],
                         ids=["c2", "c3-padded", "c3-dense"])
def test_plain_workload_every_env(gen, name, steps_all, steps_total, obs_layout):
    """gen_step_sample (the launch bench.py times) on the full workload:
    every env every step for steps_all steps, then the strided subset."""
    import torch
    wl = workloads.PLAIN[name]
    prm = wl.params()
    E, P = wl.n_envs, wl.P
    b = gen.Batch(E, wl.H, wl.W, wl.mode, gen.make_params(wl.mode, P, obs_layout=obs_layout, **prm), seed=wl.seed)
    cfg_kw = dict(H=wl.H, W=wl.W, mode=wl.mode, P=P, seed=wl.seed,
                  **{k: v for k, v in prm.items() if k != "n_players"})
    obs_host = torch.empty(tuple(b.obs.shape), dtype=torch.uint8, pin_memory=True)
    with ThreadPoolExecutor(host_threads()) as pool:
        sh = PlainShards(cfg_kw, E, pool, plane_stride=b.PS)
        torch.cuda.synchronize()
        sh.check_state(b.get_state(), f"{name} reset")
        obs_host.copy_(b.obs)
        sh.check_obs(obs_host.numpy(), f"{name} reset")
        b.sample(wl.actor_seed, 0)
        sh.sample(wl.actor_seed, 0, b.actions.cpu().numpy(), f"{name} reset")
        for t in range(steps_all):
            where = f"{name} step {t}"
            b.step_sample(wl.actor_seed, t + 1)
            obs_host.copy_(b.obs)
            act, rew, done = b.actions.cpu().numpy(), b.rewards.cpu().numpy(), b.dones.cpu().numpy()
            sh.step(rew, done, obs_host.numpy(), where)
            sh.check_state(b.get_state(), where)
            sh.sample(wl.actor_seed, t + 1, act, where)
            if t % 50 == 49:
                _progress(f"{name}: every env equal through step {t}")
        # the strided subset for the later steps, one independent oracle run per env
        ids = _subset(E, 7)
        subs = [(oracle.Config(env_base=int(e), **cfg_kw), sh.env_state(int(e))) for e in ids]
    idx_dev = torch.from_numpy(ids).long().cuda()
    for t in range(steps_all, steps_total):
        b.step_sample(wl.actor_seed, t + 1)
        gst = b.get_envs(ids)
        gobs = b.obs[idx_dev].cpu().numpy()
        if b.padded:
            assert not gobs[..., b.H * b.W:].any(), f"{name} step {t}: nonzero plane padding"
            gobs = np.ascontiguousarray(gobs[..., :b.H * b.W]).reshape(len(ids), P, 8, wl.H, wl.W)
        gact, grew, gdone = b.actions.cpu().numpy(), b.rewards.cpu().numpy(), b.dones.cpu().numpy()
        for j, (c, s) in enumerate(subs):
            e = int(ids[j])
            where = f"{name} env {e} step {t}"
            r, d = oracle.step(c, s, oracle.sample(c, s, wl.actor_seed, t))
            assert np.array_equal(grew[e], r[0]) and gdone[e] == d[0], where
            for k in KEYS:
                m = first_mismatch(gst[k][j:j + 1], s[k])
                assert m is None, f"{where} field {k}: {m}"
            m = first_mismatch(gobs[j:j + 1], oracle.observe(c, s))
            assert m is None, f"{where} observation: {m}"
            assert np.array_equal(gact[e], oracle.sample(c, s, wl.actor_seed, t + 1)[0]), where + " next actions"


def test_pool_workload_every_env(gen):
    """The mixed 131,072-env pool stepped by a captured graph (as bench.py
    replays it): every env every step for 50 steps, then the subset."""
    import torch
    wl = workloads.C4
    steps_all, steps_total = 50, 150
    specs = workloads.mixed_specs(wl.n_envs, wl.seed)
    common_kw = dict(mountain_thresh=wl.thresh, city_army_min=wl.city_army_min, city_army_max=wl.city_army_max,
                     auto_reset=wl.auto_reset, pregrow=0)
    pl = gen.Pool(specs, gen.make_params(0, 2, **common_kw), seed=wl.seed)
    s = torch.cuda.Stream()
    obs_host = torch.empty(tuple(pl.obs.shape), dtype=torch.uint8, pin_memory=True)
    with ThreadPoolExecutor(host_threads()) as pool, torch.cuda.stream(s):
        bk = PoolBuckets(specs, common_kw, wl.seed, 0, pl.obs_off, pl.act_off, pool)
        pl.reset(actor_seed=wl.actor_seed, stream=s)
        s.synchronize()
        bk.check_state(pl.get_state(stream=s), "c4 reset")
        obs_host.copy_(pl.obs)
        bk.check_obs(obs_host.numpy(), "c4 reset")
        bk.sample(wl.actor_seed, 0, pl.actions.cpu().numpy(), "c4 reset")
        pl.capture(1, wl.actor_seed, s)
        for t in range(steps_all):
            where = f"c4 step {t}"
            pl.replay(s)
            s.synchronize()
            obs_host.copy_(pl.obs)
            act, rew, done = pl.actions.cpu().numpy(), pl.rewards.cpu().numpy(), pl.dones.cpu().numpy()
            bk.step(rew, done, obs_host.numpy(), where)
            bk.check_state(pl.get_state(stream=s), where)
            bk.sample(wl.actor_seed, t + 1, act, where)
            if t % 10 == 9:
                _progress(f"c4: every env equal through step {t}")
        ids = _subset(wl.n_envs, 8)
        subs = {int(e): bk.env_state(int(e)) for e in ids}
        for t in range(steps_all, steps_total):
            pl.replay(s)
            s.synchronize()
            obs, act = pl.obs.cpu().numpy(), pl.actions.cpu().numpy()
            rew, done = pl.rewards.cpu().numpy(), pl.dones.cpu().numpy()
            for e, (c, st) in subs.items():
                where = f"c4 env {e} step {t}"
                r, d = oracle.step(c, st, oracle.sample(c, st, wl.actor_seed, t))
                assert np.array_equal(rew[pl.env_slice(e)], r[0]) and done[e] == d[0], where
                got = pl.get_env(e, stream=s)
                for k in KEYS:
                    m = first_mismatch(got[k], st[k])
                    assert m is None, f"{where} field {k}: {m}"
                want = oracle.observe(c, st)
                got_o = gen.pool_env_obs(obs, int(pl.obs_off[e]), c.H, c.W, c.P).reshape(want.shape)
                assert np.array_equal(got_o, want), where + " observation"
                assert np.array_equal(act[pl.env_slice(e)], oracle.sample(c, st, wl.actor_seed, t + 1)[0]), where


# ------------------------------------------------------------------ 3x3 boards through the GPU
def _boards(n, seed, army_hi):
    """Random 3x3 1v1 boards: 20% mountains, two generals, every other cell
    neutral or owned by either player with 0..army_hi-1 units."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        typ = np.where(rng.random(9) < 0.2, 1, 0).astype(np.uint8)
        cells = rng.permutation(np.flatnonzero(typ == 0))
        if len(cells) < 2:
            continue
        g0, g1 = cells[:2]
        own = np.where(typ == 1, -1, rng.integers(-1, 2, 9)).astype(np.int8)
        army = np.where(typ == 1, 0, rng.integers(0, army_hi, 9)).astype(np.int32)
        if len(cells) > 2 and rng.random() < 0.3:
            typ[cells[2]] = 2                 # a castle
        typ[g0], typ[g1] = 3, 3
        own[g0], own[g1] = 0, 1
        out.append((own, army, typ, np.array([g0, g1], np.int16)))
    return out


def _legal_codes(own, army, typ, p):
    """Pass (0), one illegal code, and every code of player p's legal moves."""
    codes = [0, -3]
    for cell in range(9):
        if own[cell] != p or army[cell] <= 1:
            continue
        r, c = divmod(cell, 3)
        for k in range(1, 9):
            d = (k - 1) % 4
            rr, cc = [(r - 1, c), (r + 1, c), (r, c - 1), (r, c + 1)][d]
            if 0 <= rr < 3 and 0 <= cc < 3 and typ[rr * 3 + cc] != 1:
                codes.append(cell * 9 + k)
    return codes


def _run_boards(gen, states, actions):
    """One gen_step of every env from the given host states and actions
    (1v1 3x3, auto-reset off), against one oracle step of the same input."""
    import torch
    E = len(actions)
    cfg = oracle.Config(H=3, W=3, P=2, cities_min=0, cities_max=1, min_general_dist=1, auto_reset=0, seed=1)
    b = gen.Batch(E, 3, 3, 0, gen.make_params(0, 2, cities_min=0, cities_max=1, min_general_dist=1, auto_reset=0),
                  seed=1)
    b.set_state(states)
    b.actions.copy_(torch.from_numpy(actions))
    b.step()
    torch.cuda.synchronize()
    want = {k: v.copy() for k, v in states.items()}
    r, d = oracle.step(cfg, want, actions)
    got = b.get_state()
    for k in KEYS:
        m = first_mismatch(got[k], want[k])
        assert m is None, f"field {k}: {m}"
    assert first_mismatch(b.rewards.cpu().numpy(), r) is None
    assert first_mismatch(b.dones.cpu().numpy(), d) is None
    m = first_mismatch(b.obs.cpu().numpy(), oracle.observe(cfg, want))
    assert m is None, f"observation: {m}"
    return got, r, d


def _stack(boards, reps, turns):
    E = sum(reps)
    st = {"owner": np.zeros((E, 9), np.int8), "army": np.zeros((E, 9), np.int32), "type": np.zeros((E, 9), np.uint8),
          "turn": np.zeros(E, np.int32), "episode": np.zeros(E, np.uint32), "alive": np.full(E, 3, np.uint8),
          "finished": np.zeros(E, np.uint8), "gpos": np.zeros((E, 2), np.int16)}
    at = 0
    for (own, army, typ, gp), n, turn in zip(boards, reps, turns):
        sl = slice(at, at + n)
        st["owner"][sl], st["army"][sl], st["type"][sl], st["gpos"][sl], st["turn"][sl] = own, army, typ, gp, turn
        at += n
    return st


def test_bruteforce_3x3_single_moves_gpu():
    """Every code -1..80 of player 0 (player 1 passing) on 1,500 boards, the
    set the oracle is pinned on against the rule table of Section IV-D."""
    import paper_2606_23348_amd as gen
    from tests.test_oracle_pins import _case_table
    gen.lib()
    rng = np.random.default_rng(2024)
    boards = []
    while len(boards) < 1500:                 # the same boards as the oracle's pin
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
    st = _stack(boards, [82] * len(boards), [2] * len(boards))
    acts = np.zeros((len(boards) * 82, 2), np.int32)
    acts[:, 0] = np.tile(np.arange(-1, 81, dtype=np.int32), len(boards))
    got, rew, done = _run_boards(gen, st, acts)
    for bi, (own, army, typ, gp) in enumerate(boards):
        for j, a in enumerate(range(-1, 81)):
            e = bi * 82 + j
            eo, ea, et, alive, r, d = _case_table(own, army, typ, gp, a)
            assert (got["owner"][e] == eo).all() and (got["army"][e] == ea).all() and (got["type"][e] == et).all(), \
                (bi, a)
            assert got["alive"][e] == alive and rew[e].tolist() == r and done[e] == d, (bi, a)


@pytest.mark.parametrize("turn", [2, 3, 49])
def test_bruteforce_3x3_move_pairs_gpu(turn):
    """Every pair (pass, an illegal code or a legal move of player 0) x
    (the same for player 1) on 2,000 boards, with move priority decided by
    the turn (even and odd) and the 50-turn growth on turn 49 -> 50."""
    import paper_2606_23348_amd as gen
    gen.lib()
    boards = _boards(2000, 77 + turn, 6)
    reps, acts = [], []
    for own, army, typ, gp in boards:
        c0, c1 = _legal_codes(own, army, typ, 0), _legal_codes(own, army, typ, 1)
        pairs = np.array([(a, b) for a in c0 for b in c1], np.int32)
        reps.append(len(pairs))
        acts.append(pairs)
    st = _stack(boards, reps, [turn] * len(boards))
    _run_boards(gen, st, np.concatenate(acts))
