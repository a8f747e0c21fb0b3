"""Parity of the 38-channel features (gen_features, Appendix A) and the two
temporal tokens (Section V-A) with the CPU oracle, through the C ABI.

Both sides step their own copy of the game with the same seeds (state parity
itself is covered by test_gpu_parity) and record features after the reset
and after the steps the case selects.  The tolerance comes from the
arithmetic: every channel is an exact integer, a 0/1 mask or a value computed
in double and rounded once to float32 (15, 22, 23: a division, correctly
rounded on both sides) or, for channel 21, log1p in double divided by 5
and rounded once, which the library takes from a table its host code fills
with the host C library's log1p (the oracle calls the same function), so
every channel must match bit for bit.  The tokens are integers converted to
float32: bit-exact.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
AGE = 21


@pytest.fixture(scope="module")
def gen():
    import torch
    import paper_2606_23348_amd as g
    assert torch.cuda.is_available()
    g.lib()
    return g


def assert_features_equal(got, want, where):
    """got, want: float32 [..., 38, H, W], compared bit for bit."""
    assert got.shape == want.shape, where
    g, w = got.view(np.int32), want.view(np.int32)
    if not np.array_equal(g, w):
        bad = np.argwhere(g != w)
        idx = tuple(bad[0])
        raise AssertionError(f"{where}: {len(bad)} values differ, first at {bad[:4].tolist()} "
                             f"(gpu {got[idx]}, oracle {want[idx]})")


def run_case(gen, H, W, mode, P, E, steps, seed, actor_seed, prm, record_every=1, repeat_at=()):
    import torch
    params = gen.make_params(mode, P, **prm)
    b = gen.Batch(E, H, W, mode, params, seed=seed)
    cfg = oracle.Config(H=H, W=W, mode=mode, P=P, seed=seed, env_base=0, **prm)
    ost, _ = oracle.reset(cfg, E)
    mem = oracle.feature_memory(E)
    b.sample(actor_seed, 0)
    n_done = 0
    for t in range(steps + 1):
        if t % record_every == 0:
            b.features(tokens=True)
            torch.cuda.synchronize()
            want, wtok = oracle.features(cfg, ost, mem, tokens=True)
            where = f"{H}x{W} mode {mode} P {P} turn-step {t}"
            assert_features_equal(b.feat.cpu().numpy(), want, where)
            assert np.array_equal(b.tokens.cpu().numpy(), wtok), where + " tokens"
            if t in repeat_at:                      # a second call on the same state changes nothing
                b.features(tokens=True)
                torch.cuda.synchronize()
                assert_features_equal(b.feat.cpu().numpy(), want, where + " (repeated)")
                assert np.array_equal(b.tokens.cpu().numpy(), wtok), where + " tokens (repeated)"
        if t == steps:
            break
        b.step_sample(actor_seed, t + 1)
        _, od = oracle.step(cfg, ost, oracle.sample(cfg, ost, actor_seed, t))
        n_done += int(od.sum())
    return n_done


def prm_for(H, W, **over):
    p = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=min(2, H * W // 8),
             cities_max=min(6, H * W // 4), min_general_dist=min(5, (H + W) // 3), auto_reset=1)
    p.update(over)
    return p


@pytest.mark.parametrize("H,W,mode,P,E,steps", [
    (24, 24, 0, 2, 12, 120),     # the 1v1 benchmark shape
    (10, 10, 1, 4, 16, 150),     # 2v2: team vision, two enemies
    (25, 25, 2, 8, 6, 80),       # FFA-8, 625 cells (ragged last wave)
    (7, 9, 2, 3, 20, 150),
    (3, 3, 0, 2, 16, 60),        # smallest grid
    (32, 32, 2, 4, 4, 60),       # largest grid
    (17, 6, 2, 6, 10, 100),
])
def test_features_trajectory(gen, H, W, mode, P, E, steps):
    run_case(gen, H, W, mode, P, E, steps, seed=H * 31 + W, actor_seed=5, prm=prm_for(H, W), repeat_at=(0, 7, 40))


@pytest.mark.parametrize("E,H,W,mode,P", [
    (1024, 24, 23, 0, 2),        # 8 waves per env, 552 cells: a ragged second round of 512
    (1500, 16, 17, 1, 4),        # 2 waves, 272 cells over rounds of 128
    (2048, 5, 13, 0, 2),         # 2 waves, 65 cells: the second wave has one
    (3000, 13, 11, 0, 2),        # 4 waves, 143 cells: the last wave has none
    (4097, 9, 7, 1, 4),          # 4 waves, 63 cells: only the first has any
    (2000, 7, 9, 2, 6),          # more than 4 players: 8 waves at any batch size
    (4100, 10, 10, 2, 8),
])
def test_features_waves_per_env(gen, E, H, W, mode, P):
    """Each env's cells are spread over 8 waves for batches of at most 1,024
    envs or more than 4 players, else over 2 (at most 2,048 envs) or 4:
    every split, with waves that own no cell, against the oracle."""
    run_case(gen, H, W, mode, P, E, 12, seed=E, actor_seed=3, prm=prm_for(H, W), record_every=4)


def test_features_skipped_recordings(gen):
    """Features recorded every third step on both sides: the turns in between
    are empty boards in the delta stacks."""
    run_case(gen, 12, 12, 0, 2, 16, 90, seed=4, actor_seed=6, prm=prm_for(12, 12), record_every=3)


def test_features_many_episodes(gen):
    """Small FFA maps end often under random play: each auto-reset starts a
    fresh memory in the same call."""
    prm = prm_for(4, 4, cities_min=0, cities_max=1, min_general_dist=2)
    n = run_case(gen, 4, 4, 2, 3, 48, 300, seed=21, actor_seed=22, prm=prm)
    assert n > 30


def test_tokens_window_past_512_turns(gen):
    """Long 1v1 games (auto-reset off): the 512-turn scoreboard window wraps
    its ring; every turn recorded twice; tokens checked on the way."""
    import torch
    prm = prm_for(8, 8, min_general_dist=6, auto_reset=0)
    H = W = 8
    b = gen.Batch(6, H, W, 0, gen.make_params(0, 2, **prm), seed=13)
    cfg = oracle.Config(H=H, W=W, mode=0, P=2, seed=13, env_base=0, **prm)
    ost, _ = oracle.reset(cfg, 6)
    mem = oracle.feature_memory(6)
    b.sample(14, 0)
    for t in range(700):
        b.features()
        b.features(tokens=True)
        oracle.features(cfg, ost, mem)
        want, wtok = oracle.features(cfg, ost, mem, tokens=True)
        if t in (0, 1, 300, 511, 512, 513, 650, 699):
            torch.cuda.synchronize()
            assert np.array_equal(b.tokens.cpu().numpy(), wtok), f"tokens at step {t}"
            assert_features_equal(b.feat.cpu().numpy(), want, f"features at step {t}")
        b.step_sample(14, t + 1)
        oracle.step(cfg, ost, oracle.sample(cfg, ost, 14, t))
    assert (ost["turn"] >= 600).any()


def test_features_full_size_sampled(gen):
    """The 65,536-env 1v1 24x24 batch: features of every env for the first
    steps agree in their cheap invariants; a strided env subset is compared
    with the oracle every step."""
    import torch
    wl = workloads.C2
    prm = wl.params()
    E, steps = wl.n_envs, 12
    params = gen.make_params(wl.mode, wl.P, **prm)
    b = gen.Batch(E, wl.H, wl.W, wl.mode, params, seed=wl.seed)
    ids = np.unique(np.concatenate([np.arange(0, E, 2048), np.random.default_rng(1).choice(E, 16, replace=False)]))
    cfgs = {int(e): oracle.Config(H=wl.H, W=wl.W, mode=wl.mode, P=wl.P, seed=wl.seed, env_base=int(e), **prm)
            for e in ids}
    osts = {e: oracle.reset(c, 1)[0] for e, c in cfgs.items()}
    mems = {e: oracle.feature_memory(1) for e in cfgs}
    idx = torch.as_tensor(ids, device="cuda")
    b.sample(wl.actor_seed, 0)
    for t in range(steps + 1):
        b.features(tokens=True)
        sub = b.feat.index_select(0, idx).cpu().numpy()
        tsub = b.tokens.index_select(0, idx).cpu().numpy()
        for i, e in enumerate(ids):
            want, wtok = oracle.features(cfgs[int(e)], osts[int(e)], mems[int(e)], tokens=True)
            assert_features_equal(sub[i:i + 1], want, f"c2 env {e} step {t}")
            assert np.array_equal(tsub[i:i + 1], wtok), f"c2 env {e} step {t} tokens"
        if t == steps:
            break
        b.step_sample(wl.actor_seed, t + 1)
        for e, c in cfgs.items():
            oracle.step(c, osts[e], oracle.sample(c, osts[e], wl.actor_seed, t))
    # whole-batch invariants on the last frame
    f = b.feat
    fog, seen, own = f[:, :, 12], f[:, :, 4], f[:, :, 10]
    assert bool(((fog == 0) | (fog == 1)).all())
    assert bool((seen >= 1 - fog).all())                 # visible now => seen
    assert bool((fog[own > 0] == 0).all())               # own cells are visible
    assert torch.equal(own.sum(dim=(2, 3)), f[:, :, 16, 0, 0])
    turn = torch.as_tensor(b.get_state()["turn"], device="cuda").float()
    assert torch.equal(f[:, 0, 14, 0, 0], turn)


@pytest.mark.parametrize("generator", [0, 1])
def test_rollout_matches_oracle(gen, generator):
    """gen_rollout = features, random actor, step, T times; compared with the
    oracle doing the same, step by step, on every buffer slice."""
    import torch
    H = W = 10
    E, T, seed, actor = 12, 40, 77, 78
    prm = prm_for(H, W, generator=generator, min_general_dist=5 if generator else 4, castle_radius=6)
    b = gen.Batch(E, H, W, 0, gen.make_params(0, 2, **prm), seed=seed)
    cfg = oracle.Config(H=H, W=W, mode=0, P=2, seed=seed, env_base=0, **prm)
    ost, _ = oracle.reset(cfg, E)
    mem = oracle.feature_memory(E)
    out = b.rollout(T, actor, 0, tokens=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    for t in range(T):
        want, wtok = oracle.features(cfg, ost, mem, tokens=True)
        assert_features_equal(got["feat"][t], want, f"rollout t={t}")
        assert np.array_equal(got["tokens"][t], wtok), f"rollout tokens t={t}"
        act = oracle.sample(cfg, ost, actor, t)
        assert np.array_equal(got["actions"][t], act), f"rollout actions t={t}"
        r, d = oracle.step(cfg, ost, act)
        assert np.array_equal(got["rewards"][t], r) and np.array_equal(got["dones"][t], d), f"rollout t={t}"
    st = b.get_state()
    for k in ("owner", "army", "type", "turn", "episode"):
        assert np.array_equal(st[k], ost[k]), k
    # a second rollout continues the same trajectory and memory
    out2 = b.rollout(5, actor, T, tokens=False, out={k: v[:5] for k, v in out.items() if k != "tokens"})
    torch.cuda.synchronize()
    for t in range(5):
        want = oracle.features(cfg, ost, mem)
        assert_features_equal(out2["feat"][t].cpu().numpy(), want, f"second rollout t={t}")
        oracle.step(cfg, ost, oracle.sample(cfg, ost, actor, T + t))
