"""Parity of the 38-channel features (gen_features, Appendix A) with the CPU
oracle, through the C ABI.

Both sides step their own copy of the game with the same seeds (state parity
itself is covered by test_gpu_parity) and record features after the reset
and after the steps the case selects.  The tolerance comes from the
arithmetic: every channel is an exact integer, a 0/1 mask or a value computed
in double and rounded once to float32 (15, 22, 23: a division, correctly
rounded on both sides), so all must match bit for bit -- except channel 21,
log1p in double, where the device and host math libraries may differ in the
last double bit and so, rarely, by one float32 ulp after rounding.
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
    """got, want: float32 [..., 38, H, W]."""
    assert got.shape == want.shape, where
    g = np.delete(got, AGE, axis=-3)
    w = np.delete(want, AGE, axis=-3)
    if not np.array_equal(g, w):
        bad = np.argwhere(g != w)
        idx = tuple(bad[0])
        raise AssertionError(f"{where}: {len(bad)} values differ, first at {bad[:4].tolist()} "
                             f"(gpu {g[idx]}, oracle {w[idx]}; channel index after dropping {AGE})")
    ga = got[..., AGE, :, :].view(np.int32).astype(np.int64)
    wa = want[..., AGE, :, :].view(np.int32).astype(np.int64)
    ulp = np.abs(ga - wa).max(initial=0)
    assert ulp <= 1, f"{where}: channel {AGE} off by {ulp} ulp"


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
            b.features()
            torch.cuda.synchronize()
            want = oracle.features(cfg, ost, mem)
            where = f"{H}x{W} mode {mode} P {P} turn-step {t}"
            assert_features_equal(b.feat.cpu().numpy(), want, where)
            if t in repeat_at:                      # a second call on the same state changes nothing
                b.features()
                torch.cuda.synchronize()
                assert_features_equal(b.feat.cpu().numpy(), want, where + " (repeated)")
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
        b.features()
        sub = b.feat.index_select(0, idx).cpu().numpy()
        for i, e in enumerate(ids):
            want = oracle.features(cfgs[int(e)], osts[int(e)], mems[int(e)])
            assert_features_equal(sub[i:i + 1], want, f"c2 env {e} step {t}")
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
