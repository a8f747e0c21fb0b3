"""Batched pool (mixed shapes and modes in one launch) against the CPU oracle.

Every pool env is compared with an independent single-env oracle run keyed
by its global id; the pool's random actor draws with each env's own step
counter, which equals the step number t of these runs.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
KEYS = ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")


@pytest.fixture(scope="module")
def gen():
    import torch
    import paper_2606_23348_amd as g
    assert torch.cuda.is_available()
    g.lib()
    return g


def random_specs(n, seed, lo=3, hi=32):
    """Shapes from lo..hi per side, all three modes, FFA with 2..8 players."""
    rng = np.random.default_rng(seed)
    H = rng.integers(lo, hi + 1, n)
    W = rng.integers(lo, hi + 1, n)
    mode = rng.integers(0, 3, n)
    P = np.where(mode == 0, 2, np.where(mode == 1, 4, rng.integers(2, 9, n)))
    HW = H * W
    cmax = np.minimum(HW // 6, 12)
    return {"H": H, "W": W, "mode": mode, "P": P, "cities_min": cmax // 2, "cities_max": cmax,
            "min_general_dist": np.minimum((H + W) // 4, 9)}


def common_params(gen, auto_reset=1):
    return gen.make_params(0, 2, mountain_thresh=workloads.mountain_thresh(1, 5), city_army_min=40,
                           city_army_max=50, auto_reset=auto_reset, pregrow=0)


def env_cfg(specs, e, seed, env_base=0, auto_reset=1):
    return oracle.Config(H=int(specs["H"][e]), W=int(specs["W"][e]), mode=int(specs["mode"][e]),
                         P=int(specs["P"][e]), mountain_thresh=workloads.mountain_thresh(1, 5),
                         cities_min=int(specs["cities_min"][e]), cities_max=int(specs["cities_max"][e]),
                         city_army_min=40, city_army_max=50, min_general_dist=int(specs["min_general_dist"][e]),
                         auto_reset=auto_reset, pregrow=0, seed=seed, env_base=env_base + e)


def check_env(pool, e, cfg, ost, obs_cpu, act_cpu, where, next_act=None):
    got = pool.get_env(e)
    for k in KEYS:
        assert np.array_equal(got[k], ost[k]), f"{where}: env {e} field {k}"
    import paper_2606_23348_amd as gen
    o = int(pool.obs_off[e])
    P, H, W = cfg.P, cfg.H, cfg.W
    assert np.array_equal(gen.pool_env_obs(obs_cpu, o, H, W, P).reshape(1, P, 8, H, W), oracle.observe(cfg, ost)), \
        f"{where}: env {e} obs"
    PS = gen.plane_stride(H, W, P)
    assert not obs_cpu[o:o + P * 8 * PS].reshape(P * 8, PS)[:, H * W:].any(), f"{where}: env {e} plane padding"
    if next_act is not None:
        sl = pool.env_slice(e)
        assert np.array_equal(act_cpu[sl], next_act[0]), f"{where}: env {e} actions"


def test_pool_reset_parity(gen):
    import torch
    specs = random_specs(160, 1)
    seed, actor = 31, 77
    pool = gen.Pool(specs, common_params(gen), seed=seed)
    pool.reset(actor_seed=actor)
    torch.cuda.synchronize()
    obs, act = pool.obs.cpu().numpy(), pool.actions.cpu().numpy()
    for e in range(pool.n):
        cfg = env_cfg(specs, e, seed)
        ost, _ = oracle.reset(cfg, 1)
        check_env(pool, e, cfg, ost, obs, act, "reset", oracle.sample(cfg, ost, actor, 0))


@pytest.mark.parametrize("lo,hi,n,steps", [(3, 8, 96, 300), (8, 32, 64, 120)])
def test_pool_trajectory_parity(gen, lo, hi, n, steps):
    import torch
    specs = random_specs(n, lo * 100 + hi, lo, hi)
    seed, actor = 5 + lo, 900 + hi
    pool = gen.Pool(specs, common_params(gen), seed=seed)
    pool.reset(actor_seed=actor)
    cfgs = [env_cfg(specs, e, seed) for e in range(n)]
    osts = [oracle.reset(c, 1)[0] for c in cfgs]
    for t in range(steps):
        pool.step(actor_seed=actor)
        torch.cuda.synchronize()
        obs, act = pool.obs.cpu().numpy(), pool.actions.cpu().numpy()
        rew, done = pool.rewards.cpu().numpy(), pool.dones.cpu().numpy()
        for e in range(n):
            a = oracle.sample(cfgs[e], osts[e], actor, t)
            r, d = oracle.step(cfgs[e], osts[e], a)
            assert np.array_equal(rew[pool.env_slice(e)], r[0]) and done[e] == d[0], f"step {t} env {e}"
            if t % 10 == 0 or t == steps - 1:
                check_env(pool, e, cfgs[e], osts[e], obs, act, f"step {t}",
                          oracle.sample(cfgs[e], osts[e], actor, t + 1))


def _digest(gen, specs, tuning, steps=25, buckets=None):
    import torch
    pool = gen.Pool(specs, common_params(gen), seed=9)
    pool.set_tuning(**tuning)
    if buckets is not None:
        pool.set_buckets(buckets(pool.buckets()))
    pool.reset(actor_seed=3)
    for _ in range(steps):
        pool.step(actor_seed=3)
    torch.cuda.synchronize()
    return pool.digest()


def test_pool_results_independent_of_packing(gen):
    specs = random_specs(700, 11, 3, 24)        # 4 waves x the largest env fit in 64 KiB of LDS
    ref = _digest(gen, specs, dict(waves_per_group=1, grid=0, order=0))
    for tun in (dict(waves_per_group=2, grid=0, order=0), dict(waves_per_group=4, grid=0, order=1),
                dict(waves_per_group=1, grid=37, order=1), dict(waves_per_group=2, grid=100, order=0)):
        assert _digest(gen, specs, tun) == ref, tun

    # per-bucket packings: every bucket its own choice, one launch per distinct packing
    def mixed(bks):
        choices = [(1, 2), (2, 1), (4, 1), (1, 1)]
        return [dict(n_players=b["n_players"], words=b["words"], waves_per_group=choices[i % 4][0],
                     waves_per_env=choices[i % 4][1]) for i, b in enumerate(bks)]

    def two_waves(bks):
        return [dict(n_players=b["n_players"], words=b["words"], waves_per_group=1, waves_per_env=2) for b in bks]

    assert _digest(gen, specs, dict(waves_per_group=1, grid=0, order=0), buckets=mixed) == ref
    assert _digest(gen, specs, dict(waves_per_group=2, grid=0, order=1), buckets=two_waves) == ref
    assert _digest(gen, specs, dict(waves_per_group=1, grid=64, order=0), buckets=mixed) == ref


def test_pool_bucket_packing_parity(gen):
    """Buckets with two waves per env (later players' planes on the second
    wave) and others packed 2 per workgroup, against the oracle env by env."""
    import torch
    specs = random_specs(90, 21, 4, 20)
    seed, actor = 19, 940
    pool = gen.Pool(specs, common_params(gen), seed=seed)
    bks = pool.buckets()
    pool.set_buckets([dict(n_players=b["n_players"], words=b["words"], waves_per_group=1 if i % 2 == 0 else 2,
                           waves_per_env=2 if i % 2 == 0 else 1) for i, b in enumerate(bks)])
    pool.reset(actor_seed=actor)
    cfgs = [env_cfg(specs, e, seed) for e in range(pool.n)]
    osts = [oracle.reset(c, 1)[0] for c in cfgs]
    for t in range(150):
        pool.step(actor_seed=actor)
        torch.cuda.synchronize()
        obs, act = pool.obs.cpu().numpy(), pool.actions.cpu().numpy()
        rew, done = pool.rewards.cpu().numpy(), pool.dones.cpu().numpy()
        for e in range(pool.n):
            r, d = oracle.step(cfgs[e], osts[e], oracle.sample(cfgs[e], osts[e], actor, t))
            assert np.array_equal(rew[pool.env_slice(e)], r[0]) and done[e] == d[0], f"step {t} env {e}"
            if t % 5 == 0 or t == 149:
                check_env(pool, e, cfgs[e], osts[e], obs, act, f"step {t}", oracle.sample(cfgs[e], osts[e], actor, t + 1))


@pytest.mark.skip(reason="hung twice in s.synchronize() after the first graph replay (intermittent, GPU "
                         "answered, no fault); cause not shown: kept off the GPU until it is")
def test_pool_graph_replay_equals_eager(gen):
    import torch
    specs = random_specs(300, 12, 5, 25)
    eager = gen.Pool(specs, common_params(gen), seed=4)
    eager.reset(actor_seed=8)
    for _ in range(12):
        eager.step(actor_seed=8)
    torch.cuda.synchronize()
    graphed = gen.Pool(specs, common_params(gen), seed=4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graphed.reset(actor_seed=8, stream=s)
        graphed.capture(4, 8, s)
        for _ in range(3):                 # 3 replays x 4 steps, host work in between
            graphed.replay(s)
            s.synchronize()
            _ = graphed.dones.sum().item()
    torch.cuda.synchronize()
    for a, b in ((eager.buf, graphed.buf), (eager.obs, graphed.obs), (eager.actions, graphed.actions),
                 (eager.rewards, graphed.rewards), (eager.dones, graphed.dones)):
        assert torch.equal(a, b)


def test_pool_mixed_workload_full_size(gen):
    """The 131,072-env mixed pool (shapes 10..25, 60% 1v1 / 25% 2v2 / 15%
    FFA-4), stepped by captured graphs; sampled envs checked every step."""
    import torch
    wl = workloads.C4
    specs = workloads.mixed_specs(wl.n_envs, wl.seed)
    pool = gen.Pool(specs, common_params(gen), seed=wl.seed)
    s = torch.cuda.Stream()
    rng = np.random.default_rng(0)
    ids = np.unique(np.concatenate([np.arange(0, wl.n_envs, 4096), rng.choice(wl.n_envs, 32, replace=False)]))
    cfgs = {int(e): env_cfg(specs, int(e), wl.seed) for e in ids}
    osts = {e: oracle.reset(c, 1)[0] for e, c in cfgs.items()}
    with torch.cuda.stream(s):
        pool.reset(actor_seed=wl.actor_seed, stream=s)
        pool.capture(1, wl.actor_seed, s)
        for t in range(40):
            pool.replay(s)
            s.synchronize()
            obs, act = pool.obs.cpu().numpy(), pool.actions.cpu().numpy()
            for e, c in cfgs.items():
                a = oracle.sample(c, osts[e], wl.actor_seed, t)
                oracle.step(c, osts[e], a)
                if t % 5 == 4:
                    check_env(pool, e, c, osts[e], obs, act, f"c4 step {t}",
                              oracle.sample(c, osts[e], wl.actor_seed, t + 1))
