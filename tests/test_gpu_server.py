"""The served form: continuous batching over a device arena.

Each group's results must be the same whether its steps ran alone or
batched with other groups' steps, and must match the CPU oracle."""
import threading

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
KEYS = ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")
WAIT_US = 20_000_000          # every wait is bounded


@pytest.fixture(scope="module")
def gen():
    import torch
    import paper_2606_23348_amd as g
    assert torch.cuda.is_available()
    g.lib()
    return g


def group_specs(n, seed, lo=6, hi=20):
    rng = np.random.default_rng(seed)
    H, W = rng.integers(lo, hi + 1, n), rng.integers(lo, hi + 1, n)
    mode = rng.integers(0, 3, n)
    P = np.where(mode == 0, 2, np.where(mode == 1, 4, rng.integers(2, 7, n)))
    cmax = np.minimum(H * W // 8, 8)
    return {"H": H, "W": W, "mode": mode, "P": P, "cities_min": cmax // 2, "cities_max": cmax,
            "min_general_dist": np.minimum((H + W) // 4, 8)}


def uniform_specs(n, H, W, mode, P):
    """n envs of one shape and one set of settings (the server derives their
    descriptors from the first env's instead of loading them)."""
    cmax = min(H * W // 8, 8)
    return {"H": np.full(n, H), "W": np.full(n, W), "mode": np.full(n, mode), "P": np.full(n, P),
            "cities_min": np.full(n, cmax // 2), "cities_max": np.full(n, cmax),
            "min_general_dist": np.full(n, min((H + W) // 4, 8))}


def common(gen):
    return gen.make_params(0, 2, mountain_thresh=workloads.mountain_thresh(1, 5), city_army_min=40,
                           city_army_max=50, auto_reset=1)


def gen_mod():
    import paper_2606_23348_amd
    return paper_2606_23348_amd


def snapshot(srv, gid, specs):
    """Every env's state and the bytes the step defines (each env's
    observation block, not the alignment padding between blocks)."""
    b = srv.buffers(gid)
    st = [srv.get_env(gid, e, int(specs["H"][e]), int(specs["W"][e]), int(specs["P"][e])) for e in range(b["n_envs"])]
    obs = b["obs"].cpu().numpy()
    blocks = np.concatenate([gen_mod().pool_env_obs(obs, int(b["obs_off"][e]), int(specs["H"][e]), int(specs["W"][e]),
                                                    int(specs["P"][e])).reshape(-1) for e in range(b["n_envs"])])
    return st, blocks, b["actions"].cpu().numpy(), b["rewards"].cpu().numpy(), b["dones"].cpu().numpy()


def test_server_mix_vs_alone(gen):
    specs = [group_specs(n, 100 + i) for i, n in enumerate((40, 7, 130, 64, 1, 90))]
    specs += [uniform_specs(70, 24, 24, 0, 2), uniform_specs(33, 13, 11, 1, 4), uniform_specs(20, 9, 7, 2, 5)]
    bases = np.cumsum([0] + [len(s["H"]) for s in specs])
    T = 25
    results = {}
    for mode in ("alone", "mixed"):
        srv = gen.Server(256 << 20, n_launch_streams=2)
        gids = [srv.open(s, seed=17, env_base=int(bases[i]), common=common(gen), actor_seed=23)
                for i, s in enumerate(specs)]
        for t in range(T):
            if mode == "alone":
                for g in gids:
                    assert srv.wait(srv.submit(g), WAIT_US) == gen.GEN_OK
            else:
                tickets = [srv.submit(g) for g in gids]
                for tk in tickets:
                    assert srv.wait(tk, WAIT_US) == gen.GEN_OK
        results[mode] = [snapshot(srv, g, s) for g, s in zip(gids, specs)]
        rep = srv.report()
        assert rep["requests"] == T * len(gids)
        if mode == "mixed":
            assert rep["envs_per_launch"] > max(len(s["H"]) for s in specs)   # steps of several groups per launch
        srv.close_server()
    for (sa, oa, aa, ra, da), (sb, ob, ab, rb, db) in zip(results["alone"], results["mixed"]):
        for x, y in zip(sa, sb):
            for k in KEYS:
                assert np.array_equal(x[k], y[k])
        for x, y in ((oa, ob), (aa, ab), (ra, rb), (da, db)):
            assert np.array_equal(x, y)
    # and every env of every group the same as an independent oracle run:
    # state, observation block, actions, rewards and done
    for i, s in enumerate(specs):
        st_m, obs_m, act_m, rew_m, done_m = results["mixed"][i]
        at_obs = at_act = 0
        for e in range(len(s["H"])):
            H, W, P = int(s["H"][e]), int(s["W"][e]), int(s["P"][e])
            cfg = oracle.Config(H=H, W=W, mode=int(s["mode"][e]), P=P,
                                mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=int(s["cities_min"][e]),
                                cities_max=int(s["cities_max"][e]), city_army_min=40, city_army_max=50,
                                min_general_dist=int(s["min_general_dist"][e]), auto_reset=1, seed=17,
                                env_base=int(bases[i]) + e)
            ost, _ = oracle.reset(cfg, 1)
            for t in range(T):
                r, d = oracle.step(cfg, ost, oracle.sample(cfg, ost, 23, t))
            for k in KEYS:
                assert np.array_equal(st_m[e][k], ost[k]), (i, e, k)
            want = oracle.observe(cfg, ost).reshape(-1)
            assert np.array_equal(obs_m[at_obs:at_obs + want.size], want), (i, e, "obs")
            assert np.array_equal(rew_m[at_act:at_act + P], r[0]) and done_m[e] == d[0], (i, e, "reward")
            assert np.array_equal(act_m[at_act:at_act + P], oracle.sample(cfg, ost, 23, T)[0]), (i, e, "actions")
            at_obs += want.size
            at_act += P


def test_server_budget_admission_queue(gen):
    """Admission by an HBM budget of 1 GiB: opens that do not fit are queued
    and admitted in order of arrival as closes free memory; a request
    submitted to a queued group runs once the group is admitted, with the
    results of a group that fitted at once."""
    specs = group_specs(16384, 5, 20, 24)
    srv = gen.Server(1 << 30, n_launch_streams=1)
    tables = srv.report()["bytes_in_use"]      # the server's own request tables
    opened = [srv.open(specs, seed=1, env_base=16384 * i, common=common(gen), actor_seed=2, queue=True)
              for i in range(6)]
    k = sum(adm for _, adm in opened)
    assert 1 <= k < 6 and all(adm for _, adm in opened[:k]) and not any(adm for _, adm in opened[k:])
    rep = srv.report()
    assert rep["groups_queued"] == 6 - k and rep["groups_pending"] == 6 - k and rep["groups_open"] == k
    assert rep["bytes_in_use"] <= rep["arena_bytes"]
    first_q = opened[k][0]
    with pytest.raises(gen.GenError) as ei:
        srv.buffers(first_q)                   # not admitted yet
    assert ei.value.code == gen.GEN_EBUSY
    tk = srv.submit(first_q)                   # queued behind the admission
    assert srv.wait(tk, 200_000) == gen.GEN_EBUSY
    assert srv.wait_admitted(first_q, 0) == gen.GEN_EBUSY
    last_q = opened[-1][0]
    srv.close(last_q)                          # a queued group leaves the queue
    with pytest.raises(gen.GenError) as ei:
        srv.wait_admitted(last_q, 0)
    assert ei.value.code == gen.GEN_ENOTFOUND
    srv.close(opened[0][0])                    # memory frees up -> the first queued group is admitted
    assert srv.wait_admitted(first_q, WAIT_US) == gen.GEN_OK
    assert srv.wait(tk, WAIT_US) == gen.GEN_OK
    rep = srv.report()
    assert rep["groups_pending"] == max(0, 6 - k - 2)
    # the queued group's step equals that of a group opened with room to spare
    ref = gen.Server(1 << 30, n_launch_streams=1)
    g_ref = ref.open(specs, seed=1, env_base=16384 * k, common=common(gen), actor_seed=2)
    assert ref.wait(ref.submit(g_ref), WAIT_US) == gen.GEN_OK
    got, want = snapshot(srv, first_q, specs), snapshot(ref, g_ref, specs)
    for x, y in zip(got[0][:64], want[0][:64]):
        for key in KEYS:
            assert np.array_equal(x[key], y[key])
    for x, y in zip(got[1:], want[1:]):
        assert np.array_equal(x, y)
    ref.close_server()
    with pytest.raises(gen.GenError) as ei:    # larger than the whole arena: refused, not queued
        srv.open(group_specs(200000, 6, 24, 24), seed=1, common=common(gen), actor_seed=2)
    assert ei.value.code == gen.GEN_EINVAL
    for g, _ in opened[1:-1]:
        srv.close(g)
    rep = srv.report()
    assert rep["groups_open"] == 0 and rep["groups_pending"] == 0 and rep["bytes_in_use"] == tables
    srv.close_server()


def test_server_concurrent_clients(gen):
    srv = gen.Server(128 << 20, n_launch_streams=2)
    specs = group_specs(96, 8)
    gids = [srv.open(specs, seed=3, env_base=96 * i, common=common(gen), actor_seed=4) for i in range(12)]
    errors = []

    def client(g):
        try:
            for _ in range(40):
                if srv.wait(srv.submit(g), WAIT_US) != gen.GEN_OK:
                    errors.append("timeout")
                    return
        except Exception as exc:  # pragma: no cover - reported below
            errors.append(repr(exc))

    th = [threading.Thread(target=client, args=(g,)) for g in gids]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=60)
    assert not errors and not any(t.is_alive() for t in th)
    rep = srv.report()
    assert rep["requests"] == 12 * 40 and rep["frames"] == 12 * 40 * 96
    assert rep["launches"] <= rep["requests"]
    assert 0 < rep["lat_p50_us"] <= rep["lat_p99_us"]
    srv.close_server()


def test_server_native_clients(gen):
    srv = gen.Server(512 << 20, n_launch_streams=2)
    n_clients, gpc = 16, 2
    sizes = workloads.group_sizes(5, n_clients * gpc, 64, 256)
    specs = workloads.mixed_specs(int(sizes.sum()), 5)
    gaps = np.stack([workloads.arrival_gaps(2005, c, 64, 4000.0) * 1e6 for c in range(n_clients)])
    rep = srv.drive(sizes, specs, seed=5, actor_seed=1005, gaps_us=gaps, duration_s=0.5, steps_per_group=40,
                    common=common(gen))
    assert rep["requests"] > 100 and rep["frames"] > 0 and rep["wall_s"] > 0.4
    assert 0 < rep["lat_p50_us"] <= rep["lat_p99_us"]
    assert srv.report()["groups_open"] == 0
    srv.close_server()


def test_server_back_to_back_clients_end_on_time(gen):
    """All-zero arrival gaps mean back-to-back closed-loop requests; the
    measured window still ends after duration_s."""
    import time
    srv = gen.Server(256 << 20, n_launch_streams=2)
    sizes = np.full(8, 64)
    specs = workloads.mixed_specs(int(sizes.sum()), 9)
    t0 = time.perf_counter()
    rep = srv.drive(sizes, specs, seed=9, actor_seed=10, gaps_us=np.zeros((8, 1)), duration_s=0.3,
                    steps_per_group=0, common=common(gen))
    assert time.perf_counter() - t0 < 30
    assert rep["requests"] > 8 and 0.3 <= rep["wall_s"] < 5
    srv.close_server()
