"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Both sides start from the same seeds and run independently: the oracle makes
its own maps and its own random-actor draws; nothing the GPU produced is fed
to the oracle.  Everything is integer, so every comparison is bit-exact.
"""
import hashlib

import numpy as np
import pytest

import oracle
import workloads
from tests import scenarios as scn

pytestmark = pytest.mark.gpu

KEYS = ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")


@pytest.fixture(scope="module")
def gen():
    import torch
    import paper_2606_23348_amd as g
    assert torch.cuda.is_available()
    g.lib()
    return g


def gparams(gen, mode, P, prm):
    return gen.make_params(mode, P, **{k: v for k, v in prm.items() if k != "n_players"})


def ocfg(H, W, mode, P, seed, env_base=0, **prm):
    return oracle.Config(H=H, W=W, mode=mode, P=P, seed=seed, env_base=env_base,
                         **{k: v for k, v in prm.items() if k != "n_players"})


def assert_state_equal(got, want, where=""):
    for k in KEYS:
        if not np.array_equal(got[k], want[k]):
            bad = np.argwhere(got[k] != want[k])
            raise AssertionError(f"{where}: field {k} differs at {bad[:5].tolist()} "
                                 f"(gpu {got[k][tuple(bad[0])]}, oracle {want[k][tuple(bad[0])]})")


def assert_obs_equal(got, want, where=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{where}: obs differs at {len(bad)} places, first {bad[:5].tolist()}")


def gpu_obs(b):
    """The batch's observation as uint8 [E, P, 8, H, W]; with padded planes
    (obs_layout 1) also checks that the padding bytes are zero."""
    if b.padded:
        raw = b.obs.cpu().numpy()
        assert not raw[..., b.H * b.W:].any(), "nonzero plane padding"
    return b.obs_dense()


def run_parity(gen, H, W, mode, P, E, steps, seed, actor_seed, prm, check_every=1, scoreboard=False,
               fused=False, obs_layout=0):
    """Step E envs on both sides for `steps` steps with the random actor;
    compare actions, rewards, dones, observations and full state.  With
    fused=True the GPU runs gen_step_sample (step + next actions in one
    launch) and its actions are compared with the oracle's next draw.
    obs_layout=1: the GPU writes planes padded to 32 bytes (64 with more than 2 players)."""
    import torch
    params = gparams(gen, mode, P, dict(prm, obs_layout=obs_layout))
    b = gen.Batch(E, H, W, mode, params, seed=seed, scoreboard=scoreboard)
    cfg = ocfg(H, W, mode, P, seed, **prm)
    ost, att = oracle.reset(cfg, E)
    torch.cuda.synchronize()
    assert_state_equal(b.get_state(), ost, "reset")
    assert_obs_equal(gpu_obs(b), oracle.observe(cfg, ost), "reset obs")
    n_done = 0
    if fused:
        b.sample(actor_seed, 0)
    for t in range(steps):
        oact = oracle.sample(cfg, ost, actor_seed, t)
        if fused:
            b.step_sample(actor_seed, t + 1)
        else:
            b.sample(actor_seed, t)
            if t % check_every == 0 or t == steps - 1:
                assert np.array_equal(b.actions.cpu().numpy(), oact), f"step {t} actions"
            b.step()
        orew, odone = oracle.step(cfg, ost, oact)
        if t % check_every == 0 or t == steps - 1:
            where = f"{H}x{W} mode {mode} P {P} step {t}"
            if fused:
                assert np.array_equal(b.actions.cpu().numpy(), oracle.sample(cfg, ost, actor_seed, t + 1)), \
                    where + " next actions"
            assert np.array_equal(b.rewards.cpu().numpy(), orew), where + " rewards"
            assert np.array_equal(b.dones.cpu().numpy(), odone), where + " dones"
            assert_obs_equal(gpu_obs(b), oracle.observe(cfg, ost), where)
            assert_state_equal(b.get_state(), ost, where)
            if scoreboard:
                land, army = oracle.scoreboard(cfg, ost)
                assert np.array_equal(b.land.cpu().numpy(), land), where + " land"
                assert np.array_equal(b.army.cpu().numpy(), army), where + " army"
        n_done += int(odone.sum())
    return n_done


# ------------------------------------------------------------------ resets
@pytest.mark.parametrize("H,W,mode,P,E", [
    (10, 10, 0, 2, 16), (24, 24, 0, 2, 64), (25, 25, 2, 8, 32), (13, 11, 1, 4, 40), (3, 3, 0, 2, 20),
    (32, 32, 2, 5, 9), (7, 19, 2, 3, 33), (16, 20, 1, 4, 50), (4, 9, 0, 2, 70)])
def test_reset_matches_oracle(gen, H, W, mode, P, E):
    import torch
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=min(2, H * W // 8),
               cities_max=min(5, H * W // 4), min_general_dist=min(6, (H + W) // 3), auto_reset=1)
    b = gen.Batch(E, H, W, mode, gparams(gen, mode, P, prm), seed=H * 100 + W)
    cfg = ocfg(H, W, mode, P, H * 100 + W, **prm)
    ost, _ = oracle.reset(cfg, E)
    torch.cuda.synchronize()
    assert_state_equal(b.get_state(), ost, f"reset {H}x{W}")
    assert_obs_equal(b.obs.cpu().numpy(), oracle.observe(cfg, ost), f"reset obs {H}x{W}")


def test_reset_pregrow_and_env_base(gen):
    import torch
    wl = workloads.C3
    prm = wl.params()
    b = gen.Batch(24, 25, 25, 2, gparams(gen, 2, 8, prm), seed=3, env_base=1000)
    cfg = ocfg(25, 25, 2, 8, 3, env_base=1000, **prm)
    ost, _ = oracle.reset(cfg, 24)
    torch.cuda.synchronize()
    got = b.get_state()
    assert_state_equal(got, ost, "pregrow")
    g = got["army"][np.arange(24)[:, None], got["gpos"].astype(int)]
    assert (g[::4] >= 100000).all() and (g[1::4] == 1).all()


# ------------------------------------------------------------------ trajectories
def test_c1_full_trajectory(gen):
    """Workload plain-1v1-10x10-16env in full: 1,000 steps, every field every step."""
    wl = workloads.C1
    run_parity(gen, wl.H, wl.W, wl.mode, wl.P, wl.n_envs, wl.steps, wl.seed, wl.actor_seed, wl.params())


@pytest.mark.parametrize("H,W,mode,P,E,steps", [
    (24, 24, 0, 2, 48, 300),     # planes of a multiple of 4 cells
    (10, 10, 1, 4, 40, 300),     # 2v2, planes of a multiple of 4 cells
    (25, 25, 2, 8, 24, 200),     # FFA-8, H*W = 1 mod 4 over three rounds of quads
    (7, 9, 2, 3, 37, 300),       # FFA-3, H*W = 3 mod 4 in one round
    (3, 3, 0, 2, 64, 200),       # tiny grid
    (32, 32, 2, 4, 8, 150),      # largest grid
    (11, 23, 1, 4, 30, 250),
    (17, 6, 2, 6, 30, 250),
    (17, 18, 0, 2, 24, 150),     # H*W = 2 mod 4 over two rounds of quads
    (19, 17, 2, 5, 20, 150),     # H*W = 3 mod 4 over two rounds; players 4.. draw from the second block
    (31, 31, 1, 4, 8, 100),      # H*W = 1 mod 4 over four rounds, 2v2
    (13, 9, 2, 7, 20, 150),      # FFA-7: the two waves of an env write 2 and 5 players' planes
    (32, 32, 2, 8, 6, 120),      # the largest grid with the most players: 64 planes of 1,024 cells
])
@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_trajectory_parity(gen, H, W, mode, P, E, steps, fused):
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=min(2, H * W // 8),
               cities_max=min(6, H * W // 4), min_general_dist=min(5, (H + W) // 3), auto_reset=1)
    run_parity(gen, H, W, mode, P, E, steps, seed=H * 7 + W, actor_seed=99, prm=prm, check_every=1, fused=fused)


@pytest.mark.parametrize("H,W,mode,P,E,steps", [
    (25, 25, 2, 8, 24, 200),     # FFA-8: two waves per env share the padded planes
    (13, 9, 2, 7, 20, 150),      # FFA-7, two waves (2 and 5 players' planes)
    (7, 9, 2, 3, 37, 300),       # one wave, H*W = 3 mod 4
    (17, 18, 0, 2, 24, 150),     # H*W = 2 mod 4
    (31, 31, 1, 4, 8, 100),      # 2v2, H*W = 1 mod 4
    (3, 3, 0, 2, 64, 200),       # tiny grid: one quad of map cells, seven of padding
    (8, 4, 0, 2, 16, 100),       # H*W = 32: padded and dense layouts coincide
    (32, 32, 2, 8, 6, 120),      # the largest grid with the most players
])
@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_trajectory_parity_padded_planes(gen, H, W, mode, P, E, steps, fused):
    """obs_layout 1 (planes padded to 32 or 64 bytes, every plane written by the
    dword writer): the same observation bytes, zero padding."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=min(2, H * W // 8),
               cities_max=min(6, H * W // 4), min_general_dist=min(5, (H + W) // 3), auto_reset=1)
    run_parity(gen, H, W, mode, P, E, steps, seed=H * 11 + W, actor_seed=98, prm=prm, check_every=1, fused=fused,
               obs_layout=1)


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_two_wave_padded_regenerates_maps(gen, fused):
    """Two waves per env on padded planes with many episode ends (5x5 FFA-5)."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=0, cities_max=1, min_general_dist=2,
               auto_reset=1)
    n = run_parity(gen, 5, 5, 2, 5, 64, 500, seed=43, actor_seed=44, prm=prm, fused=fused, obs_layout=1)
    assert n > 10


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_trajectory_many_player_large_batch(gen, fused):
    """More than 4 players and unaligned planes in a batch above 16,384 envs:
    the steps keep one wave per env (smaller batches share the observation
    between two waves, covered by the FFA cases above)."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=1, cities_max=3, min_general_dist=3,
               auto_reset=1)
    run_parity(gen, 6, 7, 2, 5, 16400, 25, seed=13, actor_seed=14, prm=prm, check_every=5, fused=fused)


def test_trajectory_scoreboard_many_players(gen):
    """The scoreboard outputs with more than 4 players and unaligned planes
    (the two-wave step)."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=1, cities_max=3, min_general_dist=3,
               auto_reset=1)
    run_parity(gen, 7, 9, 2, 6, 40, 150, seed=15, actor_seed=16, prm=prm, scoreboard=True)


def test_trajectory_scoreboard_and_no_autoreset(gen):
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=1, cities_max=3, min_general_dist=3,
               auto_reset=0)
    n = run_parity(gen, 6, 6, 2, 4, 40, 400, seed=5, actor_seed=6, prm=prm, scoreboard=True)
    assert n > 0          # some games ended and stayed frozen


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_many_episodes_autoreset(gen, fused):
    """Small FFA maps end quickly under random play: exercises capture,
    elimination and in-kernel regeneration many times."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=0, cities_max=1, min_general_dist=2,
               auto_reset=1)
    n = run_parity(gen, 4, 4, 2, 3, 64, 500, seed=21, actor_seed=22, prm=prm, fused=fused)
    assert n > 50


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_two_wave_step_regenerates_maps(gen, fused):
    """More than 4 players on unaligned planes (5x5 FFA-5, 64 envs): the
    two-wave step, whose games end often here, so the in-kernel map
    generator runs on wave 0 while wave 1 waits, and the new map's planes
    are split across both waves."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=0, cities_max=1, min_general_dist=2,
               auto_reset=1)
    n = run_parity(gen, 5, 5, 2, 5, 64, 500, seed=41, actor_seed=42, prm=prm, fused=fused)
    assert n > 10


def test_c1_full_trajectory_fused(gen):
    wl = workloads.C1
    run_parity(gen, wl.H, wl.W, wl.mode, wl.P, wl.n_envs, wl.steps, wl.seed, wl.actor_seed, wl.params(), fused=True)


def test_fused_scoreboard_2v2(gen):
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=1, cities_max=3, min_general_dist=3,
               auto_reset=0)
    run_parity(gen, 8, 6, 1, 4, 40, 300, seed=15, actor_seed=16, prm=prm, scoreboard=True, fused=True)


# ------------------------------------------------------------------ scenarios through the ABI
@pytest.mark.parametrize("sc", scn.load(), ids=lambda s: s["name"])
def test_scenario_gpu(gen, sc):
    import torch
    H, W = len(sc["grid"]), len(sc["grid"][0].split())
    P, mode = sc["P"], sc["mode"]
    params = gen.make_params(mode, P, cities_min=0, cities_max=1, min_general_dist=1,
                             auto_reset=sc.get("auto_reset", 0))
    b = gen.Batch(1, H, W, mode, params, seed=7)
    b.set_state(scn.initial_state(sc))
    for k, stp in enumerate(sc["steps"]):
        b.actions.copy_(torch.from_numpy(scn.encode_actions(stp, P)))
        for _ in range(stp.get("repeat", 1)):
            b.step()
        got = b.get_state()
        exp = stp["expect"]
        assert scn.grid_of(got, H, W) == exp["grid"], f"step {k}"
        assert int(got["turn"][0]) == exp["turn"]
        assert b.rewards.cpu().numpy()[0].tolist() == exp["rewards"]
        assert int(b.dones.cpu()[0]) == exp["done"]
        assert int(got["alive"][0]) == exp["alive"]
        cfg = ocfg(H, W, mode, P, 7, auto_reset=sc.get("auto_reset", 0))
        assert_obs_equal(b.obs.cpu().numpy(), oracle.observe(cfg, got), sc["name"])


def test_autoreset_capture_returns_new_map(gen):
    """R13: capture with auto-reset on: terminal rewards, done, next episode's map and obs."""
    import torch
    sc = next(s for s in scn.load() if s["name"] == "H6_general_capture_1v1")
    prm = dict(cities_min=1, cities_max=2, min_general_dist=2, auto_reset=1)
    b = gen.Batch(1, 3, 4, 0, gparams(gen, 0, 2, prm), seed=11, env_base=5)
    cfg = ocfg(3, 4, 0, 2, 11, env_base=5, **prm)
    ost = scn.initial_state(sc)
    b.set_state(ost)
    b.actions.copy_(torch.from_numpy(scn.encode_actions(sc["steps"][0], 2)))
    b.step()
    orew, odone = oracle.step(cfg, ost, scn.encode_actions(sc["steps"][0], 2))
    assert b.rewards.cpu().numpy().tolist() == orew.tolist() == [[1, -1]]
    assert int(b.dones.cpu()[0]) == 1
    got = b.get_state()
    assert got["episode"][0] == 1
    assert_state_equal(got, ost, "auto-reset")
    assert_obs_equal(b.obs.cpu().numpy(), oracle.observe(cfg, ost), "auto-reset obs")


def test_saturation_growth_at_int32_max(gen):
    import torch
    b = gen.Batch(2, 5, 5, 0, gen.make_params(0, 2, cities_min=0, cities_max=1, min_general_dist=2), seed=1)
    h = b.get_state()
    h["army"][:, h["gpos"][0, 0]] = 2 ** 31 - 1
    h["army"][1, :] = np.where(h["owner"][1] >= 0, 2 ** 31 - 3, h["army"][1])
    b.set_state(h)
    cfg = ocfg(5, 5, 0, 2, 1, cities_min=0, cities_max=1, min_general_dist=2)
    for t in range(60):
        b.actions.zero_()
        b.step()
        oracle.step(cfg, h, np.zeros((2, 2), np.int32))
    assert_state_equal(b.get_state(), h, "saturation")
    assert (b.get_state()["army"] <= 2 ** 31 - 1).all()


def test_observe_entry_point(gen):
    import torch
    prm = dict(cities_min=2, cities_max=4, min_general_dist=4)
    b = gen.Batch(32, 9, 14, 2, gparams(gen, 2, 4, prm), seed=4)
    cfg = ocfg(9, 14, 2, 4, 4, **prm)
    ost, _ = oracle.reset(cfg, 32)
    for t in range(30):
        b.sample(8, t)
        b.step()
        oracle.step(cfg, ost, oracle.sample(cfg, ost, 8, t))
    obs2 = torch.empty_like(b.obs)
    gen.gen_observe(b.st, obs2)
    torch.cuda.synchronize()
    assert_obs_equal(obs2.cpu().numpy(), oracle.observe(cfg, ost), "observe")
    assert torch.equal(obs2, b.obs)


def test_determinism(gen):
    import torch

    def digest():
        b = gen.Batch(256, 16, 16, 1, gen.make_params(1, 4, cities_min=2, cities_max=4, min_general_dist=5), seed=3)
        h = hashlib.sha256()
        for t in range(50):
            b.sample(4, t)
            b.step()
            h.update(b.obs.cpu().numpy().tobytes())
        torch.cuda.synchronize()
        return h.hexdigest()

    assert digest() == digest()


# ------------------------------------------------------------------ official generator (reading R18)
@pytest.mark.parametrize("H,W,mode,P,E,dmin,dmax,radius", [
    (23, 23, 0, 2, 64, 17, 0, 6),      # the official 1v1 rules
    (16, 16, 0, 2, 64, 1, 4, 6),       # a curriculum stage: spawn distance capped at 4
    (20, 20, 1, 4, 32, 6, 0, 6),       # 2v2
    (18, 13, 2, 5, 32, 5, 9, 5),       # FFA-5 with both bounds
    (5, 5, 0, 2, 64, 3, 0, 4),         # small: some envs need several attempts
])
def test_official_reset_matches_oracle(gen, H, W, mode, P, E, dmin, dmax, radius):
    import torch
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=min(9, H * W // 8),
               cities_max=min(11, H * W // 6), min_general_dist=dmin, auto_reset=1, generator=1,
               max_general_dist=dmax, castle_radius=radius)
    b = gen.Batch(E, H, W, mode, gparams(gen, mode, P, prm), seed=H * 7 + W)
    cfg = ocfg(H, W, mode, P, H * 7 + W, **prm)
    ost, att = oracle.reset(cfg, E)
    torch.cuda.synchronize()
    assert_state_equal(b.get_state(), ost, f"official reset {H}x{W}")
    assert_obs_equal(b.obs.cpu().numpy(), oracle.observe(cfg, ost), f"official reset obs {H}x{W}")


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_official_trajectory_with_regeneration(gen, fused):
    """Small official maps end often: every auto-reset runs the official
    generator inside the step kernel."""
    prm = dict(mountain_thresh=workloads.mountain_thresh(1, 5), cities_min=1, cities_max=2, min_general_dist=3,
               auto_reset=1, generator=1, max_general_dist=0, castle_radius=4)
    n = run_parity(gen, 5, 5, 0, 2, 64, 300, seed=33, actor_seed=34, prm=prm, fused=fused)
    assert n > 10
