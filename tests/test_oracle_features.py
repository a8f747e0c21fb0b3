"""Pins of the oracle's 38-channel features (Appendix A, reading R17).

The oracle keeps running memories and the last 8 frames.  Here every
channel is recomputed from its definition over the whole list of recorded
states of the episode (vision by scipy's binary dilation, "ever" masks as
ORs over all frames, the sticky enemy memory by a backward search, deltas by
looking frames up by turn), so a dropped term, a wrong sign or a stale
memory in the oracle shows up as a mismatch.
"""
import numpy as np
import pytest
from scipy.ndimage import binary_dilation

import oracle
import workloads

C = oracle.FEAT_CHANNELS
HH = 7


def team_of(mode, p, P):
    return [q for q in range(P) if q == p or (mode == oracle.MODE_2V2 and q % 2 == p % 2)]


def vis_map(f, p, mode, P, H, W):
    own = np.isin(f["owner"].reshape(H, W), team_of(mode, p, P))
    return binary_dilation(own, structure=np.ones((3, 3), bool))


def enemy_map(f, p, mode, P, H, W):
    o = f["owner"].reshape(H, W)
    return (o >= 0) & ~np.isin(o, team_of(mode, p, P))


def definitional(frames, mode, P, H, W):
    """Features of the last frame of `frames` (states of one env in record
    order) from every frame of its episode."""
    cur = frames[-1]
    ep = [f for f in frames if f["episode"] == cur["episode"]]
    turn = int(cur["turn"])
    army = cur["army"].reshape(H, W).astype(np.int64)
    owner = cur["owner"].reshape(H, W)
    typ = cur["type"].reshape(H, W)
    rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    out = np.zeros((P, C, H, W), np.float32)

    def by_turn(t):
        hits = [f for f in ep if int(f["turn"]) == t]
        return hits[-1] if hits else None

    for p in range(P):
        vis = vis_map(cur, p, mode, P, H, W)
        en = enemy_map(cur, p, mode, P, H, W)
        team = team_of(mode, p, P)
        enemies = [q for q in range(P) if q not in team]
        land = [(owner == q).sum() for q in range(P)]
        tot = [army[owner == q].sum() for q in range(P)]
        seen = np.zeros((H, W), bool)
        en_seen = np.zeros((H, W), bool)
        g_seen = np.zeros((H, W), bool)
        c_seen = np.zeros((H, W), bool)
        m_seen = np.zeros((H, W), bool)
        for f in ep:
            v = vis_map(f, p, mode, P, H, W)
            t = f["type"].reshape(H, W)
            seen |= v
            en_seen |= v & enemy_map(f, p, mode, P, H, W)
            g_seen |= v & (t == oracle.T_GENERAL)
            c_seen |= v & (t == oracle.T_CASTLE)
            m_seen |= v & (t == oracle.T_MOUNTAIN)
        vis_f = [vis_map(f, p, mode, P, H, W) for f in ep]
        en_f = [enemy_map(f, p, mode, P, H, W) for f in ep]
        last = np.zeros((H, W), np.int64)
        age = np.zeros((H, W), np.float32)
        for r in range(H):
            for c in range(W):
                for i in reversed(range(len(ep))):
                    if vis_f[i][r, c]:
                        last[r, c] = ep[i]["army"].reshape(H, W)[r, c] if en_f[i][r, c] else 0
                        break
                if vis[r, c]:
                    continue
                for i in reversed(range(len(ep))):
                    if vis_f[i][r, c] and en_f[i][r, c]:
                        age[r, c] = np.float32(np.log1p(float(turn - int(ep[i]["turn"]))) / 5.0)
                        break
        o = out[p]
        o[0] = np.where(vis, army, 0)
        o[1] = np.where(owner == p, army, 0)
        o[2] = np.where(vis & en, army, 0)
        o[3] = np.where(vis & (owner < 0), army, 0)
        o[4], o[5], o[6], o[7], o[8] = seen, en_seen, g_seen, c_seen, m_seen
        o[9] = vis & (owner < 0) & (typ != oracle.T_MOUNTAIN)
        o[10] = owner == p
        o[11] = vis & en
        o[12] = ~vis
        o[13] = ~vis & ((typ == oracle.T_MOUNTAIN) | (typ == oracle.T_CASTLE) | g_seen)
        o[14] = turn
        o[15] = np.float32((turn % 50) / 50.0)
        o[16] = land[p]
        o[17] = np.float32(tot[p])
        o[18] = sum(land[q] for q in enemies)
        o[19] = np.float32(sum(tot[q] for q in enemies))
        o[20] = last
        o[21] = age
        o[22] = (cc / (W - 1)).astype(np.float32)
        o[23] = (rr / (H - 1)).astype(np.float32)

        def chans(t):
            f = by_turn(t)
            if f is None:
                return np.zeros((H, W), np.int64), np.zeros((H, W), np.int64)
            a = f["army"].reshape(H, W).astype(np.int64)
            own = np.where(f["owner"].reshape(H, W) == p, a, 0)
            emy = np.where(vis_map(f, p, mode, P, H, W) & enemy_map(f, p, mode, P, H, W), a, 0)
            return own, emy

        for k in range(HH):
            o0, e0 = chans(turn - k)
            o1, e1 = chans(turn - k - 1)
            o[24 + k] = o0 - o1
            o[24 + HH + k] = e0 - e1
    return out


def definitional_tokens(frames, mode, P, H, W):
    """Temporal tokens of the last frame: for each player the enemies' army
    total (row 0) and land (row 1) at turns t-511 .. t, 0 where no frame of
    the episode has that turn."""
    cur = frames[-1]
    ep = [f for f in frames if f["episode"] == cur["episode"]]
    turn = int(cur["turn"])
    win = oracle.TOKEN_WINDOW
    tok = np.zeros((P, 2, win), np.float32)
    for f in ep:                                   # later records of a turn win
        j = int(f["turn"]) - (turn - win + 1)
        if not 0 <= j < win:
            continue
        owner, army = f["owner"], f["army"].astype(np.int64)
        for p in range(P):
            enemies = [q for q in range(P) if q not in team_of(mode, p, P)]
            sel = np.isin(owner, enemies)
            tok[p, 0, j] = np.float32(army[sel].sum())
            tok[p, 1, j] = np.float32(sel.sum())
    return tok


def env_state(st, e):
    return {k: st[k][e].copy() for k in ("owner", "army", "type", "turn", "episode")}


def run_case(H, W, mode, P, E, steps, seed, record_every=1, repeat_every=0, **prm):
    cfg = oracle.Config(H=H, W=W, mode=mode, P=P, mountain_thresh=workloads.mountain_thresh(1, 5),
                        city_army_min=40, city_army_max=50, auto_reset=1, seed=seed, env_base=0, **prm)
    st, _ = oracle.reset(cfg, E)
    mem = oracle.feature_memory(E)
    hist = [[] for _ in range(E)]
    checked = 0
    for t in range(steps):
        if t % record_every == 0:
            for e in range(E):
                hist[e].append(env_state(st, e))
            f, tok = oracle.features(cfg, st, mem, tokens=True)
            if repeat_every and t % repeat_every == 0:          # recording a turn twice changes nothing
                f2, tok2 = oracle.features(cfg, st, mem, tokens=True)
                assert np.array_equal(f2, f) and np.array_equal(tok2, tok)
            for e in range(E):
                want = definitional(hist[e], mode, P, H, W)
                np.testing.assert_array_equal(f[e], want, err_msg=f"step {t} env {e}")
                np.testing.assert_array_equal(tok[e], definitional_tokens(hist[e], mode, P, H, W),
                                              err_msg=f"tokens step {t} env {e}")
                checked += 1
        oracle.step(cfg, st, oracle.sample(cfg, st, seed + 1, t))
    return checked, st


@pytest.mark.parametrize("H,W,mode,P,E,steps,prm", [
    (5, 6, oracle.MODE_1V1, 2, 3, 60, dict(cities_min=1, cities_max=2, min_general_dist=3)),
    (6, 6, oracle.MODE_2V2, 4, 2, 50, dict(cities_min=1, cities_max=2, min_general_dist=2)),
    (4, 4, oracle.MODE_FFA, 3, 4, 80, dict(cities_min=0, cities_max=1, min_general_dist=2)),
])
def test_features_match_definition(H, W, mode, P, E, steps, prm):
    checked, st = run_case(H, W, mode, P, E, steps, seed=H * 10 + W, repeat_every=7, **prm)
    assert checked == E * steps


def test_features_skipped_frames_count_as_empty():
    """Recording every third step: the delta stacks see missing turns as
    empty boards (the definitional recomputation only knows recorded
    frames)."""
    run_case(5, 5, oracle.MODE_1V1, 2, 3, 45, seed=8, record_every=3, cities_min=1, cities_max=2,
             min_general_dist=3)


def test_features_episode_boundary_and_memory_content():
    """Small FFA maps end quickly: memories restart with every new episode;
    the enemy-age channel gets exercised."""
    cfg = oracle.Config(H=4, W=4, mode=oracle.MODE_FFA, P=3, mountain_thresh=workloads.mountain_thresh(1, 5),
                        cities_min=0, cities_max=1, city_army_min=40, city_army_max=50, min_general_dist=2,
                        auto_reset=1, seed=3, env_base=0)
    st, _ = oracle.reset(cfg, 8)
    mem = oracle.feature_memory(8)
    episodes, ages = 0, 0
    prev_ep = st["episode"].copy()
    for t in range(300):
        f = oracle.features(cfg, st, mem)
        ages += int((f[:, :, 21] > 0).sum())
        oracle.step(cfg, st, oracle.sample(cfg, st, 4, t))
        episodes += int((st["episode"] != prev_ep).sum())
        prev_ep = st["episode"].copy()
        f2 = oracle.features(cfg, st, mem)
        fresh = st["turn"] == 0
        # a new episode: nothing remembered beyond the current frame
        for e in np.flatnonzero(fresh):
            for p in range(cfg.P):
                vis = f2[e, p, 12] == 0
                assert np.array_equal(f2[e, p, 4] > 0, vis)
                assert not f2[e, p, 21].any()
                assert np.array_equal(f2[e, p, 24], f2[e, p, 1])       # delta against the empty board
                assert not f2[e, p, 25:31].any()
    assert episodes >= 4 and ages > 0


def test_features_closed_forms_and_obs_agreement():
    """Channels that restate the 8-channel observation or the scoreboard,
    coordinates in [0, 1], the timestep channels."""
    cfg = oracle.Config(H=7, W=5, mode=oracle.MODE_2V2, P=4, mountain_thresh=workloads.mountain_thresh(1, 5),
                        cities_min=1, cities_max=3, city_army_min=40, city_army_max=50, min_general_dist=2,
                        auto_reset=1, seed=11, env_base=0)
    st, _ = oracle.reset(cfg, 5)
    mem = oracle.feature_memory(5)
    for t in range(40):
        oracle.step(cfg, st, oracle.sample(cfg, st, 12, t))
        f = oracle.features(cfg, st, mem)
        obs = oracle.observe(cfg, st)
        land, army = oracle.scoreboard(cfg, st)
        assert np.array_equal(f[:, :, 10], obs[:, :, 0])
        assert np.array_equal(f[:, :, 11], obs[:, :, 1])
        assert np.array_equal(f[:, :, 9], obs[:, :, 2])
        assert np.array_equal(f[:, :, 12], obs[:, :, 6])
        assert np.array_equal(np.minimum(f[:, :, 0], 255), obs[:, :, 7])
        for p in range(cfg.P):
            assert np.array_equal(f[:, p, 16, 0, 0], land[:, p])
            assert np.array_equal(f[:, p, 17, 0, 0], army[:, p].astype(np.float32))
            enemies = [q for q in range(cfg.P) if q % 2 != p % 2]
            assert np.array_equal(f[:, p, 18, 0, 0], land[:, enemies].sum(1))
        assert np.array_equal(f[0, 0, 22, 0], np.linspace(0, 1, cfg.W, dtype=np.float64).astype(np.float32))
        assert np.array_equal(f[0, 0, 23, :, 0], np.linspace(0, 1, cfg.H, dtype=np.float64).astype(np.float32))
        assert np.all(f[:, :, 14] == st["turn"][:, None, None, None])
        assert np.all(f[:, :, 15] == (st["turn"] % 50 / 50.0).astype(np.float32)[:, None, None, None])
        # own army = army on own cells; own + ally + enemy + neutral (visible) = armies channel
        assert np.array_equal(f[:, :, 1], f[:, :, 1] * f[:, :, 10])


def test_tokens_window_slides_past_512_turns():
    """A 1v1 episode longer than the window: the oldest turns drop out.  Each
    turn is recorded twice, which must not shorten the window."""
    cfg = oracle.Config(H=8, W=8, mode=oracle.MODE_1V1, P=2, mountain_thresh=workloads.mountain_thresh(1, 5),
                        cities_min=1, cities_max=2, city_army_min=40, city_army_max=50, min_general_dist=6,
                        auto_reset=0, seed=13, env_base=0)
    st, _ = oracle.reset(cfg, 3)
    mem = oracle.feature_memory(3)
    hist = [[] for _ in range(3)]
    for t in range(700):
        for e in range(3):
            hist[e].append({k: st[k][e].copy() for k in ("owner", "army", "type", "turn", "episode")})
        oracle.features(cfg, st, mem)
        f, tok = oracle.features(cfg, st, mem, tokens=True)
        if t in (0, 1, 511, 512, 600, 699):
            for e in range(3):
                np.testing.assert_array_equal(tok[e], definitional_tokens(hist[e], cfg.mode, 2, 8, 8))
        oracle.step(cfg, st, oracle.sample(cfg, st, 14, t))
    assert (st["turn"] >= 600).any()
    e = int(np.argmax(st["turn"]))
    assert tok[e, 0, 1, -1] == f[e, 0, 18, 0, 0]           # newest token entry = current scoreboard channel
