"""CPU oracle of the Generals.io environment step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package.  The product path (``paper_2606_23348_amd``)
never imports it, and this package never imports the product path.

The simulator itself is plain C in ``oracle.c`` (one thread, no SIMD); this
module only marshals numpy arrays in the public host-state format:

    owner   int8   [E, H*W]   -1 = neutral, else player id
    army    int32  [E, H*W]
    type    uint8  [E, H*W]   0 plain, 1 mountain, 2 castle (city), 3 general
    turn    int32  [E]
    episode uint32 [E]
    alive   uint8  [E]        bit p set while player p still has a general
    finished uint8 [E]        1 once a game ended with auto-reset off
    gpos    int16  [E, P]     cell index of each player's original general
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODE_1V1, MODE_2V2, MODE_FFA = 0, 1, 2
T_PLAIN, T_MOUNTAIN, T_CASTLE, T_GENERAL = 0, 1, 2, 3
D_MAPGEN, D_ACTIONS, D_PREGROW = 1, 2, 3


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no vectoriser tricks)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("P", ctypes.c_int32), ("mountain_thresh", ctypes.c_uint32),
                ("cities_min", ctypes.c_int32), ("cities_max", ctypes.c_int32),
                ("city_army_min", ctypes.c_int32), ("city_army_max", ctypes.c_int32),
                ("min_general_dist", ctypes.c_int32), ("auto_reset", ctypes.c_int32),
                ("pregrow", ctypes.c_int32), ("seed", ctypes.c_uint64), ("env_base", ctypes.c_uint64),
                ("generator", ctypes.c_int32), ("max_general_dist", ctypes.c_int32),
                ("castle_radius", ctypes.c_int32), ("pad", ctypes.c_int32), ("env_ids", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        vp, i32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
        _lib.orc_philox4x64_10.argtypes = [vp, vp, vp]
        _lib.orc_philox4x64_10.restype = None
        _lib.orc_draw.argtypes = [u64] * 6
        _lib.orc_draw.restype = ctypes.c_uint32
        _lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
        _lib.orc_philox4x32_10.restype = None
        _lib.orc_actor_draw.argtypes = [u64, u64, u64, ctypes.c_int]
        _lib.orc_actor_draw.restype = ctypes.c_uint32
        _lib.orc_reset_batch.argtypes = [vp, i32, vp, vp]
        _lib.orc_step_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        _lib.orc_observe_batch.argtypes = [vp, i32, vp, vp]
        _lib.orc_scoreboard_batch.argtypes = [vp, i32, vp, vp, vp]
        _lib.orc_sample_batch.argtypes = [vp, i32, vp, u64, u64, vp]
        _lib.orc_run.argtypes = [vp, i32, vp, u64, u64, i32, vp, vp, vp, vp]
        _lib.orc_fmem_bytes.argtypes = []
        _lib.orc_fmem_bytes.restype = ctypes.c_int64
        _lib.orc_features_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        for f in ("orc_reset_batch", "orc_step_batch", "orc_observe_batch",
                  "orc_scoreboard_batch", "orc_sample_batch", "orc_run"):
            getattr(_lib, f).restype = ctypes.c_int
    return _lib


@dataclass
class Config:
    """Shape, mode and generator parameters of a batch of identical envs."""
    H: int
    W: int
    mode: int = MODE_1V1
    P: int = 2
    mountain_thresh: int = (2 ** 32) // 5
    cities_min: int = 9
    cities_max: int = 11
    city_army_min: int = 40
    city_army_max: int = 50
    min_general_dist: int = 9
    auto_reset: int = 1
    pregrow: int = 0
    seed: int = 0
    env_base: int = 0
    generator: int = 0            # 0 synthetic (R14), 1 official rules (R18)
    max_general_dist: int = 0     # R18 spawn-distance cap (0: none)
    castle_radius: int = 6        # R18
    env_ids: np.ndarray | None = None   # uint64 [E]: global id of each env (None: env_base + e)

    def _c(self) -> _Cfg:
        ids = None
        if self.env_ids is not None:
            if self.env_ids.dtype != np.uint64 or not self.env_ids.flags["C_CONTIGUOUS"]:
                raise TypeError("env_ids must be a C-contiguous uint64 array")
            ids = self.env_ids.ctypes.data
        return _Cfg(self.H, self.W, self.mode, self.P, self.mountain_thresh, self.cities_min,
                    self.cities_max, self.city_army_min, self.city_army_max,
                    self.min_general_dist, self.auto_reset, self.pregrow, self.seed, self.env_base,
                    self.generator, self.max_general_dist, self.castle_radius, 0, ids)


def empty_state(cfg: Config, E: int) -> dict:
    HW = cfg.H * cfg.W
    return {
        "owner": np.full((E, HW), -1, np.int8),
        "army": np.zeros((E, HW), np.int32),
        "type": np.zeros((E, HW), np.uint8),
        "turn": np.zeros(E, np.int32),
        "episode": np.zeros(E, np.uint32),
        "alive": np.zeros(E, np.uint8),
        "finished": np.zeros(E, np.uint8),
        "gpos": np.zeros((E, cfg.P), np.int16),
    }


def _batch(st: dict) -> _Batch:
    for k, dt in (("owner", np.int8), ("army", np.int32), ("type", np.uint8), ("turn", np.int32),
                  ("episode", np.uint32), ("alive", np.uint8), ("finished", np.uint8),
                  ("gpos", np.int16)):
        a = st[k]
        if a.dtype != dt or not a.flags["C_CONTIGUOUS"]:
            raise TypeError(f"host state field {k} must be C-contiguous {np.dtype(dt).name}")
    return _Batch(*(st[k].ctypes.data for k in
                    ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")))


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _cfg(cfg: Config, E: int) -> _Cfg:
    if cfg.env_ids is not None and cfg.env_ids.shape != (E,):
        raise ValueError(f"env_ids holds {cfg.env_ids.shape} ids for a batch of {E} envs")
    return cfg._c()


def _check(rc: int):
    if rc != 0:
        raise ValueError("oracle rejected the configuration")


def reset(cfg: Config, E: int):
    """Fresh maps for envs env_base..env_base+E-1.  Returns (state, attempts)."""
    st = empty_state(cfg, E)
    att = np.zeros(E, np.int32)
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_reset_batch(ctypes.byref(c), E, ctypes.byref(b), _ptr(att)))
    return st, att


def step(cfg: Config, st: dict, actions: np.ndarray):
    """Advance every env one step in place.  Returns (rewards [E,P] int32, done [E] uint8)."""
    E = st["turn"].shape[0]
    actions = np.ascontiguousarray(actions, np.int32).reshape(E, cfg.P)
    rew = np.zeros((E, cfg.P), np.int32)
    done = np.zeros(E, np.uint8)
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_step_batch(ctypes.byref(c), E, ctypes.byref(b), _ptr(actions), _ptr(rew), _ptr(done)))
    return rew, done


def observe(cfg: Config, st: dict) -> np.ndarray:
    E = st["turn"].shape[0]
    obs = np.zeros((E, cfg.P, 8, cfg.H, cfg.W), np.uint8)
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_observe_batch(ctypes.byref(c), E, ctypes.byref(b), _ptr(obs)))
    return obs


def scoreboard(cfg: Config, st: dict):
    E = st["turn"].shape[0]
    land = np.zeros((E, cfg.P), np.int32)
    army = np.zeros((E, cfg.P), np.int64)
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_scoreboard_batch(ctypes.byref(c), E, ctypes.byref(b), _ptr(land), _ptr(army)))
    return land, army


def sample(cfg: Config, st: dict, seed_act: int, step_idx: int) -> np.ndarray:
    E = st["turn"].shape[0]
    act = np.zeros((E, cfg.P), np.int32)
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_sample_batch(ctypes.byref(c), E, ctypes.byref(b), seed_act, step_idx, _ptr(act)))
    return act


def run(cfg: Config, st: dict, seed_act: int, step0: int, n_steps: int):
    """sample -> step -> observe, n_steps times (the oracle's whole loop)."""
    E = st["turn"].shape[0]
    act = np.zeros((E, cfg.P), np.int32)
    rew = np.zeros((E, cfg.P), np.int32)
    done = np.zeros(E, np.uint8)
    obs = np.zeros((E, cfg.P, 8, cfg.H, cfg.W), np.uint8)
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_run(ctypes.byref(c), E, ctypes.byref(b), seed_act, step0, n_steps,
                         _ptr(act), _ptr(rew), _ptr(done), _ptr(obs)))
    return act, rew, done, obs


FEAT_CHANNELS = 38
TOKEN_WINDOW = 512


def feature_memory(E: int) -> np.ndarray:
    """Zero-filled per-env memory of the 38-channel features (one episode's
    running masks and the last 8 frames)."""
    return np.zeros((E, int(lib().orc_fmem_bytes())), np.uint8)


def features(cfg: Config, st: dict, mem: np.ndarray, tokens: bool = False):
    """Record the current frame of every env into `mem` and return the
    38-channel features float32 [E][P][38][H][W] (Appendix A, reading R17);
    with tokens=True also the temporal tokens float32 [E][P][2][512]
    (enemies' army total, then land, for the last 512 turns)."""
    E = st["turn"].shape[0]
    assert mem.shape[0] == E and mem.flags["C_CONTIGUOUS"]
    out = np.zeros((E, cfg.P, FEAT_CHANNELS, cfg.H, cfg.W), np.float32)
    tok = np.zeros((E, cfg.P, 2, TOKEN_WINDOW), np.float32) if tokens else None
    c, b = _cfg(cfg, E), _batch(st)
    _check(lib().orc_features_batch(ctypes.byref(c), E, ctypes.byref(b), _ptr(mem), _ptr(out),
                                    _ptr(tok) if tokens else None))
    return (out, tok) if tokens else out


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, np.uint64))
    k = np.ascontiguousarray(np.asarray(key, np.uint64))
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed: int, domain: int, c0: int, c1: int, c2: int, j: int) -> int:
    return int(lib().orc_draw(seed, domain, c0, c1, c2, j))


def philox32(ctr, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter and a 2-word key (uint32)."""
    c = np.ascontiguousarray(np.asarray(ctr, np.uint32))
    k = np.ascontiguousarray(np.asarray(key, np.uint32))
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def actor_draw(seed_act: int, env_id: int, step: int, p: int) -> int:
    """The random actor's 32-bit draw for player p (reading R15)."""
    return int(lib().orc_actor_draw(seed_act, env_id, step, p))
