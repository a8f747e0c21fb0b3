"""MI355X (gfx950) batched Generals.io environment step -- Python binding.

A thin ctypes layer over ``libgenerals.so`` (declared in ``include/generals.h``)
with the same function names.  It only marshals arguments: torch tensors
supply device memory (``data_ptr``) and HIP streams (``cuda_stream``); every
step of the environment runs in the library's HIP kernels.  There is no CPU
fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgenerals.so")

GEN_OK, GEN_EINVAL, GEN_ENOMEM, GEN_EHIP, GEN_EBUDGET, GEN_EBUSY, GEN_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
GEN_1V1, GEN_2V2, GEN_FFA = 0, 1, 2
GEN_PLAIN, GEN_MOUNTAIN, GEN_CASTLE, GEN_GENERAL = 0, 1, 2, 3
GEN_LAYOUT_VERSION = 1


class GenError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gen error {code}: {msg}")
        self.code = code


class gen_params(ctypes.Structure):
    _fields_ = [("n_players", ctypes.c_int32), ("mountain_thresh", ctypes.c_uint32),
                ("cities_min", ctypes.c_int32), ("cities_max", ctypes.c_int32),
                ("city_army_min", ctypes.c_int32), ("city_army_max", ctypes.c_int32),
                ("min_general_dist", ctypes.c_int32), ("auto_reset", ctypes.c_int32),
                ("pregrow", ctypes.c_int32), ("generator", ctypes.c_int32),
                ("max_general_dist", ctypes.c_int32), ("castle_radius", ctypes.c_int32),
                ("obs_layout", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class gen_state(ctypes.Structure):
    _fields_ = [("version", ctypes.c_uint32), ("n_envs", ctypes.c_int32), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("mode", ctypes.c_int32), ("n_players", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("env_base", ctypes.c_uint64), ("params", gen_params),
                ("off_scalars", ctypes.c_uint64), ("off_owner", ctypes.c_uint64),
                ("off_type", ctypes.c_uint64), ("off_army", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("d_buf", ctypes.c_void_p)]


class gen_host_state(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("owner", "army", "type", "turn", "episode", "alive", "finished", "gpos")]


class gen_env_spec(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("H", "W", "mode", "n_players", "cities_min", "cities_max", "min_general_dist", "reserved")]


class gen_pool_info(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("max_cells", ctypes.c_int32), ("state_bytes", ctypes.c_uint64),
                ("obs_bytes", ctypes.c_uint64), ("n_actions", ctypes.c_uint64),
                ("work_list_off", ctypes.c_uint64), ("work_list_bytes", ctypes.c_uint64)]


class gen_pool_tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("waves_per_group", "grid", "order", "reserved")]


class gen_pool_bucket(ctypes.Structure):
    _fields_ = [("n_players", ctypes.c_int32), ("words", ctypes.c_int32), ("n_envs", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("waves_per_env", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class gen_group_buffers(ctypes.Structure):
    _fields_ = [("state_off", ctypes.c_uint64), ("obs_off", ctypes.c_uint64), ("actions_off", ctypes.c_uint64),
                ("rewards_off", ctypes.c_uint64), ("dones_off", ctypes.c_uint64), ("obs_bytes", ctypes.c_uint64),
                ("n_actions", ctypes.c_uint64), ("n_envs", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pool", ctypes.c_void_p)]


class gen_server_stats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("frames", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("groups_open", ctypes.c_uint64), ("groups_queued", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("lat_p50_us", ctypes.c_double), ("lat_p99_us", ctypes.c_double), ("lat_mean_us", ctypes.c_double),
                ("envs_per_launch", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("groups_pending", ctypes.c_uint64), ("lat_samples", ctypes.c_uint64), ("lat_max_us", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgenerals.so (torch first, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        _lib = load_library(LIB_PATH)
    return _lib


def load_library(path: str) -> ctypes.CDLL:
    """Open a build of the library at `path` and declare its signatures."""
    import torch  # noqa: F401  -- loads the HIP runtime the library binds to
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "(python -m paper_2606_23348_amd.build)")
    L = ctypes.CDLL(path)
    vp, i32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    P = ctypes.POINTER
    L.gen_version.argtypes, L.gen_version.restype = [], ctypes.c_int
    L.gen_last_error.argtypes, L.gen_last_error.restype = [], ctypes.c_char_p
    L.gen_default_params.argtypes = [i32, i32, P(gen_params)]
    L.gen_layout.argtypes = [i32, i32, i32, i32, P(gen_params), u64, P(gen_state)]
    L.gen_state_bytes.argtypes, L.gen_state_bytes.restype = [i32, i32, i32, i32, P(gen_params)], u64
    L.gen_reset.argtypes = [u64, u64, i32, i32, i32, i32, P(gen_params), vp, u64, vp, vp, P(gen_state)]
    L.gen_step.argtypes = [P(gen_state), vp, vp, vp, vp, vp, vp, vp]
    L.gen_sample_actions.argtypes = [P(gen_state), u64, u64, vp, vp]
    L.gen_step_sample.argtypes = [P(gen_state), vp, u64, u64, vp, vp, vp, vp, vp, vp]
    L.gen_observe.argtypes = [P(gen_state), vp, vp]
    L.gen_feat_mem_bytes.argtypes, L.gen_feat_mem_bytes.restype = [P(gen_state)], u64
    L.gen_features.argtypes = [P(gen_state), vp, u64, vp, vp, vp]
    L.gen_rollout.argtypes = [P(gen_state), vp, u64, i32, u64, u64, vp, vp, vp, vp, vp, vp]
    L.gen_get_state.argtypes = [P(gen_state), P(gen_host_state), vp]
    L.gen_set_state.argtypes = [P(gen_state), P(gen_host_state), vp]
    L.gen_get_envs.argtypes = [P(gen_state), vp, i32, P(gen_host_state), vp]
    L.gen_pool_create.argtypes = [u64, u64, i32, vp, P(gen_params), P(vp)]
    L.gen_pool_destroy.argtypes = [vp]
    L.gen_pool_query.argtypes = [vp, P(gen_pool_info)]
    L.gen_pool_offsets.argtypes = [vp, vp, vp]
    L.gen_pool_get_tuning.argtypes = [vp, P(gen_pool_tuning)]
    L.gen_pool_set_tuning.argtypes = [vp, P(gen_pool_tuning), vp]
    L.gen_pool_buckets.argtypes = [vp, vp, i32, P(i32)]
    L.gen_pool_set_buckets.argtypes = [vp, vp, i32, vp]
    L.gen_pool_reset.argtypes = [vp, vp, u64, vp, vp, u64, vp]
    L.gen_pool_step.argtypes = [vp, vp, i32, u64, vp, vp, vp, vp]
    L.gen_pool_capture.argtypes = [vp, i32, vp, u64, vp, vp, vp, vp]
    L.gen_pool_replay.argtypes = [vp, vp]
    L.gen_pool_get_env.argtypes = [vp, i32, P(gen_host_state), vp]
    L.gen_pool_get_state.argtypes = [vp, P(gen_host_state), vp]
    L.gen_stream_copy.argtypes = [vp, vp, u64, vp]
    L.gen_stream_spread.argtypes = [vp, vp, u64, ctypes.c_uint32, vp]
    L.gen_get_envs_static.argtypes = [P(gen_state), vp, i32, P(gen_host_state), vp]
    L.gen_server_create.argtypes = [vp, u64, i32, i32, P(vp)]
    L.gen_server_destroy.argtypes = [vp]
    L.gen_server_open.argtypes = [vp, u64, u64, i32, vp, P(gen_params), i32, u64, P(ctypes.c_uint64)]
    L.gen_server_wait_admitted.argtypes = [vp, u64, ctypes.c_int64]
    L.gen_server_buffers.argtypes = [vp, u64, P(gen_group_buffers)]
    L.gen_server_submit.argtypes = [vp, u64, P(ctypes.c_uint64)]
    L.gen_server_wait.argtypes = [vp, u64, ctypes.c_int64]
    L.gen_server_close.argtypes = [vp, u64]
    L.gen_server_report.argtypes = [vp, P(gen_server_stats), i32]
    L.gen_server_set_batching.argtypes = [vp, ctypes.c_int64, ctypes.c_int64]
    L.gen_server_drive.argtypes = [vp, i32, i32, vp, vp, P(gen_params), u64, u64, vp, i32, ctypes.c_int64, i32,
                                   P(gen_server_stats)]
    for f in ("gen_default_params", "gen_layout", "gen_reset", "gen_step", "gen_step_sample", "gen_sample_actions",
              "gen_observe", "gen_features", "gen_rollout", "gen_get_state", "gen_set_state", "gen_get_envs", "gen_pool_create",
              "gen_pool_destroy", "gen_pool_query", "gen_pool_offsets", "gen_pool_get_tuning",
              "gen_pool_set_tuning", "gen_pool_buckets", "gen_pool_set_buckets", "gen_pool_reset", "gen_pool_step", "gen_pool_capture", "gen_pool_replay",
              "gen_pool_get_env", "gen_pool_get_state", "gen_stream_copy", "gen_stream_spread", "gen_get_envs_static", "gen_server_create", "gen_server_destroy", "gen_server_open", "gen_server_wait_admitted",
              "gen_server_buffers", "gen_server_submit", "gen_server_wait", "gen_server_close",
              "gen_server_report", "gen_server_set_batching", "gen_server_drive"):
        getattr(L, f).restype = ctypes.c_int
    return L


def gen_last_error() -> str:
    return lib().gen_last_error().decode()


def _check(rc: int):
    if rc != GEN_OK:
        raise GenError(rc, gen_last_error())


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def gen_version() -> int:
    return lib().gen_version()


def gen_default_params(mode: int, n_players: int = 0) -> gen_params:
    p = gen_params()
    _check(lib().gen_default_params(mode, n_players, ctypes.byref(p)))
    return p


def make_params(mode: int, n_players: int = 0, **kw) -> gen_params:
    """Defaults for `mode`, overridden by keyword fields of gen_params."""
    p = gen_default_params(mode, n_players if mode == GEN_FFA else 0)
    for k, v in kw.items():
        if k == "n_players":
            continue
        setattr(p, k, int(v))
    return p


def gen_layout(n_envs: int, H: int, W: int, mode: int, params: gen_params | None = None,
               seed: int = 0) -> gen_state:
    st = gen_state()
    _check(lib().gen_layout(n_envs, H, W, mode, ctypes.byref(params) if params else None, seed,
                            ctypes.byref(st)))
    return st


def gen_state_bytes(n_envs: int, H: int, W: int, mode: int, params: gen_params | None = None) -> int:
    return int(lib().gen_state_bytes(n_envs, H, W, mode, ctypes.byref(params) if params else None))


def gen_reset(seed: int, env_base: int, n_envs: int, H: int, W: int, mode: int, params: gen_params | None,
              buf, obs=None, stream=None) -> gen_state:
    st = gen_state()
    _check(lib().gen_reset(seed, env_base, n_envs, H, W, mode, ctypes.byref(params) if params else None,
                           _ptr(buf), buf.numel() * buf.element_size(), _ptr(obs), _stream(stream),
                           ctypes.byref(st)))
    st._keep = buf  # the descriptor refers to this tensor's memory
    return st


def gen_step(st: gen_state, actions, obs, rewards, dones, land=None, army=None, stream=None):
    _check(lib().gen_step(ctypes.byref(st), _ptr(actions), _ptr(obs), _ptr(rewards), _ptr(dones),
                          _ptr(land), _ptr(army), _stream(stream)))


def gen_step_sample(st: gen_state, actions, actor_seed: int, next_step_idx: int, obs, rewards, dones,
                    land=None, army=None, stream=None):
    """gen_step, then the random actor for step `next_step_idx` into `actions` (one launch)."""
    _check(lib().gen_step_sample(ctypes.byref(st), _ptr(actions), actor_seed, next_step_idx, _ptr(obs),
                                 _ptr(rewards), _ptr(dones), _ptr(land), _ptr(army), _stream(stream)))


def gen_sample_actions(st: gen_state, actor_seed: int, step_idx: int, actions, stream=None):
    _check(lib().gen_sample_actions(ctypes.byref(st), actor_seed, step_idx, _ptr(actions), _stream(stream)))


def gen_observe(st: gen_state, obs, stream=None):
    _check(lib().gen_observe(ctypes.byref(st), _ptr(obs), _stream(stream)))


def _host_arrays(E: int, HW: int, P: int) -> dict:
    return {
        "owner": np.zeros((E, HW), np.int8), "army": np.zeros((E, HW), np.int32),
        "type": np.zeros((E, HW), np.uint8), "turn": np.zeros(E, np.int32),
        "episode": np.zeros(E, np.uint32), "alive": np.zeros(E, np.uint8),
        "finished": np.zeros(E, np.uint8), "gpos": np.zeros((E, P), np.int16),
    }


_HOST_TYPES = {"owner": np.int8, "army": np.int32, "type": np.uint8, "turn": np.int32,
               "episode": np.uint32, "alive": np.uint8, "finished": np.uint8, "gpos": np.int16}


def _host_struct(h: dict) -> gen_host_state:
    for k, dt in _HOST_TYPES.items():
        a = h[k]
        if a.dtype != dt or not a.flags["C_CONTIGUOUS"]:
            raise TypeError(f"host state field {k} must be C-contiguous {np.dtype(dt).name}")
    return gen_host_state(*(h[k].ctypes.data for k in _HOST_TYPES))


FEAT_CHANNELS = 38
TOKEN_WINDOW = 512


def gen_feat_mem_bytes(st: gen_state) -> int:
    n = int(lib().gen_feat_mem_bytes(ctypes.byref(st)))
    if n == 0:
        raise GenError(GEN_EINVAL, gen_last_error())
    return n


def gen_features(st: gen_state, mem, feat, tokens=None, stream=None):
    _check(lib().gen_features(ctypes.byref(st), _ptr(mem), mem.numel() * mem.element_size(), _ptr(feat),
                              _ptr(tokens), _stream(stream)))


def gen_rollout(st: gen_state, mem, n_steps: int, actor_seed: int, step0: int, feat, actions, rewards, dones,
                tokens=None, stream=None):
    _check(lib().gen_rollout(ctypes.byref(st), _ptr(mem), mem.numel() * mem.element_size(), n_steps, actor_seed,
                             step0, _ptr(feat), _ptr(tokens), _ptr(actions), _ptr(rewards), _ptr(dones),
                             _stream(stream)))


def gen_get_state(st: gen_state, stream=None) -> dict:
    """Blocking copy of the device state into the public host format (numpy)."""
    h = _host_arrays(st.n_envs, st.H * st.W, st.n_players)
    hs = _host_struct(h)
    _check(lib().gen_get_state(ctypes.byref(st), ctypes.byref(hs), _stream(stream)))
    return h


def gen_get_envs(st: gen_state, env_ids, stream=None) -> dict:
    """Blocking copy of the listed envs (row i = env env_ids[i])."""
    ids = np.ascontiguousarray(np.asarray(env_ids, np.int32))
    h = _host_arrays(len(ids), st.H * st.W, st.n_players)
    hs = _host_struct(h)
    _check(lib().gen_get_envs(ctypes.byref(st), ids.ctypes.data, len(ids), ctypes.byref(hs), _stream(stream)))
    return h


def gen_stream_copy(dst, src, stream=None):
    """Streaming copy of src into dst (same byte size, 16-byte aligned)."""
    n = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == n
    _check(lib().gen_stream_copy(_ptr(dst), _ptr(src), n, _stream(stream)))


def gen_stream_spread(dst, src, k: int, stream=None):
    """Chunk i (16 bytes) of dst = chunk i // k of src: k bytes written per
    byte read (src holds at least ceil(chunks of dst / k) chunks); k = 0
    writes zeros and reads nothing (src may be None)."""
    n = dst.numel() * dst.element_size()
    assert k == 0 or (k >= 1 and src.numel() * src.element_size() * k >= n)
    _check(lib().gen_stream_spread(_ptr(dst), _ptr(src) if k else None, n, k, _stream(stream)))


def gen_get_envs_static(st: gen_state, env_ids, stream=None) -> dict:
    """gen_get_envs staged through the library's static device array (no
    device allocation)."""
    ids = np.ascontiguousarray(np.asarray(env_ids, np.int32))
    h = _host_arrays(len(ids), st.H * st.W, st.n_players)
    hs = _host_struct(h)
    _check(lib().gen_get_envs_static(ctypes.byref(st), ids.ctypes.data, len(ids), ctypes.byref(hs),
                                     _stream(stream)))
    return h


def gen_set_state(st: gen_state, h: dict, stream=None):
    hs = _host_struct(h)
    _check(lib().gen_set_state(ctypes.byref(st), ctypes.byref(hs), _stream(stream)))


def _filled(device):
    """Wait for the zero fills torch just queued on its current stream: the
    library may be called on another stream, which would not wait for them
    (and a late fill would overwrite what the library wrote)."""
    import torch
    torch.cuda.current_stream(torch.device(device)).synchronize()


class Batch:
    """Device tensors of one batch of identical envs (torch allocates; the
    library computes).  Convenience only: every method is one library call."""

    def __init__(self, n_envs: int, H: int, W: int, mode: int, params: gen_params | None = None,
                 seed: int = 0, env_base: int = 0, device: str = "cuda", with_obs: bool = True,
                 scoreboard: bool = False, stream=None):
        import torch
        lay = gen_layout(n_envs, H, W, mode, params, seed)
        P = lay.n_players
        self.n_envs, self.H, self.W, self.mode, self.P = n_envs, H, W, mode, P
        self.padded = params is not None and params.obs_layout == 1
        self.PS = plane_stride(H, W, P) if self.padded else H * W
        # zero-filled, so alignment padding the library never writes is deterministic
        self.buf = torch.zeros(lay.bytes, dtype=torch.uint8, device=device)
        obs_shape = (n_envs, P, 8, self.PS) if self.padded else (n_envs, P, 8, H, W)
        self.obs = torch.zeros(obs_shape, dtype=torch.uint8, device=device) if with_obs else None
        self.actions = torch.zeros((n_envs, P), dtype=torch.int32, device=device)
        self.rewards = torch.zeros((n_envs, P), dtype=torch.int32, device=device)
        self.dones = torch.zeros(n_envs, dtype=torch.uint8, device=device)
        self.land = torch.zeros((n_envs, P), dtype=torch.int32, device=device) if scoreboard else None
        self.army = torch.zeros((n_envs, P), dtype=torch.int64, device=device) if scoreboard else None
        self.feat = self.fmem = self.tokens = None   # 38-channel features, allocated by features()
        _filled(self.buf.device)
        self.st = gen_reset(seed, env_base, n_envs, H, W, mode, params, self.buf, self.obs, stream)

    def obs_dense(self) -> np.ndarray:
        """The observation on the host as uint8 [E, P, 8, H, W] (without the
        plane padding of obs_layout 1)."""
        o = self.obs.cpu().numpy()
        if self.padded:
            o = np.ascontiguousarray(o[..., :self.H * self.W])
        return o.reshape(self.n_envs, self.P, 8, self.H, self.W)

    def sample(self, actor_seed: int, step_idx: int, stream=None):
        gen_sample_actions(self.st, actor_seed, step_idx, self.actions, stream)

    def step(self, stream=None):
        gen_step(self.st, self.actions, self.obs, self.rewards, self.dones, self.land, self.army, stream)

    def step_sample(self, actor_seed: int, next_step_idx: int, stream=None):
        gen_step_sample(self.st, self.actions, actor_seed, next_step_idx, self.obs, self.rewards, self.dones,
                        self.land, self.army, stream)

    def observe(self, stream=None):
        gen_observe(self.st, self.obs, stream)

    def features(self, tokens: bool = False, stream=None):
        """The 38-channel features float32 [E][P][38][H][W] of the current
        state into self.feat and, with tokens=True, the temporal tokens
        float32 [E][P][2][512] into self.tokens (allocated, with the
        zero-filled memory, on first use).  Call once after reset and after
        every step."""
        import torch
        dev = self.buf.device
        if self.feat is None:
            self.fmem = torch.zeros(gen_feat_mem_bytes(self.st), dtype=torch.uint8, device=dev)
            self.feat = torch.zeros((self.n_envs, self.P, FEAT_CHANNELS, self.H, self.W), dtype=torch.float32,
                                    device=dev)
            _filled(dev)
        if tokens and self.tokens is None:
            self.tokens = torch.zeros((self.n_envs, self.P, 2, TOKEN_WINDOW), dtype=torch.float32, device=dev)
            _filled(dev)
        gen_features(self.st, self.fmem, self.feat, self.tokens if tokens else None, stream)

    def rollout(self, n_steps: int, actor_seed: int, step0: int, tokens: bool = False, out: dict | None = None,
                stream=None) -> dict:
        """n_steps of features -> random actor -> step into a rollout buffer
        (allocated unless `out` holds one from an earlier call):
        feat [T][E][P][38][H][W], tokens [T][E][P][2][512] (tokens=True),
        actions/rewards [T][E][P], dones [T][E]."""
        import torch
        dev = self.buf.device
        if self.fmem is None:
            self.fmem = torch.zeros(gen_feat_mem_bytes(self.st), dtype=torch.uint8, device=dev)
            _filled(dev)
        E, P, T = self.n_envs, self.P, n_steps
        if out is None:
            out = {"feat": torch.empty((T, E, P, FEAT_CHANNELS, self.H, self.W), dtype=torch.float32, device=dev),
                   "actions": torch.empty((T, E, P), dtype=torch.int32, device=dev),
                   "rewards": torch.empty((T, E, P), dtype=torch.int32, device=dev),
                   "dones": torch.empty((T, E), dtype=torch.uint8, device=dev)}
            if tokens:
                out["tokens"] = torch.empty((T, E, P, 2, TOKEN_WINDOW), dtype=torch.float32, device=dev)
        gen_rollout(self.st, self.fmem, T, actor_seed, step0, out["feat"], out["actions"], out["rewards"],
                    out["dones"], out.get("tokens"), stream)
        return out

    def get_state(self, stream=None) -> dict:
        return gen_get_state(self.st, stream)

    def get_envs(self, env_ids, stream=None) -> dict:
        return gen_get_envs(self.st, env_ids, stream)

    def set_state(self, h: dict, stream=None):
        gen_set_state(self.st, h, stream)


# ---------------------------------------------------------------------------- batched pool
SPEC_FIELDS = ("H", "W", "mode", "P", "cities_min", "cities_max", "min_general_dist")


def gen_pool_create(seed: int, env_base: int, specs: dict, common: gen_params | None = None) -> ctypes.c_void_p:
    """specs: dict of equal-length integer arrays with keys SPEC_FIELDS."""
    n = len(specs["H"])
    arr = (gen_env_spec * n)()
    for i in range(n):
        arr[i] = gen_env_spec(int(specs["H"][i]), int(specs["W"][i]), int(specs["mode"][i]), int(specs["P"][i]),
                              int(specs["cities_min"][i]), int(specs["cities_max"][i]),
                              int(specs["min_general_dist"][i]), 0)
    h = ctypes.c_void_p()
    _check(lib().gen_pool_create(seed, env_base, n, arr, ctypes.byref(common) if common else None,
                                 ctypes.byref(h)))
    return h


class Pool:
    """Device buffers of one batched pool (torch allocates, the library
    computes).  Every method is one library call."""

    def __init__(self, specs: dict, common: gen_params | None = None, seed: int = 0, env_base: int = 0,
                 device: str = "cuda", with_obs: bool = True):
        import torch
        self.specs = {k: np.asarray(specs[k]) for k in SPEC_FIELDS}
        self.handle = gen_pool_create(seed, env_base, self.specs, common)
        info = gen_pool_info()
        _check(lib().gen_pool_query(self.handle, ctypes.byref(info)))
        self.n = info.n_envs
        self.info = info
        self.obs_off = np.zeros(self.n, np.uint64)
        self.act_off = np.zeros(self.n, np.uint32)
        _check(lib().gen_pool_offsets(self.handle, self.obs_off.ctypes.data, self.act_off.ctypes.data))
        # zero-filled, so alignment padding the library never writes is deterministic
        self.buf = torch.zeros(info.state_bytes, dtype=torch.uint8, device=device)
        self.obs = torch.zeros(max(info.obs_bytes, 16), dtype=torch.uint8, device=device) if with_obs else None
        self.actions = torch.zeros(info.n_actions, dtype=torch.int32, device=device)
        self.rewards = torch.zeros(info.n_actions, dtype=torch.int32, device=device)
        self.dones = torch.zeros(self.n, dtype=torch.uint8, device=device)
        _filled(device)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gen_pool_destroy(self.handle)
            self.handle = None

    def reset(self, actor_seed: int | None = None, stream=None):
        _check(lib().gen_pool_reset(self.handle, _ptr(self.buf), self.buf.numel(), _ptr(self.obs),
                                    _ptr(self.actions) if actor_seed is not None else None,
                                    actor_seed or 0, _stream(stream)))

    def step(self, actor_seed: int | None = None, stream=None):
        _check(lib().gen_pool_step(self.handle, _ptr(self.actions), 1 if actor_seed is not None else 0,
                                   actor_seed or 0, _ptr(self.obs), _ptr(self.rewards), _ptr(self.dones),
                                   _stream(stream)))

    def capture(self, k_steps: int, actor_seed: int, stream):
        _check(lib().gen_pool_capture(self.handle, k_steps, _ptr(self.actions), actor_seed, _ptr(self.obs),
                                      _ptr(self.rewards), _ptr(self.dones), _stream(stream)))

    def replay(self, stream=None):
        _check(lib().gen_pool_replay(self.handle, _stream(stream)))

    def tuning(self) -> dict:
        t = gen_pool_tuning()
        _check(lib().gen_pool_get_tuning(self.handle, ctypes.byref(t)))
        return {"waves_per_group": t.waves_per_group, "grid": t.grid, "order": t.order}

    def set_tuning(self, waves_per_group: int = 1, grid: int = 0, order: int = 0, stream=None):
        t = gen_pool_tuning(waves_per_group, grid, order, 0)
        _check(lib().gen_pool_set_tuning(self.handle, ctypes.byref(t), _stream(stream)))

    def buckets(self) -> list:
        """The pool's size buckets: dicts of n_players, words, n_envs and the
        packing (waves_per_group, waves_per_env)."""
        n = ctypes.c_int32()
        _check(lib().gen_pool_buckets(self.handle, None, 0, ctypes.byref(n)))
        arr = (gen_pool_bucket * max(1, n.value))()
        _check(lib().gen_pool_buckets(self.handle, arr, n.value, ctypes.byref(n)))
        return [{k: getattr(arr[i], k) for k in ("n_players", "words", "n_envs", "waves_per_group", "waves_per_env")}
                for i in range(n.value)]

    def set_buckets(self, table: list, stream=None):
        """Per-bucket packing: a list of dicts with n_players, words,
        waves_per_group and waves_per_env ([] clears it)."""
        arr = (gen_pool_bucket * max(1, len(table)))()
        for i, t in enumerate(table):
            arr[i] = gen_pool_bucket(int(t["n_players"]), int(t["words"]), 0, int(t["waves_per_group"]),
                                     int(t.get("waves_per_env", 1)))
        _check(lib().gen_pool_set_buckets(self.handle, arr, len(table), _stream(stream)))

    def get_env(self, e: int, stream=None) -> dict:
        HW = int(self.specs["H"][e]) * int(self.specs["W"][e])
        h = _host_arrays(1, HW, int(self.specs["P"][e]))
        hs = _host_struct(h)
        _check(lib().gen_pool_get_env(self.handle, e, ctypes.byref(hs), _stream(stream)))
        return h

    def get_state(self, stream=None) -> dict:
        """Every env in the ragged host format: owner/army/type [sum of H*W]
        (env e's cells from cell_off[e]), per-env scalars, gpos [n, 8]."""
        HW = self.specs["H"].astype(np.int64) * self.specs["W"].astype(np.int64)
        n_cells = int(HW.sum())
        h = {"owner": np.zeros(n_cells, np.int8), "army": np.zeros(n_cells, np.int32),
             "type": np.zeros(n_cells, np.uint8), "turn": np.zeros(self.n, np.int32),
             "episode": np.zeros(self.n, np.uint32), "alive": np.zeros(self.n, np.uint8),
             "finished": np.zeros(self.n, np.uint8), "gpos": np.zeros((self.n, 8), np.int16)}
        hs = _host_struct(h)
        _check(lib().gen_pool_get_state(self.handle, ctypes.byref(hs), _stream(stream)))
        h["cell_off"] = np.concatenate([[0], np.cumsum(HW)[:-1]]).astype(np.int64)
        return h

    def digest(self) -> str:
        """SHA-256 of every output and of the state except the work list
        (the one part of the state that depends on the packing)."""
        import hashlib
        h = hashlib.sha256()
        buf = self.buf.cpu().numpy()
        a, b = self.info.work_list_off, self.info.work_list_off + self.info.work_list_bytes
        h.update(buf[:a].tobytes())
        h.update(buf[b:].tobytes())
        for t in (self.obs, self.actions, self.rewards, self.dones):
            if t is not None:
                h.update(t.cpu().numpy().tobytes())
        return h.hexdigest()

    def env_obs(self, e: int):
        """Env e's observation [P, 8, H*W] (a strided view: planes are padded
        to a multiple of 32 bytes)."""
        return pool_env_obs(self.obs, int(self.obs_off[e]), *(int(self.specs[k][e]) for k in ("H", "W", "P")))

    def env_slice(self, e: int):
        a = int(self.act_off[e])
        return slice(a, a + int(self.specs["P"][e]))


def plane_stride(H: int, W: int, P: int) -> int:
    """Bytes between two planes of a padded observation block (pool envs,
    plain batches with obs_layout 1): H*W rounded up to 32 bytes, to 64 with
    more than 2 players."""
    return (H * W + 63) & ~63 if P > 2 else (H * W + 31) & ~31


def pool_env_obs(obs, off: int, H: int, W: int, P: int):
    """The [P, 8, H*W] observation of the pool env whose block starts at byte
    `off` of a ragged observation buffer (torch tensor or numpy array)."""
    PS = plane_stride(H, W, P)
    return obs[off:off + P * 8 * PS].reshape(P, 8, PS)[:, :, :H * W]


# ---------------------------------------------------------------------------- served form
def _spec_array(specs: dict, lo: int = 0, hi: int | None = None):
    hi = len(specs["H"]) if hi is None else hi
    arr = (gen_env_spec * (hi - lo))()
    for i in range(lo, hi):
        arr[i - lo] = gen_env_spec(int(specs["H"][i]), int(specs["W"][i]), int(specs["mode"][i]),
                                   int(specs["P"][i]), int(specs["cities_min"][i]), int(specs["cities_max"][i]),
                                   int(specs["min_general_dist"][i]), 0)
    return arr


def _stats_dict(st: gen_server_stats) -> dict:
    return {k: getattr(st, k) for k, _ in gen_server_stats._fields_}


class Server:
    """An environment server over a torch-allocated device arena (the
    memory budget).  Every method is one library call."""

    def __init__(self, arena_bytes: int, n_launch_streams: int = 2, max_batch_envs: int = 0,
                 device: str = "cuda"):
        import torch
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        self.handle = ctypes.c_void_p()
        _check(lib().gen_server_create(_ptr(self.arena), arena_bytes, n_launch_streams, max_batch_envs,
                                       ctypes.byref(self.handle)))

    def close_server(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gen_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close_server()

    def open(self, specs: dict, seed: int, env_base: int = 0, common: gen_params | None = None,
             actor_seed: int | None = None, queue: bool = False):
        """Open a group.  queue=False: its id, or GenError(GEN_EBUDGET) if it
        had to be queued for memory (it still is: close it or wait for it).
        queue=True: (id, admitted) -- admitted False when it was queued."""
        arr = _spec_array(specs)
        gid = ctypes.c_uint64()
        rc = lib().gen_server_open(self.handle, seed, env_base, len(arr), arr,
                                   ctypes.byref(common) if common else None, 1 if actor_seed is not None else 0,
                                   actor_seed or 0, ctypes.byref(gid))
        if queue and rc == GEN_EBUDGET:
            return gid.value, False
        if rc == GEN_EBUDGET:
            err = GenError(rc, gen_last_error())
            err.group = gid.value
            raise err
        _check(rc)
        return (gid.value, True) if queue else gid.value

    def wait_admitted(self, group: int, timeout_us: int = -1) -> int:
        rc = lib().gen_server_wait_admitted(self.handle, group, timeout_us)
        if rc not in (GEN_OK, GEN_EBUSY):
            _check(rc)
        return rc

    def buffers(self, group: int) -> dict:
        b = gen_group_buffers()
        _check(lib().gen_server_buffers(self.handle, group, ctypes.byref(b)))
        n = b.n_envs
        obs_off = np.zeros(n, np.uint64)
        act_off = np.zeros(n, np.uint32)
        _check(lib().gen_pool_offsets(b.pool, obs_off.ctypes.data, act_off.ctypes.data))
        a = self.arena
        return {"n_envs": n, "pool": b.pool, "obs_off": obs_off, "act_off": act_off,
                "obs": a[b.obs_off:b.obs_off + b.obs_bytes],
                "actions": a[b.actions_off:b.actions_off + 4 * b.n_actions].view(__import__("torch").int32),
                "rewards": a[b.rewards_off:b.rewards_off + 4 * b.n_actions].view(__import__("torch").int32),
                "dones": a[b.dones_off:b.dones_off + n]}

    def get_env(self, group: int, e: int, H: int, W: int, P: int) -> dict:
        b = gen_group_buffers()
        _check(lib().gen_server_buffers(self.handle, group, ctypes.byref(b)))
        h = _host_arrays(1, H * W, P)
        hs = _host_struct(h)
        _check(lib().gen_pool_get_env(b.pool, e, ctypes.byref(hs), None))
        return h

    def submit(self, group: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().gen_server_submit(self.handle, group, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        rc = lib().gen_server_wait(self.handle, ticket, timeout_us)
        if rc not in (GEN_OK, GEN_EBUSY):
            _check(rc)
        return rc

    def close(self, group: int):
        _check(lib().gen_server_close(self.handle, group))

    def set_batching(self, min_batch_envs: int = 0, max_wait_us: int = 100):
        _check(lib().gen_server_set_batching(self.handle, min_batch_envs, max_wait_us))

    def report(self, reset: bool = False) -> dict:
        st = gen_server_stats()
        _check(lib().gen_server_report(self.handle, ctypes.byref(st), 1 if reset else 0))
        return _stats_dict(st)

    def drive(self, group_envs, specs: dict, seed: int, actor_seed: int, gaps_us, duration_s: float,
              steps_per_group: int = 0, common: gen_params | None = None) -> dict:
        """Native closed-loop clients (see gen_server_drive).  gaps_us: array
        [n_clients, k] of inter-arrival gaps in microseconds."""
        gaps = np.ascontiguousarray(np.asarray(gaps_us, np.float64))
        n_clients, k = gaps.shape
        ge = np.ascontiguousarray(np.asarray(group_envs, np.int32))
        groups_per_client = len(ge) // n_clients
        arr = _spec_array(specs)
        st = gen_server_stats()
        _check(lib().gen_server_drive(self.handle, n_clients, groups_per_client, ge.ctypes.data, arr,
                                      ctypes.byref(common) if common else None, seed, actor_seed, gaps.ctypes.data,
                                      k, int(duration_s * 1e6), steps_per_group, ctypes.byref(st)))
        return _stats_dict(st)
