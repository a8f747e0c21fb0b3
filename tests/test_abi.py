"""The C-ABI library: it loads, exports every symbol the header declares, and
its host-side logic (layout, parameter checks, error reporting) behaves as
documented.  No kernel is launched here, so these run without a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_2606_23348_amd as gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "generals.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gen_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(gen.LIB_PATH):
        pytest.fail("libgenerals.so is not built (run __graft_entry__.build())")
    return gen.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("gen_reset", "gen_step", "gen_sample_actions", "gen_observe", "gen_get_state",
              "gen_set_state", "gen_layout", "gen_state_bytes", "gen_last_error"):
        assert f in names


def test_every_declared_symbol_is_exported(L):
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing
    # plain C names (no C++ mangling) in the dynamic symbol table
    out = subprocess.run(["nm", "-D", "--defined-only", gen.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(gen_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_version(L):
    assert gen.gen_version() == gen.GEN_LAYOUT_VERSION


def test_default_params():
    p = gen.gen_default_params(gen.GEN_1V1)
    assert p.n_players == 2 and p.mountain_thresh == (2 ** 32) // 5
    assert (p.cities_min, p.cities_max, p.city_army_min, p.city_army_max) == (9, 11, 40, 50)
    assert gen.gen_default_params(gen.GEN_2V2).n_players == 4
    assert gen.gen_default_params(gen.GEN_FFA, 8).n_players == 8
    with pytest.raises(gen.GenError):
        gen.gen_default_params(gen.GEN_FFA, 9)


@pytest.mark.parametrize("E,H,W,mode,P", [(16, 10, 10, 0, 2), (65536, 24, 24, 0, 2), (16384, 25, 25, 2, 8),
                                          (7, 3, 3, 1, 4), (3, 32, 32, 2, 5)])
def test_layout(E, H, W, mode, P):
    prm = gen.make_params(mode, P, cities_min=0, cities_max=min(11, H * W // 4))
    st = gen.gen_layout(E, H, W, mode, prm, seed=9)
    S = (H * W + 15) // 16 * 16
    assert st.stride == S and st.n_players == P and st.version == 1
    assert st.off_scalars == 0 and st.off_owner >= 32 * E
    assert st.off_type - st.off_owner >= E * S and st.off_army - st.off_type >= E * S
    assert st.bytes - st.off_army >= 4 * E * S
    for off in (st.off_owner, st.off_type, st.off_army, st.bytes):
        assert off % 256 == 0
    assert gen.gen_state_bytes(E, H, W, mode, prm) == st.bytes


@pytest.mark.parametrize("args", [(0, 10, 10, 0), (4, 2, 10, 0), (4, 10, 33, 0), (4, 10, 10, 7)])
def test_layout_rejects_bad_shapes(args):
    with pytest.raises(gen.GenError) as ei:
        gen.gen_layout(*args)
    assert ei.value.code == gen.GEN_EINVAL
    assert gen.gen_last_error() != ""


def test_layout_rejects_bad_params():
    p = gen.make_params(gen.GEN_1V1, cities_min=5, cities_max=3)
    with pytest.raises(gen.GenError):
        gen.gen_layout(4, 10, 10, gen.GEN_1V1, p)
    p = gen.make_params(gen.GEN_1V1)
    p.reserved[2] = 1
    with pytest.raises(gen.GenError):
        gen.gen_layout(4, 10, 10, gen.GEN_1V1, p)
    with pytest.raises(gen.GenError):            # FFA needs a player count
        gen.gen_layout(4, 10, 10, gen.GEN_FFA, None)


def test_calls_reject_missing_state_without_touching_the_device(L):
    assert L.gen_step(None, None, None, None, None, None, None, None) == gen.GEN_EINVAL
    assert "NULL" in gen.gen_last_error()
    st = gen.gen_layout(4, 10, 10, gen.GEN_1V1)
    assert L.gen_step(ctypes.byref(st), None, None, None, None, None, None, None) == gen.GEN_EINVAL
    assert "device buffer" in gen.gen_last_error()
    assert L.gen_reset(1, 0, 4, 10, 10, 0, None, None, 0, None, None, None) == gen.GEN_EINVAL


def test_empty_batches_are_rejected(L):
    """An empty batch or pool has no layout: GEN_EINVAL before any device call."""
    with pytest.raises(gen.GenError) as ei:
        gen.gen_layout(0, 10, 10, gen.GEN_1V1)
    assert ei.value.code == gen.GEN_EINVAL and "positive" in str(ei.value)
    out = ctypes.c_void_p()
    spec = (gen.gen_env_spec * 1)()
    assert L.gen_pool_create(0, 0, 0, spec, None, ctypes.byref(out)) == gen.GEN_EINVAL
    assert "positive" in gen.gen_last_error() and not out.value
    assert L.gen_pool_create(0, 0, -3, spec, None, ctypes.byref(out)) == gen.GEN_EINVAL


def test_stream_helpers_reject_bad_arguments(L):
    """The measurement copies check their arguments before any HIP call
    (the fake addresses are never dereferenced)."""
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21)
    assert L.gen_stream_copy(None, b, 64, None) == gen.GEN_EINVAL
    assert L.gen_stream_copy(ctypes.c_void_p((1 << 20) + 8), b, 64, None) == gen.GEN_EINVAL
    assert L.gen_stream_copy(a, b, 65, None) == gen.GEN_EINVAL
    assert L.gen_stream_copy(a, b, 0, None) == gen.GEN_OK
    assert L.gen_stream_spread(a, None, 64, 2, None) == gen.GEN_EINVAL
    assert L.gen_stream_spread(a, ctypes.c_void_p((1 << 21) + 4), 64, 2, None) == gen.GEN_EINVAL
    assert L.gen_stream_spread(a, b, 40, 2, None) == gen.GEN_EINVAL
    assert L.gen_stream_spread(None, b, 64, 0, None) == gen.GEN_EINVAL
    assert L.gen_stream_spread(a, None, 40, 0, None) == gen.GEN_EINVAL
    assert L.gen_stream_spread(a, b, 16 << 32, 1, None) == gen.GEN_EINVAL       # 2^32 chunks
    assert L.gen_stream_spread(a, b, 0, 3, None) == gen.GEN_OK


def test_reset_rejects_small_buffer(L):
    need = gen.gen_state_bytes(4, 10, 10, 0)
    fake = ctypes.c_void_p(1 << 20)                # never dereferenced: the size check comes first
    rc = L.gen_reset(1, 0, 4, 10, 10, 0, None, fake, need - 1, None, None, None)
    assert rc == gen.GEN_ENOMEM


def test_product_path_never_loads_the_oracle():
    """Importing the binding must not import or load the CPU oracle."""
    code = ("import sys, paper_2606_23348_amd as g; g.lib(); "
            "assert 'oracle' not in sys.modules, 'oracle imported'; "
            "maps = open('/proc/self/maps').read(); assert 'liboracle' not in maps; print('ok')")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert "ok" in out.stdout


def test_one_hip_runtime_in_process():
    """The library binds to the HIP runtime torch already loaded."""
    code = ("import paper_2606_23348_amd as g; g.lib(); "
            "import re; maps = open('/proc/self/maps').read(); "
            "libs = set(re.findall(r'(\\S*libamdhip64[^\\s]*)', maps)); print(len(libs), sorted(libs))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[0] == "1", out.stdout


def test_pool_plan_host_side(L):
    import numpy as np
    specs = {"H": np.array([10, 25, 3]), "W": np.array([12, 25, 3]), "mode": np.array([0, 1, 2]),
             "P": np.array([2, 4, 3]), "cities_min": np.array([2, 8, 0]), "cities_max": np.array([3, 13, 1]),
             "min_general_dist": np.array([9, 6, 1])}
    h = gen.gen_pool_create(5, 0, specs)
    info = gen.gen_pool_info()
    assert L.gen_pool_query(h, ctypes.byref(info)) == 0
    assert info.n_envs == 3 and info.max_cells == 625 and info.n_actions == 9
    obs = np.zeros(3, np.uint64)
    act = np.zeros(3, np.uint32)
    assert L.gen_pool_offsets(h, obs.ctypes.data, act.ctypes.data) == 0
    sizes = [2 * 8 * 128, 4 * 8 * 640, 3 * 8 * 64]      # planes padded to 32 bytes, 64 with more than 2 players
    assert obs.tolist() == [0, (sizes[0] + 15) // 16 * 16, ((sizes[0] + 15) // 16 + (sizes[1] + 15) // 16) * 16]
    assert act.tolist() == [0, 2, 6]
    assert info.obs_bytes == sum((s + 15) // 16 * 16 for s in sizes)
    bad = gen.gen_pool_tuning(3, 0, 0, 0)
    assert L.gen_pool_set_tuning(h, ctypes.byref(bad), None) == gen.GEN_EINVAL
    ok = gen.gen_pool_tuning(4, 64, 1, 0)
    assert L.gen_pool_set_tuning(h, ctypes.byref(ok), None) == 0        # not bound: nothing uploaded
    assert L.gen_pool_step(h, None, 1, 0, None, None, None, None) == gen.GEN_EINVAL
    assert "gen_pool_reset" in gen.gen_last_error()
    L.gen_pool_destroy(h)


def test_pool_rejects_bad_spec(L):
    import numpy as np
    specs = {"H": np.array([10, 40]), "W": np.array([10, 10]), "mode": np.array([0, 0]), "P": np.array([2, 2]),
             "cities_min": np.array([1, 1]), "cities_max": np.array([2, 2]), "min_general_dist": np.array([3, 3])}
    with pytest.raises(gen.GenError) as ei:
        gen.gen_pool_create(1, 0, specs)
    assert "env spec 1" in str(ei.value)


def test_pool_buckets_host_side(L):
    """Size buckets (players, 64-cell words) of a pool and their packing,
    listed and set on the host (no device needed before a pool is bound)."""
    import numpy as np
    specs = {"H": np.array([10, 25, 3, 10, 25]), "W": np.array([12, 25, 3, 13, 24]), "mode": np.array([0, 1, 2, 0, 1]),
             "P": np.array([2, 4, 3, 2, 4]), "cities_min": np.array([2, 8, 0, 2, 8]),
             "cities_max": np.array([3, 13, 1, 3, 13]), "min_general_dist": np.array([9, 6, 1, 9, 6])}
    h = gen.gen_pool_create(5, 0, specs)
    n = ctypes.c_int32()
    assert L.gen_pool_buckets(h, None, 0, ctypes.byref(n)) == 0 and n.value == 4
    arr = (gen.gen_pool_bucket * 4)()
    assert L.gen_pool_buckets(h, arr, 4, ctypes.byref(n)) == 0
    got = [(b.n_players, b.words, b.n_envs, b.waves_per_group, b.waves_per_env) for b in arr]
    # 10x12 takes 2 words, 10x13 3, 25x25 and 25x24 10, 3x3 1; in order of players, then words
    assert got == [(2, 2, 1, 1, 1), (2, 3, 1, 1, 1), (3, 1, 1, 1, 1), (4, 10, 2, 1, 1)]
    table = (gen.gen_pool_bucket * 2)(gen.gen_pool_bucket(4, 10, 0, 1, 2), gen.gen_pool_bucket(2, 2, 0, 2, 1))
    assert L.gen_pool_set_buckets(h, table, 2, None) == 0
    assert L.gen_pool_buckets(h, arr, 4, ctypes.byref(n)) == 0
    packing = {(b.n_players, b.words): (b.waves_per_group, b.waves_per_env) for b in arr[:n.value]}
    assert packing[(4, 10)] == (1, 2) and packing[(2, 2)] == (2, 1)
    bad = (gen.gen_pool_bucket * 1)(gen.gen_pool_bucket(4, 10, 0, 2, 2))   # two waves per env need their own group
    assert L.gen_pool_set_buckets(h, bad, 1, None) == gen.GEN_EINVAL
    bad = (gen.gen_pool_bucket * 1)(gen.gen_pool_bucket(9, 10, 0, 1, 1))
    assert L.gen_pool_set_buckets(h, bad, 1, None) == gen.GEN_EINVAL
    assert L.gen_pool_set_buckets(h, None, 0, None) == 0
    assert L.gen_pool_destroy(h) == 0
