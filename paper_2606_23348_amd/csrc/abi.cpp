// abi.cpp -- the extern "C" boundary of libgenerals.so: argument checks,
// device layout, launches, host-format copies and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/generals.h"
#include "internal.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    g_last_error.clear();
    return GEN_OK;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(GEN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

int players_of(int32_t mode, int32_t n_players)
{
    if (mode == GEN_1V1) return 2;
    if (mode == GEN_2V2) return 4;
    if (mode == GEN_FFA) return n_players;
    return -1;
}

int check_params(const gen_params &p, int P, int HW)
{
    if (p.cities_min < 0 || p.cities_max < p.cities_min || p.cities_max > HW)
        return fail(GEN_EINVAL, "cities range [%d, %d] invalid", p.cities_min, p.cities_max);
    if (p.city_army_min < 0 || p.city_army_max < p.city_army_min)
        return fail(GEN_EINVAL, "city army range [%d, %d] invalid", p.city_army_min, p.city_army_max);
    if (p.min_general_dist < 0 || p.min_general_dist > 64)
        return fail(GEN_EINVAL, "min_general_dist %d outside [0, 64]", p.min_general_dist);
    if ((p.auto_reset != 0 && p.auto_reset != 1) || (p.pregrow != 0 && p.pregrow != 1))
        return fail(GEN_EINVAL, "auto_reset and pregrow must be 0 or 1");
    if (p.generator != 0 && p.generator != 1) return fail(GEN_EINVAL, "generator must be 0 or 1");
    if (p.max_general_dist < 0 || p.max_general_dist > GEN_MAX_CELLS)
        return fail(GEN_EINVAL, "max_general_dist %d outside [0, %d]", p.max_general_dist, GEN_MAX_CELLS);
    if (p.castle_radius < 0 || p.castle_radius > 64)
        return fail(GEN_EINVAL, "castle_radius %d outside [0, 64]", p.castle_radius);
    if (p.obs_layout != 0 && p.obs_layout != 1) return fail(GEN_EINVAL, "obs_layout must be 0 or 1");
    for (int i = 0; i < 3; ++i)
        if (p.reserved[i] != 0) return fail(GEN_EINVAL, "gen_params.reserved must be zero");
    (void)P;
    return GEN_OK;
}

gen::Geom geom_of(const gen_state &st)
{
    gen::Geom g;
    g.H = st.H;
    g.W = st.W;
    g.HW = st.H * st.W;
    g.S = st.stride;
    g.P = st.n_players;
    g.mode = st.mode;
    g.NW = (g.HW + 63) / 64;
    g.magic_w = (uint32_t)(((1u << 20) + (uint32_t)st.W - 1) / (uint32_t)st.W);
    g.magic_hw = (uint32_t)(((uint64_t(1) << 32) + (uint64_t)g.HW - 1) / (uint64_t)g.HW);
    g.PS = st.params.obs_layout == 1 ? gen::pool_plane_stride(g.HW, g.P) : g.HW;
    return g;
}


int check_state(const gen_state *st)
{
    if (st == nullptr) return fail(GEN_EINVAL, "state descriptor is NULL");
    if (st->version != GEN_LAYOUT_VERSION)
        return fail(GEN_EINVAL, "state descriptor version %u, library expects %u", st->version, GEN_LAYOUT_VERSION);
    if (st->d_buf == nullptr) return fail(GEN_EINVAL, "state descriptor has no device buffer (call gen_reset)");
    gen_state chk;
    if (gen_layout(st->n_envs, st->H, st->W, st->mode, &st->params, st->seed, &chk) != GEN_OK) return GEN_EINVAL;
    if (chk.stride != st->stride || chk.bytes != st->bytes || chk.off_army != st->off_army ||
        chk.n_players != st->n_players)
        return fail(GEN_EINVAL, "state descriptor fields are inconsistent");
    return GEN_OK;
}

gen::EnvArgs env_args(const gen_state &st)
{
    gen::EnvArgs a{};
    a.g = geom_of(st);
    a.prm = gen::prm_of(st.params);
    a.seed = st.seed;
    a.env_base = st.env_base;
    uint8_t *base = static_cast<uint8_t *>(st.d_buf);
    a.sc = reinterpret_cast<gen::EnvScalars *>(base + st.off_scalars);
    a.owner = reinterpret_cast<int8_t *>(base + st.off_owner);
    a.type = base + st.off_type;
    a.army = reinterpret_cast<int32_t *>(base + st.off_army);
    return a;
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int check_obs_ptr(const gen_state &st, const uint8_t *d_obs)
{
    if (d_obs == nullptr) return GEN_OK;
    const uint64_t PS = st.params.obs_layout == 1 ? (uint64_t)gen::pool_plane_stride(st.H * st.W, st.n_players)
                                                  : (uint64_t)st.H * st.W;
    const uint64_t B = (uint64_t)st.n_players * 8 * PS;
    const uintptr_t need = (B % 16 == 0) ? 16 : 8;
    if (!aligned(d_obs, need)) return fail(GEN_EINVAL, "d_obs must be %u-byte aligned", (unsigned)need);
    return GEN_OK;
}

// The gather's staging buffer per device (gen_get_envs): allocated on first
// use, grown when a larger gather comes, held until the process ends.
struct Staging {
    uint8_t *ptr = nullptr;
    uint64_t bytes = 0;
};
constexpr int kStagingDevices = 64;
std::mutex g_staging_mu;
Staging g_staging[kStagingDevices];

int check_gather(const gen_state *st, const int32_t *h_env_ids, int32_t n_ids, const gen_host_state *h,
                 gen::GatherLayout *lay)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (h == nullptr || !h->owner || !h->army || !h->type || !h->turn || !h->episode || !h->alive || !h->finished ||
        !h->gpos)
        return fail(GEN_EINVAL, "host state has a NULL field");
    if (n_ids < 0 || (n_ids > 0 && h_env_ids == nullptr)) return fail(GEN_EINVAL, "bad env id list");
    for (int32_t i = 0; i < n_ids; ++i)
        if (h_env_ids[i] < 0 || h_env_ids[i] >= st->n_envs)
            return fail(GEN_EINVAL, "env id %d outside [0, %d)", h_env_ids[i], st->n_envs);
    *lay = gen::gather_layout((uint64_t)n_ids, (uint64_t)st->H * st->W, (uint64_t)st->n_players);
    int dev = 0;
    hipPointerAttribute_t attr;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipPointerGetAttributes(&attr, st->d_buf);
    if (e != hipSuccess) return hip_fail(e, "state buffer query");
    if (attr.device != dev)
        return fail(GEN_EINVAL, "the state lives on device %d, the current device is %d", attr.device, dev);
    return GEN_OK;
}

// Ids up, one gather launch into the staging block `stg`, one copy per field
// down into the caller's host arrays (blocking on `s`).
int gather_to_host(const gen_state &st, const int32_t *h_env_ids, int32_t n_ids, gen_host_state *h,
                   const gen::GatherLayout &lay, uint8_t *stg, hipStream_t s)
{
    const uint64_t n = (uint64_t)n_ids, HW = (uint64_t)st.H * st.W, P = (uint64_t)st.n_players;
    const gen::EnvArgs ea = env_args(st);
    gen::GatherArgs a{};
    a.lay = lay;
    a.S = st.stride;
    a.HW = (int32_t)HW;
    a.P = (int32_t)P;
    a.sc = ea.sc;
    a.owner = ea.owner;
    a.type = ea.type;
    a.army = ea.army;
    a.staging = stg;
    hipError_t e = hipMemcpyAsync(stg + lay.ids, h_env_ids, 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = gen::launch_gather(a, (uint32_t)n, s);
    const struct { void *dst; uint64_t off, bytes; } part[] = {
        {h->owner, lay.owner, n * HW}, {h->type, lay.type, n * HW}, {h->army, lay.army, 4 * n * HW},
        {h->turn, lay.turn, 4 * n}, {h->episode, lay.episode, 4 * n}, {h->alive, lay.alive, n},
        {h->finished, lay.finished, n}, {h->gpos, lay.gpos, 2 * n * P}};
    for (const auto &x : part)
        if (e == hipSuccess) e = hipMemcpyAsync(x.dst, stg + x.off, x.bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "env gather");
    return ok();
}

}  // namespace

namespace {

// Size bucket of env i: (players, 64-cell words of its map).
std::pair<int, int> bucket_of(const gen_pool &pl, size_t i)
{
    const gen::PoolDesc &d = pl.desc[i];
    return {(int)d.P, ((int)d.H * (int)d.W + 63) / 64};
}

// Packing (waves per group, waves per env) of env i: its bucket's entry of
// the table, else the pool-wide waves per group and one wave per env.
std::pair<uint32_t, uint32_t> packing_of(const gen_pool &pl, size_t i)
{
    const auto b = bucket_of(pl, i);
    for (const gen_pool_bucket &t : pl.buckets)
        if (t.n_players == b.first && t.words == b.second)
            return {(uint32_t)t.waves_per_group, (uint32_t)t.waves_per_env};
    return {(uint32_t)pl.tuning.waves_per_group, 1u};
}

// Work list: envs grouped into segments of one packing (in order of the
// packing), inside a segment in env order or largest first (tuning.order).
void pool_make_order(gen_pool &pl)
{
    const size_t n = (size_t)pl.n;
    std::vector<uint32_t> key(n);
    for (size_t i = 0; i < n; ++i) {
        const auto pk = packing_of(pl, i);
        key[i] = pk.first * 4 + pk.second;            // distinct per (waves_per_group, waves_per_env)
    }
    pl.order.resize(n);
    for (size_t i = 0; i < n; ++i) pl.order[i] = (uint32_t)i;
    std::stable_sort(pl.order.begin(), pl.order.end(), [&](uint32_t a, uint32_t b) {
        if (key[a] != key[b]) return key[a] < key[b];
        return pl.tuning.order == 1 && pl.work[a] > pl.work[b];
    });
    pl.segments.clear();
    for (size_t s = 0; s < n;) {
        size_t e = s;
        while (e < n && key[pl.order[e]] == key[pl.order[s]]) ++e;
        const auto pk = packing_of(pl, pl.order[s]);
        pl.segments.push_back({(uint32_t)s, (uint32_t)e, pk.first, pk.second});
        s = e;
    }
}

// One step of every env: one launch per segment of the work list, in order
// on the caller's stream.
hipError_t pool_step_launches(const gen_pool &pl, gen::PoolArgs a, bool act, hipStream_t s)
{
    for (const auto &sg : pl.segments) {
        a.slot_begin = sg.begin;
        a.slot_end = sg.end;
        a.wpg = sg.wpg;
        const hipError_t e = gen::launch_pool(a, 0 /* step */, act, (uint32_t)pl.tuning.grid, sg.nwv, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

gen::PoolArgs pool_args(const gen_pool &pl)
{
    gen::PoolArgs a{};
    a.prm = gen::prm_of(pl.common);
    a.seed = pl.seed;
    a.env_base = pl.env_base;
    a.n_envs = (uint32_t)pl.n;
    a.slot_begin = 0;
    a.slot_end = (uint32_t)pl.n;
    a.wpg = (uint32_t)pl.tuning.waves_per_group;
    a.lds_per_wave = pl.lds_per_wave;
    uint8_t *base = static_cast<uint8_t *>(pl.d_state);
    a.desc = reinterpret_cast<const gen::PoolDesc *>(base + pl.off_desc);
    a.sc = reinterpret_cast<gen::EnvScalars *>(base + pl.off_scalars);
    a.owner = reinterpret_cast<int8_t *>(base + pl.off_owner);
    a.type = base + pl.off_type;
    a.army = reinterpret_cast<int32_t *>(base + pl.off_army);
    return a;
}

// The device work list: the envs' descriptors in slot order (each carries
// its env index), so a wave reaches its env's geometry with one load.
int pool_upload_work(gen_pool &pl, hipStream_t s)
{
    std::vector<gen::PoolDesc> work(pl.order.size());
    for (size_t i = 0; i < work.size(); ++i) work[i] = pl.desc[pl.order[i]];
    hipError_t e = hipMemcpyAsync(static_cast<uint8_t *>(pl.d_state) + pl.off_desc, work.data(),
                                  work.size() * sizeof(gen::PoolDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GEN_OK : hip_fail(e, "pool work-list upload");
}

int check_bound(const gen_pool *pl)
{
    if (pl == nullptr) return fail(GEN_EINVAL, "pool is NULL");
    if (pl->d_state == nullptr) return fail(GEN_EINVAL, "pool has no state buffer (call gen_pool_reset)");
    return GEN_OK;
}

}  // namespace

int gen::set_error(int code, const char *msg)
{
    g_last_error = msg ? msg : "";
    return code;
}

extern "C" {

int gen_version(void) { return GEN_LAYOUT_VERSION; }

const char *gen_last_error(void) { return g_last_error.c_str(); }

int gen_default_params(int32_t mode, int32_t n_players, gen_params *out)
{
    if (out == nullptr) return fail(GEN_EINVAL, "out is NULL");
    const int P = players_of(mode, n_players);
    if (P < 2 || P > GEN_MAX_PLAYERS) return fail(GEN_EINVAL, "mode %d with %d players is not a game", mode, n_players);
    std::memset(out, 0, sizeof *out);
    out->n_players = P;
    out->mountain_thresh = 858993459u;  // floor(2^32 / 5): 20% mountains
    out->cities_min = 9;
    out->cities_max = 11;
    out->city_army_min = 40;
    out->city_army_max = 50;
    out->min_general_dist = 9;
    out->auto_reset = 1;
    out->pregrow = 0;
    out->generator = 0;
    out->max_general_dist = 0;
    out->castle_radius = 6;
    return ok();
}

int gen_layout(int32_t n_envs, int32_t H, int32_t W, int32_t mode, const gen_params *params, uint64_t seed,
               gen_state *out)
{
    if (out == nullptr) return fail(GEN_EINVAL, "out is NULL");
    if (n_envs < 1) return fail(GEN_EINVAL, "n_envs %d must be positive", n_envs);
    if (H < GEN_MIN_SIDE || H > GEN_MAX_SIDE || W < GEN_MIN_SIDE || W > GEN_MAX_SIDE)
        return fail(GEN_EINVAL, "grid %dx%d outside %d..%d per side", H, W, GEN_MIN_SIDE, GEN_MAX_SIDE);
    gen_params p;
    if (params == nullptr) {
        if (mode == GEN_FFA) return fail(GEN_EINVAL, "free-for-all needs params (n_players)");
        if (gen_default_params(mode, 0, &p) != GEN_OK) return GEN_EINVAL;
    } else {
        p = *params;
    }
    const int P = players_of(mode, p.n_players);
    if (P < 2 || P > GEN_MAX_PLAYERS)
        return fail(GEN_EINVAL, "mode %d with %d players is not a game", mode, p.n_players);
    p.n_players = P;
    if (check_params(p, P, H * W) != GEN_OK) return GEN_EINVAL;

    std::memset(out, 0, sizeof *out);
    out->version = GEN_LAYOUT_VERSION;
    out->n_envs = n_envs;
    out->H = H;
    out->W = W;
    out->mode = mode;
    out->n_players = P;
    out->stride = (H * W + 15) & ~15;
    out->seed = seed;
    out->params = p;
    const uint64_t E = (uint64_t)n_envs, S = (uint64_t)out->stride;
    out->off_scalars = 0;
    out->off_owner = align256(E * sizeof(gen::EnvScalars));
    out->off_type = out->off_owner + align256(E * S);
    out->off_army = out->off_type + align256(E * S);
    out->bytes = out->off_army + align256(E * S * 4);
    out->d_buf = nullptr;
    return ok();
}

uint64_t gen_state_bytes(int32_t n_envs, int32_t H, int32_t W, int32_t mode, const gen_params *params)
{
    gen_state st;
    if (gen_layout(n_envs, H, W, mode, params, 0, &st) != GEN_OK) return 0;
    return st.bytes;
}

int gen_reset(uint64_t seed, uint64_t env_base, int32_t n_envs, int32_t H, int32_t W, int32_t mode,
              const gen_params *params, void *d_buf, uint64_t buf_bytes, uint8_t *d_obs, void *stream, gen_state *out)
{
    gen_state st;
    if (gen_layout(n_envs, H, W, mode, params, seed, &st) != GEN_OK) return GEN_EINVAL;
    if (d_buf == nullptr || !aligned(d_buf, 256)) return fail(GEN_EINVAL, "d_buf must be a 256-byte aligned device pointer");
    if (buf_bytes < st.bytes)
        return fail(GEN_ENOMEM, "state buffer holds %llu bytes, layout needs %llu", (unsigned long long)buf_bytes,
                    (unsigned long long)st.bytes);
    st.env_base = env_base;
    st.d_buf = d_buf;
    if (check_obs_ptr(st, d_obs) != GEN_OK) return GEN_EINVAL;
    gen::EnvArgs a = env_args(st);
    a.obs = d_obs;
    hipError_t e = gen::launch_reset(a, n_envs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "reset launch");
    if (out) *out = st;
    return ok();
}

int gen_step(const gen_state *st, const int32_t *d_actions, uint8_t *d_obs, int32_t *d_rewards, uint8_t *d_dones,
             int32_t *d_land, int64_t *d_army, void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (d_actions == nullptr || d_rewards == nullptr || d_dones == nullptr)
        return fail(GEN_EINVAL, "d_actions, d_rewards and d_dones are required");
    if ((d_land == nullptr) != (d_army == nullptr)) return fail(GEN_EINVAL, "d_land and d_army go together");
    if (check_obs_ptr(*st, d_obs) != GEN_OK) return GEN_EINVAL;
    if (!aligned(d_actions, 4) || !aligned(d_rewards, 4) || (d_army && !aligned(d_army, 8)) ||
        (d_land && !aligned(d_land, 4)))
        return fail(GEN_EINVAL, "misaligned action, reward or scoreboard pointer");
    gen::EnvArgs a = env_args(*st);
    a.actions = d_actions;
    a.obs = d_obs;
    a.rewards = d_rewards;
    a.dones = d_dones;
    a.land = d_land;
    a.army_tot = d_army;
    hipError_t e = gen::launch_step(a, st->n_envs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return ok();
}

int gen_step_sample(const gen_state *st, int32_t *d_actions, uint64_t actor_seed, uint64_t next_step_idx,
                    uint8_t *d_obs, int32_t *d_rewards, uint8_t *d_dones, int32_t *d_land, int64_t *d_army,
                    void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (d_actions == nullptr || d_rewards == nullptr || d_dones == nullptr)
        return fail(GEN_EINVAL, "d_actions, d_rewards and d_dones are required");
    if ((d_land == nullptr) != (d_army == nullptr)) return fail(GEN_EINVAL, "d_land and d_army go together");
    if (check_obs_ptr(*st, d_obs) != GEN_OK) return GEN_EINVAL;
    if (!aligned(d_actions, 4) || !aligned(d_rewards, 4) || (d_army && !aligned(d_army, 8)) ||
        (d_land && !aligned(d_land, 4)))
        return fail(GEN_EINVAL, "misaligned action, reward or scoreboard pointer");
    gen::EnvArgs a = env_args(*st);
    a.actions = d_actions;
    a.next_actions = d_actions;
    a.actor_seed = actor_seed;
    a.step_idx = next_step_idx;
    a.obs = d_obs;
    a.rewards = d_rewards;
    a.dones = d_dones;
    a.land = d_land;
    a.army_tot = d_army;
    hipError_t e = gen::launch_step(a, st->n_envs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return ok();
}

int gen_sample_actions(const gen_state *st, uint64_t actor_seed, uint64_t step_idx, int32_t *d_actions, void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (d_actions == nullptr || !aligned(d_actions, 4)) return fail(GEN_EINVAL, "d_actions must be an aligned device pointer");
    const gen::EnvArgs ea = env_args(*st);
    gen::SampleArgs a{};
    a.g = ea.g;
    a.env_base = st->env_base;
    a.actor_seed = actor_seed;
    a.step_idx = step_idx;
    a.sc = ea.sc;
    a.owner = ea.owner;
    a.type = ea.type;
    a.army = ea.army;
    a.actions = d_actions;
    hipError_t e = gen::launch_sample(a, st->n_envs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "sample launch");
    return ok();
}

int gen_observe(const gen_state *st, uint8_t *d_obs, void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (d_obs == nullptr) return fail(GEN_EINVAL, "d_obs is NULL");
    if (check_obs_ptr(*st, d_obs) != GEN_OK) return GEN_EINVAL;
    gen::EnvArgs a = env_args(*st);
    a.obs = d_obs;
    hipError_t e = gen::launch_observe(a, st->n_envs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "observe launch");
    return ok();
}

uint64_t gen_feat_mem_bytes(const gen_state *st)
{
    if (check_state(st) != GEN_OK) return 0;
    return (uint64_t)gen::feat_block(st->stride, st->n_players).bytes * (uint64_t)st->n_envs;
}

int gen_features(const gen_state *st, void *d_mem, uint64_t mem_bytes, float *d_feat, float *d_tokens, void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (d_mem == nullptr || !aligned(d_mem, 256))
        return fail(GEN_EINVAL, "d_mem must be a 256-byte aligned device pointer");
    if (d_feat == nullptr || !aligned(d_feat, 4)) return fail(GEN_EINVAL, "d_feat must be a 4-byte aligned device pointer");
    if (d_tokens != nullptr && !aligned(d_tokens, 4)) return fail(GEN_EINVAL, "d_tokens must be 4-byte aligned");
    const gen::FeatBlock fb = gen::feat_block(st->stride, st->n_players);
    const uint64_t need = (uint64_t)fb.bytes * (uint64_t)st->n_envs;
    if (mem_bytes < need)
        return fail(GEN_ENOMEM, "feature memory holds %llu bytes, the batch needs %llu", (unsigned long long)mem_bytes,
                    (unsigned long long)need);
    const gen::EnvArgs ea = env_args(*st);
    gen::FeatArgs a{};
    a.g = ea.g;
    a.blk = fb;
    a.sc = ea.sc;
    a.owner = ea.owner;
    a.type = ea.type;
    a.army = ea.army;
    a.mem = static_cast<uint8_t *>(d_mem);
    a.feat = d_feat;
    a.tokens = d_tokens;
    hipError_t e = gen::feature_tables_ready();
    if (e != hipSuccess) return hip_fail(e, "feature table upload");
    e = gen::launch_features(a, st->n_envs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "features launch");
    return ok();
}

int gen_rollout(const gen_state *st, void *d_mem, uint64_t mem_bytes, int32_t n_steps, uint64_t actor_seed,
                uint64_t step0, float *d_feat, float *d_tokens, int32_t *d_actions, int32_t *d_rewards, uint8_t *d_dones,
                void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (n_steps < 1) return fail(GEN_EINVAL, "n_steps %d must be positive", n_steps);
    if (d_mem == nullptr || !aligned(d_mem, 256))
        return fail(GEN_EINVAL, "d_mem must be a 256-byte aligned device pointer");
    if (d_feat == nullptr || d_actions == nullptr || d_rewards == nullptr || d_dones == nullptr)
        return fail(GEN_EINVAL, "d_feat, d_actions, d_rewards and d_dones are required");
    if (!aligned(d_feat, 4) || !aligned(d_actions, 4) || !aligned(d_rewards, 4) || (d_tokens && !aligned(d_tokens, 4)))
        return fail(GEN_EINVAL, "misaligned rollout buffer");
    const gen::FeatBlock fb = gen::feat_block(st->stride, st->n_players);
    if (mem_bytes < (uint64_t)fb.bytes * (uint64_t)st->n_envs)
        return fail(GEN_ENOMEM, "feature memory holds %llu bytes, the batch needs %llu", (unsigned long long)mem_bytes,
                    (unsigned long long)((uint64_t)fb.bytes * (uint64_t)st->n_envs));
    hipError_t e = gen::feature_tables_ready();
    if (e != hipSuccess) return hip_fail(e, "feature table upload");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t E = (size_t)st->n_envs, P = (size_t)st->n_players, HW = (size_t)st->H * st->W;
    const size_t f_stride = E * P * GEN_FEAT_CHANNELS * HW, t_stride = E * P * 2 * GEN_TOKEN_WINDOW;
    const gen::EnvArgs base = env_args(*st);

    gen::SampleArgs sa{};
    sa.g = base.g;
    sa.env_base = st->env_base;
    sa.actor_seed = actor_seed;
    sa.step_idx = step0;
    sa.sc = base.sc;
    sa.owner = base.owner;
    sa.type = base.type;
    sa.army = base.army;
    sa.actions = d_actions;
    e = gen::launch_sample(sa, st->n_envs, s);
    if (e != hipSuccess) return hip_fail(e, "rollout sample launch");
    for (int32_t t = 0; t < n_steps; ++t) {
        gen::FeatArgs fa{};
        fa.g = base.g;
        fa.blk = fb;
        fa.sc = base.sc;
        fa.owner = base.owner;
        fa.type = base.type;
        fa.army = base.army;
        fa.mem = static_cast<uint8_t *>(d_mem);
        fa.feat = d_feat + (size_t)t * f_stride;
        fa.tokens = d_tokens ? d_tokens + (size_t)t * t_stride : nullptr;
        e = gen::launch_features(fa, st->n_envs, s);
        if (e != hipSuccess) return hip_fail(e, "rollout features launch");
        gen::EnvArgs ea = base;
        ea.actions = d_actions + (size_t)t * E * P;
        ea.rewards = d_rewards + (size_t)t * E * P;
        ea.dones = d_dones + (size_t)t * E;
        if (t + 1 < n_steps) {           // the next step's actions, sampled in the same launch
            ea.next_actions = d_actions + (size_t)(t + 1) * E * P;
            ea.actor_seed = actor_seed;
            ea.step_idx = step0 + (uint64_t)t + 1;
        }
        e = gen::launch_step(ea, st->n_envs, s);
        if (e != hipSuccess) return hip_fail(e, "rollout step launch");
    }
    return ok();
}

int gen_get_state(const gen_state *st, gen_host_state *h, void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (h == nullptr || !h->owner || !h->army || !h->type || !h->turn || !h->episode || !h->alive || !h->finished ||
        !h->gpos)
        return fail(GEN_EINVAL, "host state has a NULL field");
    std::vector<uint8_t> buf(st->bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(buf.data(), st->d_buf, st->bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "state download");
    const int HW = st->H * st->W, S = st->stride, P = st->n_players;
    const gen::EnvScalars *sc = reinterpret_cast<const gen::EnvScalars *>(buf.data() + st->off_scalars);
    for (int64_t i = 0; i < st->n_envs; ++i) {
        std::memcpy(h->owner + i * HW, buf.data() + st->off_owner + i * S, HW);
        std::memcpy(h->type + i * HW, buf.data() + st->off_type + i * S, HW);
        std::memcpy(h->army + i * HW, buf.data() + st->off_army + i * S * 4, (size_t)HW * 4);
        h->turn[i] = sc[i].turn;
        h->episode[i] = sc[i].episode;
        h->alive[i] = sc[i].alive;
        h->finished[i] = sc[i].finished;
        for (int p = 0; p < P; ++p) h->gpos[i * P + p] = sc[i].gpos[p];
    }
    return ok();
}

int gen_get_envs(const gen_state *st, const int32_t *h_env_ids, int32_t n_ids, gen_host_state *h, void *stream)
{
    uint8_t *stg = nullptr;
    gen::GatherLayout lay{};
    if (check_gather(st, h_env_ids, n_ids, h, &lay) != GEN_OK) return GEN_EINVAL;
    if (n_ids == 0) return ok();
    std::lock_guard<std::mutex> lk(g_staging_mu);      // one gather at a time uses a device's staging
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= kStagingDevices) return fail(GEN_EINVAL, "device %d beyond the staging table", dev);
    Staging &sg = g_staging[dev];
    if (sg.bytes < lay.bytes) {
        if (sg.ptr) {
            e = hipFree(sg.ptr);
            sg.ptr = nullptr;
            sg.bytes = 0;
            if (e != hipSuccess) return hip_fail(e, "staging release");
        }
        const uint64_t want = std::max<uint64_t>(lay.bytes, 1ull << 20);
        e = hipMalloc(reinterpret_cast<void **>(&sg.ptr), want);
        if (e != hipSuccess) return hip_fail(e, "staging allocation");
        sg.bytes = want;
    }
    stg = sg.ptr;
    return gather_to_host(*st, h_env_ids, n_ids, h, lay, stg, static_cast<hipStream_t>(stream));
}

int gen_get_envs_static(const gen_state *st, const int32_t *h_env_ids, int32_t n_ids, gen_host_state *h,
                        void *stream)
{
    gen::GatherLayout lay{};
    if (check_gather(st, h_env_ids, n_ids, h, &lay) != GEN_OK) return GEN_EINVAL;
    if (lay.bytes > GEN_STATIC_STAGING_BYTES)
        return fail(GEN_ENOMEM, "a gather of %d envs stages %llu bytes, the static array holds %llu", n_ids,
                    (unsigned long long)lay.bytes, (unsigned long long)GEN_STATIC_STAGING_BYTES);
    if (n_ids == 0) return ok();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    void *stg = nullptr;
    e = gen::static_staging(dev, &stg);
    if (e != hipSuccess) return hip_fail(e, "static staging address");
    return gather_to_host(*st, h_env_ids, n_ids, h, lay, static_cast<uint8_t *>(stg), static_cast<hipStream_t>(stream));
}

int gen_stream_copy(void *d_dst, const void *d_src, uint64_t bytes, void *stream)
{
    if (d_dst == nullptr || d_src == nullptr || !aligned(d_dst, 16) || !aligned(d_src, 16) || bytes % 16 != 0)
        return fail(GEN_EINVAL, "gen_stream_copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    if (bytes == 0) return ok();
    hipError_t e = gen::launch_stream_copy(d_dst, d_src, bytes / 16, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return ok();
}

int gen_stream_spread(void *d_dst, const void *d_src, uint64_t dst_bytes, uint32_t k, void *stream)
{
    if (d_dst == nullptr || !aligned(d_dst, 16) || (k != 0 && (d_src == nullptr || !aligned(d_src, 16))) ||
        dst_bytes % 16 != 0)
        return fail(GEN_EINVAL, "gen_stream_spread needs 16-byte aligned buffers and a multiple of 16 bytes");
    if (dst_bytes / 16 > 0xFFFFFFFFull) return fail(GEN_EINVAL, "gen_stream_spread writes fewer than 2^32 chunks");
    if (dst_bytes == 0) return ok();
    hipError_t e = gen::launch_stream_spread(d_dst, d_src, (uint32_t)(dst_bytes / 16), k, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "spread launch");
    return ok();
}

int gen_pool_create(uint64_t seed, uint64_t env_base, int32_t n_envs, const gen_env_spec *h_specs,
                    const gen_params *common, gen_pool **out)
{
    if (out == nullptr || h_specs == nullptr) return fail(GEN_EINVAL, "out and h_specs are required");
    *out = nullptr;
    if (n_envs < 1) return fail(GEN_EINVAL, "n_envs %d must be positive", n_envs);
    gen_params cp;
    if (common) cp = *common;
    else gen_default_params(GEN_1V1, 0, &cp);
    gen_pool *pl = new (std::nothrow) gen_pool();
    if (pl == nullptr) return fail(GEN_ENOMEM, "host allocation failed");
    pl->seed = seed;
    pl->env_base = env_base;
    pl->n = n_envs;
    pl->common = cp;
    pl->desc.resize((size_t)n_envs);
    pl->work.resize((size_t)n_envs);
    uint64_t cells = 0, obs16 = 0, acts = 0;
    int max_s = 16, max_p = 2;
    for (int32_t i = 0; i < n_envs; ++i) {
        const gen_env_spec &sp = h_specs[i];
        gen_params p = cp;
        p.n_players = sp.n_players;
        p.cities_min = sp.cities_min;
        p.cities_max = sp.cities_max;
        p.min_general_dist = sp.min_general_dist;
        gen_state st;
        if (sp.reserved != 0 || gen_layout(1, sp.H, sp.W, sp.mode, &p, seed, &st) != GEN_OK) {
            const std::string why = g_last_error;
            delete pl;
            return fail(GEN_EINVAL, "env spec %d: %s", i, sp.reserved != 0 ? "reserved must be zero" : why.c_str());
        }
        if (sp.cities_max > 255 || sp.min_general_dist > 255) {
            delete pl;
            return fail(GEN_EINVAL, "env spec %d: cities_max and min_general_dist must be <= 255", i);
        }
        const gen::Geom g = geom_of(st);
        gen::PoolDesc &d = pl->desc[(size_t)i];
        d.cell_off = (uint32_t)cells;
        d.obs_off16 = (uint32_t)obs16;
        d.act_off = (uint32_t)acts;
        d.magic_w = g.magic_w;
        d.magic_hw = g.magic_hw;
        d.H = (uint8_t)sp.H;
        d.W = (uint8_t)sp.W;
        d.mode = (uint8_t)sp.mode;
        d.P = (uint8_t)st.n_players;
        d.cmin = (uint8_t)sp.cities_min;
        d.cmax = (uint8_t)sp.cities_max;
        d.dmin = (uint8_t)sp.min_general_dist;
        d.pad8 = 0;
        d.env = (uint32_t)i;
        cells += (uint64_t)st.stride;
        obs16 += ((uint64_t)st.n_players * 8 * (uint64_t)gen::pool_plane_stride(sp.H * sp.W, st.n_players) + 15) / 16;
        acts += (uint64_t)st.n_players;
        pl->work[(size_t)i] = (uint64_t)st.n_players * sp.H * sp.W;
        if (st.stride > max_s) max_s = st.stride;
        if (st.n_players > max_p) max_p = st.n_players;
        if (sp.H * sp.W > pl->max_cells) pl->max_cells = sp.H * sp.W;
    }
    if (cells > 0xFFFFFFFFull || obs16 > 0xFFFFFFFFull) {
        delete pl;
        return fail(GEN_EINVAL, "pool too large for 32-bit offsets");
    }
    const uint64_t E = (uint64_t)n_envs;
    pl->off_scalars = 0;
    pl->off_desc = align256(E * sizeof(gen::EnvScalars));
    pl->off_owner = pl->off_desc + align256(E * sizeof(gen::PoolDesc));
    pl->off_type = pl->off_owner + align256(cells);
    pl->off_army = pl->off_type + align256(cells);
    pl->state_bytes = pl->off_army + align256(cells * 4);
    pl->obs_bytes = obs16 * 16;
    pl->n_actions = acts;
    pl->lds_per_wave = (gen::lds_bytes_for(max_s, max_p) + 15) & ~15u;
    pool_make_order(*pl);
    *out = pl;
    return ok();
}

int gen_pool_destroy(gen_pool *pool)
{
    if (pool == nullptr) return ok();
    if (pool->exec) (void)hipGraphExecDestroy(pool->exec);
    if (pool->graph) (void)hipGraphDestroy(pool->graph);
    delete pool;
    return ok();
}

int gen_pool_query(const gen_pool *pool, gen_pool_info *out)
{
    if (pool == nullptr || out == nullptr) return fail(GEN_EINVAL, "pool and out are required");
    out->n_envs = pool->n;
    out->max_cells = pool->max_cells;
    out->state_bytes = pool->state_bytes;
    out->obs_bytes = pool->obs_bytes;
    out->n_actions = pool->n_actions;
    out->work_list_off = pool->off_desc;
    out->work_list_bytes = (uint64_t)pool->n * sizeof(gen::PoolDesc);
    return ok();
}

int gen_pool_offsets(const gen_pool *pool, uint64_t *h_obs_off, uint32_t *h_act_off)
{
    if (pool == nullptr) return fail(GEN_EINVAL, "pool is NULL");
    for (int32_t i = 0; i < pool->n; ++i) {
        if (h_obs_off) h_obs_off[i] = (uint64_t)pool->desc[(size_t)i].obs_off16 * 16;
        if (h_act_off) h_act_off[i] = pool->desc[(size_t)i].act_off;
    }
    return ok();
}

int gen_pool_get_tuning(const gen_pool *pool, gen_pool_tuning *out)
{
    if (pool == nullptr || out == nullptr) return fail(GEN_EINVAL, "pool and out are required");
    *out = pool->tuning;
    return ok();
}

int gen_pool_set_tuning(gen_pool *pool, const gen_pool_tuning *t, void *stream)
{
    if (pool == nullptr || t == nullptr) return fail(GEN_EINVAL, "pool and tuning are required");
    if (t->waves_per_group != 1 && t->waves_per_group != 2 && t->waves_per_group != 4)
        return fail(GEN_EINVAL, "waves_per_group must be 1, 2 or 4");
    if (t->grid < 0 || (t->order != 0 && t->order != 1) || t->reserved != 0)
        return fail(GEN_EINVAL, "grid must be >= 0, order 0 or 1, reserved 0");
    if ((uint64_t)pool->lds_per_wave * (uint64_t)t->waves_per_group > 65536)
        return fail(GEN_EINVAL, "%d waves per group need more than 64 KiB of LDS", t->waves_per_group);
    pool->tuning = *t;
    pool_make_order(*pool);
    if (pool->d_state) return pool_upload_work(*pool, static_cast<hipStream_t>(stream)) == GEN_OK ? ok() : GEN_EHIP;
    return ok();
}

int gen_pool_buckets(const gen_pool *pool, gen_pool_bucket *out, int32_t capacity, int32_t *n_out)
{
    if (pool == nullptr || n_out == nullptr) return fail(GEN_EINVAL, "pool and n_out are required");
    if (capacity < 0 || (capacity > 0 && out == nullptr)) return fail(GEN_EINVAL, "bad output capacity");
    std::vector<gen_pool_bucket> list;
    for (size_t i = 0; i < (size_t)pool->n; ++i) {
        const auto b = bucket_of(*pool, i);
        auto it = std::find_if(list.begin(), list.end(),
                               [&](const gen_pool_bucket &x) { return x.n_players == b.first && x.words == b.second; });
        if (it == list.end()) {
            gen_pool_bucket x{};
            x.n_players = b.first;
            x.words = b.second;
            const auto pk = packing_of(*pool, i);
            x.waves_per_group = (int32_t)pk.first;
            x.waves_per_env = (int32_t)pk.second;
            list.push_back(x);
            it = list.end() - 1;
        }
        it->n_envs += 1;
    }
    std::sort(list.begin(), list.end(), [](const gen_pool_bucket &a, const gen_pool_bucket &b) {
        return a.n_players != b.n_players ? a.n_players < b.n_players : a.words < b.words;
    });
    *n_out = (int32_t)list.size();
    for (int32_t i = 0; i < capacity && i < (int32_t)list.size(); ++i) out[i] = list[(size_t)i];
    return ok();
}

int gen_pool_set_buckets(gen_pool *pool, const gen_pool_bucket *table, int32_t n, void *stream)
{
    if (pool == nullptr || n < 0 || (n > 0 && table == nullptr)) return fail(GEN_EINVAL, "pool and table are required");
    for (int32_t i = 0; i < n; ++i) {
        const gen_pool_bucket &t = table[i];
        if (t.n_players < 2 || t.n_players > GEN_MAX_PLAYERS || t.words < 1 || t.words > GEN_MAX_CELLS / 64)
            return fail(GEN_EINVAL, "bucket %d: %d players, %d words is not a bucket", i, t.n_players, t.words);
        if (t.waves_per_group != 1 && t.waves_per_group != 2 && t.waves_per_group != 4)
            return fail(GEN_EINVAL, "bucket %d: waves_per_group must be 1, 2 or 4", i);
        if (t.waves_per_env != 1 && t.waves_per_env != 2)
            return fail(GEN_EINVAL, "bucket %d: waves_per_env must be 1 or 2", i);
        if (t.waves_per_env == 2 && t.waves_per_group != 1)
            return fail(GEN_EINVAL, "bucket %d: two waves per env take a workgroup of their own", i);
        if (t.reserved[0] || t.reserved[1] || t.reserved[2])
            return fail(GEN_EINVAL, "bucket %d: reserved must be zero", i);
        if ((uint64_t)pool->lds_per_wave * (uint64_t)t.waves_per_group > 65536)
            return fail(GEN_EINVAL, "bucket %d: %d waves per group need more than 64 KiB of LDS", i, t.waves_per_group);
    }
    pool->buckets.assign(table, table + n);
    pool_make_order(*pool);
    if (pool->d_state) return pool_upload_work(*pool, static_cast<hipStream_t>(stream)) == GEN_OK ? ok() : GEN_EHIP;
    return ok();
}

int gen_pool_reset(gen_pool *pool, void *d_state, uint64_t state_bytes, uint8_t *d_obs, int32_t *d_actions,
                   uint64_t actor_seed, void *stream)
{
    if (pool == nullptr) return fail(GEN_EINVAL, "pool is NULL");
    if (d_state == nullptr || !aligned(d_state, 256)) return fail(GEN_EINVAL, "d_state must be 256-byte aligned");
    if (state_bytes < pool->state_bytes)
        return fail(GEN_ENOMEM, "state buffer holds %llu bytes, pool needs %llu", (unsigned long long)state_bytes,
                    (unsigned long long)pool->state_bytes);
    if ((d_obs && !aligned(d_obs, 16)) || (d_actions && !aligned(d_actions, 4)))
        return fail(GEN_EINVAL, "d_obs must be 16-byte and d_actions 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    pool->d_state = d_state;
    if (pool_upload_work(*pool, s) != GEN_OK) return GEN_EHIP;
    gen::PoolArgs a = pool_args(*pool);
    hipError_t e = hipSuccess;
    a.obs = d_obs;
    a.actions = d_actions;
    a.actor_seed = actor_seed;
    a.actor = d_actions != nullptr ? 1u : 0u;
    e = gen::launch_pool(a, 1 /* reset */, d_actions != nullptr, (uint32_t)pool->tuning.grid, 1, s);
    if (e != hipSuccess) return hip_fail(e, "pool reset launch");
    return ok();
}

int gen_pool_step(gen_pool *pool, int32_t *d_actions, int32_t actor, uint64_t actor_seed, uint8_t *d_obs,
                  int32_t *d_rewards, uint8_t *d_dones, void *stream)
{
    if (check_bound(pool) != GEN_OK) return GEN_EINVAL;
    if (d_actions == nullptr || d_rewards == nullptr || d_dones == nullptr)
        return fail(GEN_EINVAL, "d_actions, d_rewards and d_dones are required");
    if ((d_obs && !aligned(d_obs, 16)) || !aligned(d_actions, 4) || !aligned(d_rewards, 4))
        return fail(GEN_EINVAL, "misaligned obs, action or reward pointer");
    gen::PoolArgs a = pool_args(*pool);
    a.obs = d_obs;
    a.actions = d_actions;
    a.rewards = d_rewards;
    a.dones = d_dones;
    a.actor_seed = actor_seed;
    a.actor = actor != 0 ? 1u : 0u;
    hipError_t e = pool_step_launches(*pool, a, actor != 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pool step launch");
    return ok();
}

int gen_pool_capture(gen_pool *pool, int32_t k_steps, int32_t *d_actions, uint64_t actor_seed, uint8_t *d_obs,
                     int32_t *d_rewards, uint8_t *d_dones, void *stream)
{
    if (check_bound(pool) != GEN_OK) return GEN_EINVAL;
    if (stream == nullptr) return fail(GEN_EINVAL, "capture needs a non-null stream");
    if (k_steps < 1 || k_steps > 100000) return fail(GEN_EINVAL, "k_steps %d outside [1, 100000]", k_steps);
    if (d_actions == nullptr || d_rewards == nullptr || d_dones == nullptr)
        return fail(GEN_EINVAL, "d_actions, d_rewards and d_dones are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (pool->exec) { (void)hipGraphExecDestroy(pool->exec); pool->exec = nullptr; }
    if (pool->graph) { (void)hipGraphDestroy(pool->graph); pool->graph = nullptr; }
    gen::PoolArgs a = pool_args(*pool);
    a.obs = d_obs;
    a.actions = d_actions;
    a.rewards = d_rewards;
    a.dones = d_dones;
    a.actor_seed = actor_seed;
    a.actor = 1u;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    for (int32_t k = 0; k < k_steps && e == hipSuccess; ++k) e = pool_step_launches(*pool, a, true, s);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e != hipSuccess ? e : e2, "capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "graph instantiate");
    }
    pool->graph = graph;
    pool->exec = exec;
    return ok();
}

int gen_pool_replay(gen_pool *pool, void *stream)
{
    if (check_bound(pool) != GEN_OK) return GEN_EINVAL;
    if (pool->exec == nullptr) return fail(GEN_EINVAL, "no captured graph (call gen_pool_capture)");
    hipError_t e = hipGraphLaunch(pool->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return ok();
}

int gen_pool_get_env(const gen_pool *pool, int32_t env, gen_host_state *h, void *stream)
{
    if (check_bound(pool) != GEN_OK) return GEN_EINVAL;
    if (env < 0 || env >= pool->n) return fail(GEN_EINVAL, "env %d outside [0, %d)", env, pool->n);
    if (h == nullptr || !h->owner || !h->army || !h->type || !h->turn || !h->episode || !h->alive || !h->finished ||
        !h->gpos)
        return fail(GEN_EINVAL, "host state has a NULL field");
    const gen::PoolDesc &d = pool->desc[(size_t)env];
    const int HW = d.H * d.W;
    const uint8_t *base = static_cast<const uint8_t *>(pool->d_state);
    gen::EnvScalars sc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(h->owner, base + pool->off_owner + d.cell_off, HW, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h->type, base + pool->off_type + d.cell_off, HW, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->army, base + pool->off_army + (uint64_t)d.cell_off * 4, (size_t)HW * 4,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&sc, base + pool->off_scalars + (uint64_t)env * sizeof(sc), sizeof(sc),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pool env download");
    h->turn[0] = sc.turn;
    h->episode[0] = sc.episode;
    h->alive[0] = sc.alive;
    h->finished[0] = sc.finished;
    for (int p = 0; p < d.P; ++p) h->gpos[p] = sc.gpos[p];
    return ok();
}

int gen_pool_get_state(const gen_pool *pool, gen_host_state *h, void *stream)
{
    if (check_bound(pool) != GEN_OK) return GEN_EINVAL;
    if (h == nullptr || !h->owner || !h->army || !h->type || !h->turn || !h->episode || !h->alive || !h->finished ||
        !h->gpos)
        return fail(GEN_EINVAL, "host state has a NULL field");
    std::vector<uint8_t> buf;
    try {
        buf.resize(pool->state_bytes);
    } catch (const std::bad_alloc &) {
        return fail(GEN_ENOMEM, "host allocation of %llu bytes failed", (unsigned long long)pool->state_bytes);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(buf.data(), pool->d_state, pool->state_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pool state download");
    const gen::EnvScalars *sc = reinterpret_cast<const gen::EnvScalars *>(buf.data() + pool->off_scalars);
    uint64_t cell = 0;   // first cell of env i in the ragged host rows
    for (int32_t i = 0; i < pool->n; ++i) {
        const gen::PoolDesc &d = pool->desc[(size_t)i];
        const size_t HW = (size_t)d.H * d.W;
        std::memcpy(h->owner + cell, buf.data() + pool->off_owner + d.cell_off, HW);
        std::memcpy(h->type + cell, buf.data() + pool->off_type + d.cell_off, HW);
        std::memcpy(h->army + cell, buf.data() + pool->off_army + (uint64_t)d.cell_off * 4, HW * 4);
        cell += HW;
        h->turn[i] = sc[i].turn;
        h->episode[i] = sc[i].episode;
        h->alive[i] = sc[i].alive;
        h->finished[i] = sc[i].finished;
        for (int p = 0; p < GEN_MAX_PLAYERS; ++p)
            h->gpos[(size_t)i * GEN_MAX_PLAYERS + p] = p < d.P ? sc[i].gpos[p] : (int16_t)-1;
    }
    return ok();
}

int gen_set_state(const gen_state *st, const gen_host_state *h, void *stream)
{
    if (check_state(st) != GEN_OK) return GEN_EINVAL;
    if (h == nullptr || !h->owner || !h->army || !h->type || !h->turn || !h->episode || !h->alive || !h->finished ||
        !h->gpos)
        return fail(GEN_EINVAL, "host state has a NULL field");
    const int HW = st->H * st->W, S = st->stride, P = st->n_players;
    for (int64_t i = 0; i < st->n_envs; ++i) {
        for (int c = 0; c < HW; ++c) {
            const int o = h->owner[i * HW + c], t = h->type[i * HW + c];
            if (o < -1 || o >= P) return fail(GEN_EINVAL, "env %lld cell %d: owner %d outside [-1, %d)", (long long)i, c, o, P);
            if (t > GEN_GENERAL) return fail(GEN_EINVAL, "env %lld cell %d: type %d outside [0, 3]", (long long)i, c, t);
            if (h->army[i * HW + c] < 0) return fail(GEN_EINVAL, "env %lld cell %d: negative army", (long long)i, c);
        }
        for (int p = 0; p < P; ++p) {
            const int g = h->gpos[i * P + p];
            if (g < 0 || g >= HW) return fail(GEN_EINVAL, "env %lld: general %d at cell %d outside the grid", (long long)i, p, g);
        }
        if (h->alive[i] >> P) return fail(GEN_EINVAL, "env %lld: alive mask has bits beyond %d players", (long long)i, P);
        if (h->turn[i] < 0) return fail(GEN_EINVAL, "env %lld: negative turn", (long long)i);
        if (h->finished[i] > 1) return fail(GEN_EINVAL, "env %lld: finished must be 0 or 1", (long long)i);
    }
    std::vector<uint8_t> buf(st->bytes, 0);
    gen::EnvScalars *sc = reinterpret_cast<gen::EnvScalars *>(buf.data() + st->off_scalars);
    for (int64_t i = 0; i < st->n_envs; ++i) {
        int8_t *ow = reinterpret_cast<int8_t *>(buf.data() + st->off_owner + i * S);
        std::memset(ow, 0xFF, S);   // padding cells: neutral
        std::memcpy(ow, h->owner + i * HW, HW);
        std::memcpy(buf.data() + st->off_type + i * S, h->type + i * HW, HW);
        std::memcpy(buf.data() + st->off_army + i * S * 4, h->army + i * HW, (size_t)HW * 4);
        sc[i].turn = h->turn[i];
        sc[i].episode = h->episode[i];
        sc[i].alive = h->alive[i];
        sc[i].finished = h->finished[i];
        for (int p = 0; p < gen::kMaxP; ++p) sc[i].gpos[p] = (int16_t)(p < P ? h->gpos[i * P + p] : -1);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(st->d_buf, buf.data(), st->bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "state upload");
    return ok();
}

}  // extern "C"
