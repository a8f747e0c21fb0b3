// internal.hpp -- launch arguments and launchers shared by the host ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/generals.h"
#include "device.hpp"

namespace gen {

constexpr int kMaxDevices = 64;     // devices the library keeps per-device state for

struct EnvArgs {
    Geom g;
    GenParamsDev prm;
    uint64_t seed, env_base;
    EnvScalars *sc;
    int8_t *owner;
    uint8_t *type;
    int32_t *army;
    const int32_t *actions;
    uint8_t *obs;
    int32_t *rewards;
    uint8_t *dones;
    int32_t *land;
    int64_t *army_tot;
    int32_t *next_actions;        // fused actor output (nullptr: no actor)
    uint64_t actor_seed, step_idx;
};

struct SampleArgs {
    Geom g;
    uint64_t env_base, actor_seed, step_idx;
    const EnvScalars *sc;
    const int8_t *owner;
    const uint8_t *type;
    const int32_t *army;
    int32_t *actions;
};

struct PoolArgs {
    GenParamsDev prm;            // common settings; cities and spawn distance per env
    uint64_t seed, env_base, actor_seed;
    uint32_t n_envs, wpg, lds_per_wave;
    uint32_t slot_begin, slot_end;    // the segment of the work list this launch steps
    uint32_t actor;              // 1: draw the next actions after the step (ACT kernels)
    const PoolDesc *desc;        // work list: the descriptor of each slot's env
    EnvScalars *sc;
    int8_t *owner;
    uint8_t *type;
    int32_t *army;
    int32_t *actions;            // ragged int32, read and (with the actor) rewritten
    int32_t *rewards;
    uint8_t *dones;
    uint8_t *obs;
};

// One request of a served batch: one step of a group whose buffers all live
// in the server's arena (byte offsets from the arena base).
struct ServeReq {
    uint64_t off_desc, off_sc, off_owner, off_type, off_army;
    uint64_t off_actions, off_rewards, off_dones, off_obs;
    uint64_t seed, env_base, actor_seed;
    GenParamsDev prm;
    uint32_t n_envs, actor;
    // uniform != 0: every env of the group has tmpl's shape and settings,
    // cells_per_env cells and obs16_per_env 16-byte units of observation,
    // in env order, so the kernel derives each env's descriptor
    PoolDesc tmpl;
    uint32_t uniform, cells_per_env, obs16_per_env;
};

// One served launch, passed by value as the kernel argument so that a
// launch needs no host-to-device copy: the requests as indices into the
// server's table of group records (device memory, one record per open
// group, written when the group is admitted).
constexpr uint32_t kServeMaxReqs = 512;       // requests per launch
constexpr uint32_t kServeMaxGroups = 16384;   // open groups (16-bit indices)
struct ServeLaunch {
    uint8_t *arena;
    const ServeReq *groups;
    uint32_t n_req;
    uint32_t first[kServeMaxReqs];   // first workgroup of each request: 0, then running sums of n_envs
    uint16_t idx[kServeMaxReqs];
};
static_assert(sizeof(ServeReq) == 192, "group record size stated in generals.h");
static_assert(sizeof(ServeLaunch) <= 4096, "kernel arguments are limited to 4 KiB");

// One env's block of the feature memory (38-channel features), byte offsets:
//   header  64 B  {uint32 magic; uint32 episode; int32 stamp[8]; pad}
//           stamp[j] = turn of the frame held in ring slot j (-1: none)
//   bits    uint8 [P][S]   bit 0 seen, 1 enemy seen, 2 general seen,
//                          3 castle seen, 4 mountain seen
//   last    int32 [P][S]   enemy army at the cell's last visible frame
//   lturn   int32 [P][S]   turn of the last enemy sighting (valid with bit 1)
//   fowner  int8  [8][S]   ring of the last 8 frames, slot = turn mod 8:
//   fvis    uint8 [8][S]     owner, visibility (bit p: visible to p), army
//   farmy   int32 [8][S]
//   tstamp  int32 [512]    scoreboard ring, slot = turn mod 512: turn held (-1: none)
//   tarmy   int64 [P][512] army total of p's enemies at that turn
//   tland   int32 [P][512] their land
struct FeatBlock {
    uint32_t bits, last, lturn, fowner, fvis, farmy, tstamp, tarmy, tland, bytes;
};

constexpr int kTokenWindow = 512;

__host__ __device__ inline FeatBlock feat_block(int S, int P)
{
    FeatBlock b;
    b.bits = 64;
    b.last = b.bits + (uint32_t)(P * S);
    b.lturn = b.last + (uint32_t)(4 * P * S);
    b.fowner = b.lturn + (uint32_t)(4 * P * S);
    b.fvis = b.fowner + (uint32_t)(8 * S);
    b.farmy = b.fvis + (uint32_t)(8 * S);
    b.tstamp = b.farmy + (uint32_t)(32 * S);
    b.tarmy = b.tstamp + 4u * kTokenWindow;
    b.tland = b.tarmy + (uint32_t)(8 * P) * kTokenWindow;
    b.bytes = (b.tland + (uint32_t)(4 * P) * kTokenWindow + 255u) & ~255u;
    return b;
}

constexpr uint32_t kFeatMagic = 0x3846454Eu;   // header tag of a block in use

struct FeatArgs {
    Geom g;
    FeatBlock blk;
    const EnvScalars *sc;
    const int8_t *owner;
    const uint8_t *type;
    const int32_t *army;
    uint8_t *mem;
    float *feat;
    float *tokens;               // [E][P][2][512] or nullptr
};

hipError_t launch_features(const FeatArgs &a, int n_envs, hipStream_t stream);
// Entries of the channel-21 table (log(1 + dt) / 5 for dt below this).
constexpr int kAgeTable = 65536;
// Upload the feature kernel's tables to the current device once (blocking);
// called by every entry point that launches the features kernel.
hipError_t feature_tables_ready();

// Staging block of a gather of selected envs (byte offsets; each section is
// a host-format array of the selected envs, 256-byte aligned):
//   ids int32 [n] | owner int8 [n][HW] | type uint8 [n][HW] | army int32 [n][HW]
//   | turn int32 [n] | episode uint32 [n] | alive uint8 [n] | finished uint8 [n]
//   | gpos int16 [n][P]
struct GatherLayout {
    uint64_t ids, owner, type, army, turn, episode, alive, finished, gpos, bytes;
};

struct GatherArgs {
    GatherLayout lay;
    int32_t S, HW, P;
    const EnvScalars *sc;
    const int8_t *owner;
    const uint8_t *type;
    const int32_t *army;
    uint8_t *staging;
};

GatherLayout gather_layout(uint64_t n, uint64_t HW, uint64_t P);
hipError_t launch_gather(const GatherArgs &a, uint32_t n_ids, hipStream_t stream);
// Device address of the static staging array (GEN_STATIC_STAGING_BYTES) on
// `device`, which must be the current device; looked up once per device.
hipError_t static_staging(int device, void **out);
hipError_t launch_stream_copy(void *dst, const void *src, uint64_t n16, hipStream_t stream);
hipError_t launch_stream_spread(void *dst, const void *src, uint32_t n16, uint32_t k, hipStream_t stream);

uint32_t lds_bytes(const Geom &g);
uint32_t lds_bytes_for(int S, int P);
// One workgroup per env of the launch (total_envs = the requests' env
// counts summed): workgroup b steps env b - first[i] of request i, the last
// i with first[i] <= b.
// all_uniform: every request's group record has uniform set.
hipError_t launch_serve(const ServeLaunch &la, uint32_t total_envs, uint32_t lds, bool all_uniform, hipStream_t stream);
int obs_variant(int HW, int P);
hipError_t launch_pool(const PoolArgs &a, int kind, bool act, uint32_t grid, uint32_t nwv, hipStream_t stream);
hipError_t launch_step(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_reset(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_observe(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_sample(const SampleArgs &a, int n_envs, hipStream_t stream);

// Sets the calling thread's gen_last_error() message; returns code.
int set_error(int code, const char *msg);

inline GenParamsDev prm_of(const gen_params &p)
{
    GenParamsDev d;
    d.thresh = p.mountain_thresh;
    d.cmin = p.cities_min;
    d.cmax = p.cities_max;
    d.amin = p.city_army_min;
    d.amax = p.city_army_max;
    d.dmin = p.min_general_dist;
    d.auto_reset = p.auto_reset;
    d.pregrow = p.pregrow;
    d.generator = p.generator;
    d.dmax = p.max_general_dist;
    d.radius = p.castle_radius;
    return d;
}

}  // namespace gen

// Host plan of a batched pool (see generals.h).
struct gen_pool {
    uint64_t seed = 0, env_base = 0;
    int32_t n = 0;
    gen_params common{};
    std::vector<gen::PoolDesc> desc;      // in env order (the device copy is in work-list order)
    std::vector<uint64_t> work;           // P*H*W per env, for the work order
    std::vector<uint32_t> order;          // env of each work-list slot
    uint64_t off_scalars = 0, off_desc = 0, off_owner = 0, off_type = 0, off_army = 0;
    uint64_t state_bytes = 0, obs_bytes = 0, n_actions = 0;
    uint32_t lds_per_wave = 0;
    int32_t max_cells = 0;
    gen_pool_tuning tuning{1, 0, 0, 0};
    std::vector<gen_pool_bucket> buckets;  // per-bucket packing (gen_pool_set_buckets); empty = pool-wide
    // launches of a step: work-list segments [begin, end) sharing a packing
    struct Segment { uint32_t begin, end, wpg, nwv; };
    std::vector<Segment> segments;
    void *d_state = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
