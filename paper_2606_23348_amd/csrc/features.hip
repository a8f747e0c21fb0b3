// features.hip -- the paper's full feature tensor (Appendix A, table of
// observation channels; reading R17 of this library): 38 float32 maps per
// player and env, computed by one workgroup of 2, 4 or 8 wave64s per env
// from the env's state and a per-env memory in HBM (persistent masks, the
// last enemy sighting per cell, a ring of the last 8 frames).  Small batches
// (a training rollout's 512 envs) cannot fill the GPU with one wave per env,
// so their cells are spread over more waves.
//
// Memory traffic dominates (the output alone is 152 bytes per cell and
// player), so the kernel keeps every store coalesced: lane i of a round
// handles cell 64r + i, and each of the 38 channel stores of a player is one
// contiguous 256-byte wave store, nontemporal.  The state sits in LDS only
// for the ballots and the team-vision dilation.  A cell's 7 earlier frames
// are loaded from the ring before its 24 instantaneous channels are written,
// so their latency hides behind those stores; the delta stacks then walk the
// frames for all players with two running values per player.
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace gen {

namespace {

constexpr int kFeatC = 38;
constexpr int kHist = 7;

enum : uint32_t { B_SEEN = 1, B_ENEMY = 2, B_GENERAL = 4, B_CASTLE = 8, B_MOUNTAIN = 16 };

// Owned by a player outside p's team (team = p, and p ^ 2 in 2v2).
__device__ __forceinline__ bool enemy_of(int owner, int p, int mode)
{
    return owner >= 0 && owner != p && !(mode == MODE_2V2 && owner == (p ^ 2));
}

// Every per-env access goes through a raw buffer descriptor of the env's own
// block (base in scalar registers, bounds = the block), so a channel or
// memory-section offset is a scalar operand rather than a 64-bit address
// per lane, and an access past the block is dropped by the hardware.
constexpr int kNT = kAuxNT;                // cache policy of the stores: nontemporal

__device__ __forceinline__ Rsrc rsrc(void *base, uint32_t bytes) { return buffer_rsrc(base, bytes); }

}  // namespace

// log(1 + dt) / 5 (channel 21) for dt in [0, kAgeTable): filled once per
// device by host code from the host C library's double log1p, divided by 5
// in double and rounded once to float32; larger gaps are computed here in
// double the same way.
__device__ float g_age_table[kAgeTable];

namespace {

__device__ __forceinline__ float age_of(int32_t dt)
{
    if ((uint32_t)dt < (uint32_t)kAgeTable) return g_age_table[dt];
    return (float)(log1p((double)dt) / 5.0);
}

}  // namespace

// NT: the feature planes are whole 32-byte sectors (H*W a multiple of 8),
// so their stores can be nontemporal; otherwise two stores share the sector
// at each plane boundary and plain stores let the cache merge them.
template <bool NT>
__global__ __launch_bounds__(512) void k_features(FeatArgs a)
{
    constexpr int kOut = NT ? kNT : 0;        // cache policy of the feature and token stores
    extern __shared__ __align__(16) uint8_t smem[];
    const int e = (int)xcd_env(blockIdx.x, gridDim.x), lane = lane_id();   // see xcd_env
    const int tid = (int)threadIdx.x, nt = (int)blockDim.x;   // nt = 64 x (waves per env)
    const bool wave0 = readfirst(tid >> 6) == 0;
    const Geom g = a.g;
    const FeatBlock fb = a.blk;
    const int S = g.S, HW = g.HW, P = g.P;

    // LDS: owner [S] | type [S] | army int32 [S] | obm [P][16] | vis [P][16] |
    //      enemy army total [P] int64 | enemy land [P] int32 |
    //      army total [P] int64 | land [P] int32
    int8_t *Lo = reinterpret_cast<int8_t *>(smem);
    uint8_t *Lt = smem + S;
    int32_t *La = reinterpret_cast<int32_t *>(smem + 2 * S);
    uint64_t *obm = reinterpret_cast<uint64_t *>(smem + 6 * S);
    uint64_t *vis = obm + P * 16;
    int64_t *opp_army_l = reinterpret_cast<int64_t *>(vis + P * 16);
    int32_t *opp_land_l = reinterpret_cast<int32_t *>(opp_army_l + P);
    int64_t *armt_l = reinterpret_cast<int64_t *>(smem + 6 * S + 2 * P * 16 * 8 + 16 * P);
    int32_t *land_l = reinterpret_cast<int32_t *>(armt_l + P);

    const EnvScalars s = a.sc[e];
    {
        const size_t cell0 = (size_t)e * S;
        const uint4 *go = reinterpret_cast<const uint4 *>(a.owner + cell0);
        const uint4 *gt = reinterpret_cast<const uint4 *>(a.type + cell0);
        const uint4 *ga = reinterpret_cast<const uint4 *>(a.army + cell0);
        const int n16 = S >> 4;
        for (int i = tid; i < n16; i += nt) {
            reinterpret_cast<uint4 *>(Lo)[i] = go[i];
            reinterpret_cast<uint4 *>(Lt)[i] = gt[i];
        }
        for (int i = tid; i < 4 * n16; i += nt) reinterpret_cast<uint4 *>(La)[i] = ga[i];
    }
    // the memory header is read by every wave before the first barrier (the
    // last barrier orders its rewrite after all of them)
    uint8_t *blk = a.mem + (size_t)e * fb.bytes;
    uint32_t *hdr = reinterpret_cast<uint32_t *>(blk);
    const int32_t t = s.turn;
    const int slot = t & 7;
    const bool fresh = readfirst((int)hdr[0]) != (int)kFeatMagic || (uint32_t)readfirst((int)hdr[1]) != s.episode;
    int32_t stamp[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) stamp[j] = fresh ? -1 : readfirst((int)hdr[2 + j]);
    __syncthreads();

    // owned-cell bitmaps, team vision, land and army totals (wave 0; the
    // others wait at the barrier)
    int land[kMaxP];
    int64_t armt[kMaxP];
#pragma unroll
    for (int p = 0; p < kMaxP; ++p) { land[p] = 0; armt[p] = 0; }
    if (wave0) {
        for (int w = 0; w < g.NW; ++w) {
            const int c = w * 64 + lane;
            const int o = c < HW ? (int)Lo[c] : -1;
            for (int p = 0; p < P; ++p) {
                const uint64_t m = ballot(o == readfirst(p));
                if (lane == 0) obm[p * 16 + w] = m;
            }
            if (o >= 0) {
                const int32_t av = La[c];
#pragma unroll
                for (int p = 0; p < kMaxP; ++p)
                    if (o == p) { land[p] += 1; armt[p] += av; }
            }
        }
        wave_sync();
        team_vision(obm, vis, g);
#pragma unroll
        for (int p = 0; p < kMaxP; ++p) {
            if (p < P) {               // wave-uniform totals live in scalar registers
                land[p] = readfirst((int)wave_sum_u32((uint32_t)land[p]));
                const uint64_t at = (uint64_t)wave_sum_i64(armt[p]);
                armt[p] = (int64_t)(((uint64_t)(uint32_t)readfirst((int)(at >> 32)) << 32) |
                                    (uint32_t)readfirst((int)(uint32_t)at));
            }
        }
        // the enemies' totals of each player, kept in LDS for the scoreboard ring
        // (scalar registers are scarce across the cell loop), and the players'
        // own totals for the other waves
        if (lane < P) {
            int32_t ol = 0;
            int64_t oa = 0;
#pragma unroll
            for (int q = 0; q < kMaxP; ++q) {
                if (q < P && q != lane && !(g.mode == MODE_2V2 && q == (lane ^ 2))) {
                    ol += land[q];
                    oa += armt[q];
                }
            }
            opp_army_l[lane] = oa;
            opp_land_l[lane] = ol;
#pragma unroll
            for (int q = 0; q < kMaxP; ++q)
                if (q == lane) { armt_l[lane] = armt[q]; land_l[lane] = land[q]; }
        }
    }
    __syncthreads();
    if (!wave0) {
#pragma unroll
        for (int p = 0; p < kMaxP; ++p) {
            if (p < P) {
                land[p] = readfirst(land_l[p]);
                const uint64_t at = (uint64_t)armt_l[p];
                armt[p] = (int64_t)(((uint64_t)(uint32_t)readfirst((int)(at >> 32)) << 32) |
                                    (uint32_t)readfirst((int)(uint32_t)at));
            }
        }
    }

    // memory header: a block of another episode (or never used) starts empty
    uint32_t hv = 0;                  // bit k: the frame of turn t - k is in the ring
#pragma unroll
    for (int k = 1; k <= kHist; ++k) {
        const int32_t tau = t - k;
        if (tau >= 0 && stamp[tau & 7] == tau) hv |= 1u << k;
    }

    const float ch15 = (float)((double)(t % 50) / 50.0);
    float *fe = a.feat + (size_t)e * (size_t)P * kFeatC * HW;

    const Rsrc rm = rsrc(blk, fb.bytes);
    const Rsrc rf = rsrc(fe, (uint32_t)(P * kFeatC * HW * 4));
    for (int c = tid; c < HW; c += nt) {
        const int o = Lo[c], ty = Lt[c];
        const int32_t av = La[c];
        const int w = c >> 6, b = c & 63;
        uint32_t vb = 0;
        for (int p = 0; p < P; ++p) vb |= (uint32_t)((vis[p * 16 + w] >> b) & 1ull) << p;

        int hq[kHist];
        uint32_t hqv[kHist];
        int32_t hqa[kHist];
#pragma unroll
        for (int k = 0; k < kHist; ++k) {
            const int sl = (t - k - 1) & 7;
            const bool have = (hv >> (k + 1)) & 1u;
            hq[k] = have ? (int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(rm, c, (int)fb.fowner + sl * S, 0) : -1;
            hqv[k] = have ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rm, c, (int)fb.fvis + sl * S, 0) : 0u;
            hqa[k] = have ? (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rm, 4 * c, (int)fb.farmy + 4 * sl * S, 0) : 0;
        }
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)o, rm, c, (int)fb.fowner + slot * S, kNT);
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)vb, rm, c, (int)fb.fvis + slot * S, kNT);
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)av, rm, 4 * c, (int)fb.farmy + 4 * slot * S, kNT);

        const int row = div_w(c, g), col = c - row * g.W;
        const float cx = (float)((double)col / (double)(g.W - 1));
        const float cy = (float)((double)row / (double)(g.H - 1));

        int32_t own_prev[kMaxP], en_prev[kMaxP];
#pragma unroll
        for (int p = 0; p < kMaxP; ++p) {
            if (p >= P) break;
            const bool v = (vb >> p) & 1u;
            const bool en = enemy_of(o, p, g.mode);
            uint32_t bits = fresh ? 0u : (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rm, c, (int)fb.bits + p * S, 0);
            int32_t last = fresh ? 0 : (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rm, 4 * c, (int)fb.last + 4 * p * S, 0);
            int32_t lturn = fresh ? 0 : (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rm, 4 * c, (int)fb.lturn + 4 * p * S, 0);
            if (v) {
                bits |= B_SEEN;
                if (en) { bits |= B_ENEMY; lturn = t; }
                if (ty == GENERAL) bits |= B_GENERAL;
                if (ty == CASTLE) bits |= B_CASTLE;
                if (ty == MOUNTAIN) bits |= B_MOUNTAIN;
                last = en ? av : 0;
            }
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)bits, rm, c, (int)fb.bits + p * S, kNT);
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)last, rm, 4 * c, (int)fb.last + 4 * p * S, kNT);
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)lturn, rm, 4 * c, (int)fb.lturn + 4 * p * S, kNT);

            int32_t opp_land = 0;
            int64_t opp_army = 0;
#pragma unroll
            for (int q = 0; q < kMaxP; ++q) {
                if (q < P && q != p && !(g.mode == MODE_2V2 && q == (p ^ 2))) {
                    opp_land += land[q];
                    opp_army += armt[q];
                }
            }
            const int pb = p * kFeatC * HW * 4;
            auto put = [&](int ch, float x) {
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rf, 4 * c, pb + ch * HW * 4, kOut);
            };
            put(0, (float)(v ? av : 0));
            put(1, (float)(o == p ? av : 0));
            put(2, (float)(v && en ? av : 0));
            put(3, (float)(v && o < 0 ? av : 0));
            put(4, (float)(bits & 1u));
            put(5, (float)((bits >> 1) & 1u));
            put(6, (float)((bits >> 2) & 1u));
            put(7, (float)((bits >> 3) & 1u));
            put(8, (float)((bits >> 4) & 1u));
            put(9, (v && o < 0 && ty != MOUNTAIN) ? 1.0f : 0.0f);
            put(10, o == p ? 1.0f : 0.0f);
            put(11, (v && en) ? 1.0f : 0.0f);
            put(12, v ? 0.0f : 1.0f);
            put(13, (!v && (ty == MOUNTAIN || ty == CASTLE || (bits & B_GENERAL))) ? 1.0f : 0.0f);
            put(14, (float)t);
            put(15, ch15);
            put(16, (float)land[p]);
            put(17, (float)armt[p]);
            put(18, (float)opp_land);
            put(19, (float)opp_army);
            put(20, (float)last);
            put(21, (v || !(bits & B_ENEMY)) ? 0.0f : age_of(t - lturn));
            put(22, cx);
            put(23, cy);
            own_prev[p] = o == p ? av : 0;
            en_prev[p] = (v && en) ? av : 0;
        }

        // delta stacks: frame t-k-1 from the ring (absent: empty board)
#pragma unroll
        for (int k = 0; k < kHist; ++k) {
            const int q = hq[k];
            const uint32_t qv = hqv[k];
            const int32_t qa = hqa[k];
#pragma unroll
            for (int p = 0; p < kMaxP; ++p) {
                if (p >= P) break;
                const int pb = p * kFeatC * HW * 4;
                const int32_t own_k = q == p ? qa : 0;
                const int32_t en_k = (((qv >> p) & 1u) && enemy_of(q, p, g.mode)) ? qa : 0;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)(own_prev[p] - own_k)), rf, 4 * c,
                                                      pb + (24 + k) * HW * 4, kOut);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)(en_prev[p] - en_k)), rf, 4 * c,
                                                      pb + (24 + kHist + k) * HW * 4, kOut);
                own_prev[p] = own_k;
                en_prev[p] = en_k;
            }
        }
    }

    // scoreboard ring (Section V-A: the two temporal tokens): this turn's
    // enemy totals per player, then the 512-turn windows if asked for
    const int ts = t & (kTokenWindow - 1);
    for (int j = tid; j < kTokenWindow; j += nt) {
        if (fresh || j == ts)
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(j == ts ? t : -1), rm, 4 * j, (int)fb.tstamp, 0);
    }
    if (tid < P) {
        const int64_t oa = opp_army_l[tid];
        const int off = tid * kTokenWindow + ts;
        const u32x2 oav = {(uint32_t)(uint64_t)oa, (uint32_t)((uint64_t)oa >> 32)};
        __builtin_amdgcn_raw_buffer_store_b64(oav, rm, 8 * off, (int)fb.tarmy, 0);
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)opp_land_l[tid], rm, 4 * off, (int)fb.tland, 0);
    }
    if (a.tokens != nullptr) {
        const Rsrc rt = rsrc(a.tokens + (size_t)e * P * 2 * kTokenWindow, (uint32_t)(P * 2 * kTokenWindow * 4));
        for (int j = tid; j < kTokenWindow; j += nt) {
            const int32_t tau = t - (kTokenWindow - 1) + j;
            const int sl = tau & (kTokenWindow - 1);
            const bool now = j == kTokenWindow - 1;          // this turn: from registers
            const bool have = !now && !fresh && tau >= 0 &&
                              (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rm, 4 * sl, (int)fb.tstamp, 0) == tau;
#pragma unroll
            for (int p = 0; p < kMaxP; ++p) {
                if (p >= P) break;
                int64_t oa = 0;
                int32_t ol = 0;
                if (now) {
                    oa = opp_army_l[p];
                    ol = opp_land_l[p];
                } else if (have) {
                    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rm, 8 * (p * kTokenWindow + sl), (int)fb.tarmy, 0);
                    oa = (int64_t)(((uint64_t)v.y << 32) | v.x);
                    ol = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rm, 4 * (p * kTokenWindow + sl), (int)fb.tland, 0);
                }
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)oa), rt, 4 * j,
                                                      4 * (p * 2 * kTokenWindow), kOut);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)ol), rt, 4 * j,
                                                      4 * (p * 2 * kTokenWindow + kTokenWindow), kOut);
            }
        }
    }

    __syncthreads();
    if (tid == 0) {
        hdr[0] = kFeatMagic;
        hdr[1] = s.episode;
#pragma unroll
        for (int j = 0; j < 8; ++j) hdr[2 + j] = (uint32_t)(j == slot ? t : stamp[j]);
    }
}

namespace {
std::mutex g_age_mu;
bool g_age_ready[kMaxDevices] = {};
}  // namespace

hipError_t feature_tables_ready()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_age_mu);
    if (g_age_ready[dev]) return hipSuccess;
    std::vector<float> t(kAgeTable);
    for (int dt = 0; dt < kAgeTable; ++dt) t[(size_t)dt] = (float)(std::log1p((double)dt) / 5.0);
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_age_table), t.data(), t.size() * sizeof(float), 0, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) g_age_ready[dev] = true;
    return e;
}

hipError_t launch_features(const FeatArgs &a, int n_envs, hipStream_t stream)
{
    const uint32_t lds = (uint32_t)(6 * a.g.S + 2 * a.g.P * 16 * 8 + 28 * a.g.P);
    // waves per env: 8 for small batches and for more than 4 players (the
    // cell loop's work grows with P), 2 where 4 would leave a ragged last
    // round of waves on the chip, else 4 (fewer envs written at once, and
    // the ring loads of one env's cells overlap across its waves)
    const int nwv = (n_envs <= 1024 || a.g.P > 4) ? 8 : n_envs <= 2048 ? 2 : 4;
    if (a.g.HW % 8 == 0)
        hipLaunchKernelGGL(k_features<true>, dim3((unsigned)n_envs), dim3(kWave * nwv), lds, stream, a);
    else
        hipLaunchKernelGGL(k_features<false>, dim3((unsigned)n_envs), dim3(kWave * nwv), lds, stream, a);
    return hipGetLastError();
}

}  // namespace gen
