// device.hpp -- gfx950 device helpers for the batched Generals.io step:
// Philox4x64-10 (map generator) and 4x32-10 (actor), wave64 primitives, SWAR byte tests, per-launch geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gen {

constexpr int kWave = 64;
constexpr int kMaxP = 8;
constexpr int kMaxCells = 1024;
constexpr int kMaxWords = 16;            // 64-bit words of a per-cell bitmap

enum : int { PLAIN = 0, MOUNTAIN = 1, CASTLE = 2, GENERAL = 3 };
enum : int { MODE_1V1 = 0, MODE_2V2 = 1, MODE_FFA = 2 };
enum : uint32_t { DOM_MAPGEN = 1, DOM_PREGROW = 3 };   // key words of the generator's streams

// 32-byte per-env record of the device layout (documented in generals.h).
struct __align__(16) EnvScalars {
    int32_t turn;
    uint32_t episode;
    uint8_t alive;
    uint8_t finished;
    uint8_t pad[2];
    uint32_t tick;          // steps applied since reset (batched pool: the actor's step index)
    int16_t gpos[8];
};
static_assert(sizeof(EnvScalars) == 32, "scalar record is 32 bytes");

// Geometry of one launch (all envs the same shape).
struct Geom {
    int H, W, HW, S, P, mode, NW;
    uint32_t magic_w;    // ceil(2^20 / W): c / W == (c * magic_w) >> 20 for c < 1024
    uint32_t magic_hw;   // ceil(2^32 / HW): b / HW == (b * magic_hw) >> 32 for b < 65536
    int PS;              // observation plane stride in bytes (HW, or HW padded to 32 bytes)
};

// Plane stride of a padded observation block (pool envs; plain batches with
// obs_layout 1): H*W rounded up to a multiple of 32 bytes, so every plane
// starts on its own 32-byte sector and nontemporal stores never write part
// of a sector another plane shares (measured on the mixed pool: 365 us per
// step with the unaligned-plane writer, 291 us with planes rounded to 4
// bytes, 283 us rounded to 32).  Envs of more than 2 players round to 64
// bytes: with 32 or more planes per env, planes that end in the middle of
// a 64-byte block cost 30-45% of the step (131,072-env pools, FFA-4 436 ->
// 304 us, 2v2 454 -> 308 us; 20x20 2v2, 400-byte planes: 188 -> 101 us);
// 1v1 envs and the mixed pool measured the same either way, and 64 bytes
// for every env slowed the served mix by 5%.
__host__ __device__ __forceinline__ int pool_plane_stride(int HW, int P)
{
    return P > 2 ? (HW + 63) & ~63 : (HW + 31) & ~31;
}

// Workgroup b of an n-workgroup grid -> the env it steps, so that the
// workgroups the dispatcher hands to one XCD (b mod 8, round robin) take a
// contiguous range of envs: neighbouring envs share 64-byte blocks of the
// scalar records, rewards, done flags and actions, and their partial writes
// then meet in the same XCD's L2 instead of reaching memory separately from
// different XCDs (plain batches, where every env has the same work: 1v1
// 24x24 144.3 -> 140.9 us, FFA-8 25x25 144.6 -> 139.4 us per step; the
// 38-channel features 3,271 -> 3,255 us).  Not
// for pools and served launches: their envs differ in work, and contiguous
// ranges unbalance the XCDs (served mix 3% slower).
__device__ __forceinline__ uint32_t xcd_env(uint32_t b, uint32_t n)
{
    const uint32_t x = b & 7u, i = b >> 3, per = n >> 3, rem = n & 7u;
    return x * per + min(x, rem) + i;
}

// The same for pools, by chunks of 32 slots: XCD x takes chunks x, x + 8,
// x + 16, ... of the work list, so neighbouring slots share an XCD while
// each XCD still samples the whole list (the envs differ in work); the
// slots past the last whole round of 8 chunks keep the plain order
// (mixed pool 281.7 -> 276.8 us per step; the served kernel, tried the same
// way, lost 2% on the served mix and keeps the plain order).
__device__ __forceinline__ uint32_t xcd_chunk32(uint32_t b, uint32_t n)
{
    constexpr uint32_t C = 32;
    const uint32_t full = n / (8u * C) * (8u * C);
    if (b >= full) return b;
    const uint32_t x = b & 7u, i = b >> 3;
    return ((i / C) * 8u + x) * C + i % C;
}

// Per-env descriptor of a batched pool (32 bytes, device resident).
struct PoolDesc {
    uint32_t cell_off;   // first cell of the env in the owner/type/army arrays (multiple of 16)
    uint32_t obs_off16;  // offset of the env's observation block ([P][8] planes of
                         // pool_plane_stride(H*W, P) bytes), in 16-byte units
    uint32_t act_off;    // first int32 of the env's actions and rewards
    uint32_t magic_w, magic_hw;
    uint8_t H, W, mode, P;
    uint8_t cmin, cmax, dmin, pad8;
    uint32_t env;        // the env's index in the pool (the device array is in work-list order)
};
static_assert(sizeof(PoolDesc) == 32, "pool descriptor is 32 bytes");

struct GenParamsDev {
    uint32_t thresh;
    int cmin, cmax, amin, amax, dmin, auto_reset, pregrow;
    int generator, dmax, radius;     // official generator: BFS spacing cap, castle radius
};

// ---------------------------------------------------------------- wave ops
// Make LDS writes of one lane visible to the other lanes of the same wave and
// keep the compiler from moving LDS accesses across this point.  What it
// relies on: (1) the release fence makes the wave wait for its own
// outstanding LDS operations (s_waitcnt lgkmcnt(0)) before anything after
// it issues, and the acquire fence keeps later LDS reads after that point;
// (2) the wave barrier is a compiler-only barrier for one wave (its lanes
// run in lockstep, so no hardware barrier is needed); (3) LDS accesses of
// one wave take effect in the order the wave issues them.  Code between
// two wave_sync calls may read a location another lane wrote only if the
// write came before the first call.  Data passed through registers
// (readlane, ds_bpermute, DPP) needs no wave_sync.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Value of `v` held by lane `src` (any lane index; taken mod 64).  Call it
// with every lane of the wave active: ds_bpermute returns 0 for a source
// lane that is masked off, so a shuffle inside a divergent branch loses data.
__device__ __forceinline__ uint32_t shfl32(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((src & 63) << 2, (int)v);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    uint32_t lo = shfl32((uint32_t)v, src), hi = shfl32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Broadcast of a wave-uniform lane's value.
__device__ __forceinline__ int readlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ int readfirst(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    for (int d = 32; d >= 1; d >>= 1) v += shfl32(v, lane_id() ^ d);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    for (int d = 32; d >= 1; d >>= 1) v += (int64_t)shfl64((uint64_t)v, lane_id() ^ d);
    return v;
}

// Lane i receives v of lane i - 1, lane 0 receives `first` (a DPP wave
// shift; every lane of the wave must be active).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v, uint32_t first)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)first, (int)v, 0x138, 0xF, 0xF, false);
}

// Raw buffer descriptor of one block of device memory (base in scalar
// registers, bounds = the block): offsets become scalar or 32-bit vector
// operands, and an access past the block is dropped by the hardware.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRawWord3 = 0x00020000;      // gfx9-family raw (stride 0) buffer descriptor flags
constexpr int kAuxNT = 2;                  // buffer store cache policy: nontemporal

__device__ __forceinline__ Rsrc buffer_rsrc(void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, kRawWord3);
}

// Inclusive prefix sum over the wave (lane order), in DPP moves: shifts by
// 1, 2, 4 and 8 lanes within each row of 16 (lanes shifted in from outside
// the row add 0), then the last lane of row 0 added to row 1 and that of
// row 2 to row 3, then the last lane of row 1 added to rows 2 and 3.  Every
// lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15, rows 1 and 3
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31, rows 2 and 3
    return v;
}

// ---------------------------------------------------------------- Philox4x64-10
// 64x64 -> 128-bit product as four 32x32+64 multiply-adds (v_mad_u64_u32 on
// the vector unit): t = a0 m0, u = a1 m0 + hi(t), v = a0 m1 + lo(u); then
// a m = lo(t) + 2^32 lo(v) + 2^64 (a1 m1 + hi(u) + hi(v)), no sum overflowing.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t m, uint64_t &lo, uint64_t &hi)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
    const uint64_t t = (uint64_t)a0 * m0;
    const uint64_t u = (uint64_t)a1 * m0 + (t >> 32);
    const uint64_t v = (uint64_t)a0 * m1 + (uint32_t)u;
    hi = (uint64_t)a1 * m1 + (u >> 32) + (v >> 32);
    lo = (v << 32) | (uint32_t)t;
}

// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of two 64x64->128 multiplies; the key advances by the
// two Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t &x0, uint64_t &x1, uint64_t &x2, uint64_t &x3,
                                              uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t lo0, hi0, lo1, hi1;
        mulhilo64(x0, M0, lo0, hi0);
        mulhilo64(x2, M1, lo1, hi1);
        const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
        k0 += W0; k1 += W1;
    }
}

// Philox4x32-10 (same paper): the 32-bit member of the family, one
// 32x32 -> 64-bit multiply-add per product.
__device__ __forceinline__ void philox4x32_10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0, y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The random actor's block of one env and step (reading R15): lanes 0..31
// compute the block of players 0..3, lanes 32..63 that of players 4..7 (the
// counter's top bit flipped), both in the same vector instructions.  Returns
// this lane's block packed as two 64-bit words: player p's draw is 32-bit
// half p % 2 (low first) of word (p / 2) % 2 of the block of lane 32 * (p / 4).
__device__ __forceinline__ void actor_block(uint64_t seed, uint64_t env_id, uint64_t step, uint64_t &w0,
                                            uint64_t &w1)
{
    // the lane-dependent counter word keeps the block on the vector unit
    uint32_t x0 = (uint32_t)step, x1 = (uint32_t)(step >> 32), x2 = (uint32_t)env_id;
    uint32_t x3 = (uint32_t)(env_id >> 32) ^ (lane_id() >= 32 ? 0x80000000u : 0u);
    philox4x32_10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    w0 = (uint64_t)x0 | ((uint64_t)x1 << 32);
    w1 = (uint64_t)x2 | ((uint64_t)x3 << 32);
}

// 32-bit draw j of the stream keyed (seed, dom) with counter prefix (c0, c1, c2):
// block j/8 is counter word 3; 64-bit word (j/2)%4; low half first.
__device__ __forceinline__ uint32_t draw32(uint64_t seed, uint32_t dom, uint64_t c0, uint64_t c1, uint64_t c2,
                                           uint32_t j)
{
    uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = j >> 3;
    philox4x64_10(x0, x1, x2, x3, seed, dom);
    const uint32_t w = (j >> 1) & 3;
    const uint64_t v = w == 0 ? x0 : w == 1 ? x1 : w == 2 ? x2 : x3;
    return (j & 1) ? (uint32_t)(v >> 32) : (uint32_t)v;
}

// Uniform pick in [0, n): floor(r * n / 2^32).
__device__ __forceinline__ uint32_t pick(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }

// ---------------------------------------------------------------- SWAR bytes
// 0x01 in every byte of x equal to the byte b, else 0x00 (exact, no carries
// across bytes).
__device__ __forceinline__ uint32_t bytes_eq(uint32_t x, uint32_t b)
{
    const uint32_t d = x ^ (b * 0x01010101u);
    const uint32_t t = ((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d;
    return (~t >> 7) & 0x01010101u;
}

// Bits 0..3 of v to 0x01 in bytes 0..3.
__device__ __forceinline__ uint32_t spread4(uint32_t v) { return (v * 0x00204081u) & 0x01010101u; }

__device__ __forceinline__ int32_t sat_add(int32_t a, int32_t b)
{
    const int64_t s = (int64_t)a + (int64_t)b;
    return s > INT32_MAX ? INT32_MAX : (int32_t)s;
}

__device__ __forceinline__ int div_w(int c, const Geom &g) { return (int)(((uint32_t)c * g.magic_w) >> 20); }
__device__ __forceinline__ uint32_t div_hw(uint32_t b, const Geom &g)
{
    return (uint32_t)(((uint64_t)b * g.magic_hw) >> 32);
}

// Bit positions b of word w (cell 64w + b) that lie in column 0 / column W-1,
// and the positions that are real cells (< HW).
struct ColMasks { uint64_t col0, colL, valid; };

// Bits 0, W, 2W, ... of a word (wave-uniform W: a short scalar loop).
__device__ __forceinline__ uint64_t col_pattern(int W)
{
    uint64_t m = 0;
    for (int b = 0; b < 64; b += W) m |= 1ull << b;
    return m;
}

__device__ __forceinline__ ColMasks col_masks(int w, const Geom &g)
{
    ColMasks m;
    const uint64_t pat = col_pattern(g.W);
    const int c0 = 64 * w;                             // first cell of the word (< 1024)
    const int r0 = c0 - g.W * div_w(c0, g);           // its column
    // cells of column 0 sit at positions == -r0 (mod W), of column W-1 at W-1-r0
    m.col0 = pat << (r0 == 0 ? 0 : g.W - r0);
    m.colL = pat << (g.W - 1 - r0);
    const int left = g.HW - c0;
    m.valid = left >= 64 ? ~0ull : left <= 0 ? 0ull : ((1ull << left) - 1);
    return m;
}

// ---------------------------------------------------------------- streaming stores
// Observation planes and the state are written once per step and not read
// again by the same launch; nontemporal stores keep them from crowding the
// caches (measured: a step at the copy ceiling instead of 20% below it).
// Only for whole, sector-aligned runs: where two stores share a 32-byte
// sector (unaligned observation planes) plain stores are faster.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void st_nt(uint32_t *p, uint32_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(uint2 *p, uint2 v)
{
    const u32x2 x = {v.x, v.y};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x2 *>(p));
}
__device__ __forceinline__ void st_nt(uint4 *p, uint4 v)
{
    const u32x4 x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x4 *>(p));
}

// Fog (Section IV-B; team vision R10): vis[p] = the 8-neighbour dilation of
// the cells of p's team (p, and p ^ 2 in 2v2), horizontal 3 then vertical 3
// on the row-major cell bitmaps.  obm and vis are [P][16] words in LDS; lane
// (p, w) of each round handles word w of player p, 64 / NW players a round.
// Every lane must call it (the shuffles read neighbouring words).
__device__ __forceinline__ void team_vision(const uint64_t *obm, uint64_t *vis, const Geom &g)
{
    const int lane = lane_id();
    const int ppr = kWave / g.NW;
    const int lp = lane / g.NW, w = lane - lp * g.NW;
    const ColMasks cm = col_masks(w, g);
    for (int p0 = 0; p0 < g.P; p0 += ppr) {
        const int p = p0 + lp;
        const bool valid = lp < ppr && p < g.P;
        uint64_t m = valid ? obm[p * 16 + w] : 0ull;
        if (valid && g.mode == MODE_2V2) m |= obm[(p ^ 2) * 16 + w];
        uint64_t mp = shfl64(m, lane - 1), mn = shfl64(m, lane + 1);
        if (w == 0) mp = 0ull;
        if (w == g.NW - 1) mn = 0ull;
        const uint64_t h = m | (((m << 1) | (mp >> 63)) & ~cm.col0) | (((m >> 1) | (mn << 63)) & ~cm.colL);
        uint64_t hp = shfl64(h, lane - 1), hn = shfl64(h, lane + 1);
        if (w == 0) hp = 0ull;
        if (w == g.NW - 1) hn = 0ull;
        const uint64_t v = (h | (h << g.W) | (hp >> (64 - g.W)) | (h >> g.W) | (hn << (64 - g.W))) & cm.valid;
        if (valid) vis[p * 16 + w] = v;
    }
}

// Position of the idx-th set bit (idx < popcount) of a bitmap of nw words.
__device__ __forceinline__ int bm_select(const uint64_t *bm, int nw, uint32_t idx)
{
    for (int w = 0; w < nw; ++w) {
        uint64_t x = bm[w];
        const uint32_t pc = (uint32_t)__popcll(x);
        if (idx < pc) {
            int base = 0;
            for (int width = 32; width >= 1; width >>= 1) {
                const uint32_t c = (uint32_t)__popcll(x & ((1ull << width) - 1));
                if (idx >= c) { idx -= c; x >>= width; base += width; }
            }
            return w * 64 + base;
        }
        idx -= pc;
    }
    return -1;
}

}  // namespace gen
