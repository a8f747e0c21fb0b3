// kernels.hip -- gfx950 kernels of the batched Generals.io environment step
// (arxiv 2606.23348, Section IV).  One wave64 owns one environment: the grid
// (owner int8, type uint8, army int32) is loaded from HBM into LDS once, the
// whole step runs on it, and owner/army plus the uint8 observation stream
// back out with 16-byte stores.  No MFMA: nothing here is a contraction.
#include "device.hpp"
#include "internal.hpp"

namespace gen {

// ---------------------------------------------------------------- LDS carve-up
// Per env, S = padded cells per row (multiple of 16):
//   army  int32 [S] | owner int8 [S] | type uint8 [S] | armyc uint8 [S] + 16
//   obm   u64 [P][16]                 (cells owned by each player)
//   vis   u64 [P][16]                 (visible cell bitmaps)
//   gbm   u64 [3][16] + int32 [8]      (map generator scratch bitmaps, general cells)
//         + u64 [4]                    (the actor's Philox block, computed early)
struct Lds {
    int32_t *army;
    int8_t *owner;
    uint8_t *type;
    uint8_t *armyc;
    uint64_t *obm, *vis, *gbm;
};

uint32_t lds_bytes_for(int S, int P)
{
    return (uint32_t)(4 * S + S + S + (S + 16) + 8 * 16 * (2 * P + 3) + 32 + 32);
}

__device__ __forceinline__ Lds carve(uint8_t *smem, const Geom &g)
{
    Lds L;
    uint32_t o = 0;
    L.army = reinterpret_cast<int32_t *>(smem + o); o += 4 * g.S;
    L.owner = reinterpret_cast<int8_t *>(smem + o); o += g.S;
    L.type = smem + o; o += g.S;
    L.armyc = smem + o; o += g.S + 16;
    L.obm = reinterpret_cast<uint64_t *>(smem + o); o += 8 * 16 * g.P;
    L.vis = reinterpret_cast<uint64_t *>(smem + o); o += 8 * 16 * g.P;
    L.gbm = reinterpret_cast<uint64_t *>(smem + o);
    return L;
}

// ---------------------------------------------------------------- map generation
// Cells within BFS distance r of `src` (4-neighbour steps over the passable
// bitmap), for up to three radii in one sweep: lane w < NW gets word w of
// each set.  r < 0 means unlimited (the connected component).  Layer by
// layer bitmap dilation (like the fog, with 4 instead of 8 neighbours) until
// the last requested radius or a fixpoint.  Every lane must call it.
struct Reach3 { uint64_t a, b, c; };

__device__ Reach3 bfs_reach(const uint64_t *pass, int src, int ra, int rb, int rc, const Geom &g)
{
    const int lane = lane_id(), NW = g.NW, W = g.W;
    const ColMasks cm = col_masks(lane < NW ? lane : 0, g);
    const uint64_t pw = lane < NW ? pass[lane] : 0ull;
    uint64_t cw = (lane == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    Reach3 out{cw, cw, cw};
    const int rmax = (ra < 0 || rb < 0 || rc < 0) ? INT32_MAX : max(ra, max(rb, rc));
    for (int r = 1; r <= rmax; ++r) {
        const uint64_t prev = shfl64(cw, lane - 1), next = shfl64(cw, lane + 1);
        const uint64_t pv = lane > 0 ? prev : 0ull, nx = lane < NW - 1 ? next : 0ull;
        uint64_t n = cw;
        n |= ((cw << 1) | (pv >> 63)) & ~cm.col0;
        n |= ((cw >> 1) | (nx << 63)) & ~cm.colL;
        n |= (cw << W) | (pv >> (64 - W));
        n |= (cw >> W) | (nx << (64 - W));
        n &= pw;
        const bool changed = ballot(n != cw) != 0ull;
        cw = n;
        if (ra < 0 || r <= ra) out.a = cw;
        if (rb < 0 || r <= rb) out.b = cw;
        if (rc < 0 || r <= rc) out.c = cw;
        if (!changed) break;
    }
    return out;
}

// The official rules after G1/G2 (reading R18): each further general among
// the cells whose BFS distance to every earlier general lies in
// [dmin, dmax], the castle count, a castle within the radius of every
// general that has none, the rest anywhere.  `j` is the next draw index.
// Returns false when this attempt has to be abandoned.
__device__ bool mapgen_official(const Lds &L, const Geom &g, const GenParamsDev &prm, uint64_t seed,
                                uint64_t env_id, uint32_t episode, int attempt, uint32_t &j, int *gp)
{
    const int lane = lane_id(), NW = g.NW, HW = g.HW;
    const uint64_t *pass = L.gbm;
    uint64_t *cand = L.gbm + 32;
    const int lo_r = prm.dmin - 1;                       // cells within dmin-1 are too close
    const int hi_r = prm.dmax > 0 ? prm.dmax : -1;
    uint64_t acc = lane < NW ? pass[lane] : 0ull;        // word `lane` of the candidate set
    uint64_t gens = 0ull;                                // word `lane` of the general cells
    for (int i = 0;; ++i) {
        const int gi = gp[i];
        if (lane == (gi >> 6)) gens |= 1ull << (gi & 63);
        if (i == g.P - 1) break;
        const Reach3 r = bfs_reach(pass, gi, lo_r < 0 ? 0 : lo_r, hi_r, 0, g);
        acc &= r.b & (lo_r < 0 ? ~0ull : ~r.a);
        acc &= ~gens;
        if (lane < NW) cand[lane] = acc;
        const uint32_t n = (uint32_t)readfirst((int)wave_sum_u32(lane < NW ? (uint32_t)__popcll(acc) : 0u));
        wave_sync();
        if (n == 0) return false;
        const int gn = bm_select(cand, NW, pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++), n));
        if (lane == 0) { gp[i + 1] = gn; L.type[gn] = GENERAL; }
        wave_sync();
    }
    const int ncas = prm.cmin + (int)pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++),
                                          (uint32_t)(prm.cmax - prm.cmin + 1));
    uint64_t cas = 0ull;                                 // word `lane` of the castle cells
    int placed = 0;
    for (int i = 0; i < g.P; ++i) {
        const Reach3 r = bfs_reach(pass, gp[i], prm.radius, 0, 0, g);
        if (ballot((r.a & cas) != 0ull) != 0ull) continue;
        const uint64_t c_w = lane < NW ? (r.a & pass[lane] & ~gens & ~cas) : 0ull;
        if (lane < NW) cand[lane] = c_w;
        const uint32_t n = (uint32_t)readfirst((int)wave_sum_u32((uint32_t)__popcll(c_w)));
        wave_sync();
        if (n == 0) return false;
        const int c = bm_select(cand, NW, pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++), n));
        const int32_t a = prm.amin + (int32_t)pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++),
                                                   (uint32_t)(prm.amax - prm.amin + 1));
        if (lane == 0) { L.type[c] = CASTLE; L.army[c] = a; }
        if (lane == (c >> 6)) cas |= 1ull << (c & 63);
        ++placed;
        wave_sync();
    }
    for (int t = placed; t < ncas; ++t) {
        uint32_t n = 0;
        for (int w = 0; w < NW; ++w) {
            const int c = w * 64 + lane;
            const uint64_t m = ballot(c < HW && L.type[c] == PLAIN);
            if (lane == 0) cand[w] = m;
            n += (uint32_t)__popcll(m);
        }
        wave_sync();
        if (n == 0) break;
        const int c = bm_select(cand, NW, pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++), n));
        const int32_t a = prm.amin + (int32_t)pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++),
                                                   (uint32_t)(prm.amax - prm.amin + 1));
        if (lane == 0) { L.type[c] = CASTLE; L.army[c] = a; }
        wave_sync();
    }
    return true;
}

// Section IV-A generator family (reading R14; the official rules, R18).  Executed by the whole wave
// with uniform control flow; every random choice is a Philox draw indexed
// exactly as the generator's draw order defines.  Leaves the grid in LDS and
// the scalars in `s`.
__device__ void mapgen_wave(const Lds &L, const Geom &g, const GenParamsDev &prm, uint64_t seed, uint64_t env_id,
                            uint32_t episode, EnvScalars &s)
{
    const int lane = lane_id();
    const int HW = g.HW, W = g.W, NW = g.NW;
    uint64_t *pass = L.gbm, *comp = L.gbm + 16, *cand = L.gbm + 32;
    int *gp = reinterpret_cast<int *>(L.gbm + 48);   // general cells, written by lane 0
    bool placed = false;

    for (int attempt = 0; attempt < 128 && !placed; ++attempt) {
        const uint32_t T = attempt < 64 ? prm.thresh : 0u;
        // G1: one draw per cell; a Philox block gives the draws of 8 cells.
        for (int b = lane; b * 8 < g.S; b += kWave) {
            uint64_t x0 = env_id, x1 = episode, x2 = (uint64_t)attempt, x3 = (uint64_t)b;
            philox4x64_10(x0, x1, x2, x3, seed, DOM_MAPGEN);
            const uint64_t w4[4] = {x0, x1, x2, x3};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int c = b * 8 + t;
                const uint32_t r = (t & 1) ? (uint32_t)(w4[t >> 1] >> 32) : (uint32_t)w4[t >> 1];
                if (c < g.S) {
                    L.type[c] = (c < HW && r < T) ? MOUNTAIN : PLAIN;
                    L.owner[c] = -1;
                    L.army[c] = 0;
                }
            }
        }
        wave_sync();
        // passable bitmap and its population
        uint32_t K = 0;
        for (int w = 0; w < NW; ++w) {
            const int c = w * 64 + lane;
            const uint64_t m = ballot(c < HW && L.type[c] != MOUNTAIN);
            if (lane == 0) pass[w] = m;
            K += (uint32_t)__popcll(m);
        }
        wave_sync();
        if (K == 0) continue;
        uint32_t j = (uint32_t)HW;
        // G2: first general over the non-mountain cells in row-major order
        const int g0 = bm_select(pass, NW, pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++), K));
        if (lane == 0) { gp[0] = g0; L.type[g0] = GENERAL; }
        if (prm.generator == 1) {
            wave_sync();
            placed = mapgen_official(L, g, prm, seed, env_id, episode, attempt, j, gp);
            continue;
        }
        // G3: 4-connected component of gp[0] (bitmap flood fill to a fixpoint)
        {
            const ColMasks cm = col_masks(lane < NW ? lane : 0, g);
            const uint64_t pw = lane < NW ? pass[lane] : 0ull;
            uint64_t cw = (lane == (g0 >> 6)) ? (1ull << (g0 & 63)) : 0ull;
            for (;;) {
                const uint64_t prev = shfl64(cw, lane - 1), next = shfl64(cw, lane + 1);
                const uint64_t pv = lane > 0 ? prev : 0ull, nx = lane < NW - 1 ? next : 0ull;
                uint64_t n = cw;
                n |= ((cw << 1) | (pv >> 63)) & ~cm.col0;
                n |= ((cw >> 1) | (nx << 63)) & ~cm.colL;
                n |= (cw << W) | (pv >> (64 - W));
                n |= (cw >> W) | (nx << (64 - W));
                n &= pw;
                const bool changed = ballot(n != cw) != 0ull;
                cw = n;
                if (!changed) break;
            }
            if (lane < NW) comp[lane] = cw;
        }
        wave_sync();
        // G4: each further general in the component, far enough from all earlier ones
        bool ok = true;
        for (int i = 1; i < g.P; ++i) {
            uint32_t n = 0;
            for (int w = 0; w < NW; ++w) {
                const int c = w * 64 + lane;
                bool in = c < HW && ((comp[w] >> lane) & 1ull) && L.type[c] != GENERAL;
                if (in) {
                    const int r = div_w(c, g), col = c - r * W;
                    for (int k = 0; k < i; ++k) {
                        const int gr = div_w(gp[k], g), gc = gp[k] - gr * W;
                        const int d = abs(r - gr) + abs(col - gc);
                        if (d < prm.dmin) in = false;
                    }
                }
                const uint64_t m = ballot(in);
                if (lane == 0) cand[w] = m;
                n += (uint32_t)__popcll(m);
            }
            wave_sync();
            if (n == 0) { ok = false; break; }
            const int gi = bm_select(cand, NW, pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++), n));
            if (lane == 0) { gp[i] = gi; L.type[gi] = GENERAL; }
            wave_sync();
        }
        if (!ok) continue;
        // G5: cities on remaining plain cells anywhere
        const int ncity = prm.cmin + (int)pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++),
                                               (uint32_t)(prm.cmax - prm.cmin + 1));
        for (int t = 0; t < ncity; ++t) {
            uint32_t n = 0;
            for (int w = 0; w < NW; ++w) {
                const int c = w * 64 + lane;
                const uint64_t m = ballot(c < HW && L.type[c] == PLAIN);
                if (lane == 0) cand[w] = m;
                n += (uint32_t)__popcll(m);
            }
            wave_sync();
            if (n == 0) break;
            const int c = bm_select(cand, NW, pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++), n));
            const int32_t a = prm.amin + (int32_t)pick(draw32(seed, DOM_MAPGEN, env_id, episode, attempt, j++),
                                                       (uint32_t)(prm.amax - prm.amin + 1));
            if (lane == 0) { L.type[c] = CASTLE; L.army[c] = a; }
            wave_sync();
        }
        placed = true;
    }
    if (!placed) {
        // deterministic last resort: no mountains, no cities, fixed border cells
        for (int c = lane; c < g.S; c += kWave) { L.type[c] = PLAIN; L.owner[c] = -1; L.army[c] = 0; }
        if (lane == 0) {
            for (int i = 0; i < g.P; ++i) {
                const int r = (i == 0 || i == 2 || i == 4) ? 0 : (i == 1 || i == 3 || i == 5) ? g.H - 1 : g.H / 2;
                const int c = (i == 0 || i == 3 || i == 6) ? 0 : (i == 1 || i == 2 || i == 7) ? W - 1 : W / 2;
                gp[i] = r * W + c;
            }
        }
    }
    wave_sync();
    // G6: generals (plus pre-grown armies on the overflow-stress workload)
    if (lane == 0) {
        for (int i = 0; i < g.P; ++i) {
            const int c = gp[i];
            L.type[c] = GENERAL;
            L.owner[c] = (int8_t)i;
            int32_t a = 1;
            if (prm.pregrow && episode == 0 && (env_id & 3) == 0)
                a = 100000 + (int32_t)pick(draw32(seed, DOM_PREGROW, env_id, 0, 0, (uint32_t)i), 900001u);
            L.army[c] = a;
        }
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < kMaxP; ++i) s.gpos[i] = (int16_t)(i < g.P ? gp[i] : -1);
    s.turn = 0;
    s.episode = episode;
    s.alive = (uint8_t)((1u << g.P) - 1u);
    s.finished = 0;
    wave_sync();
}

// ---------------------------------------------------------------- moves (Section IV-D)
__device__ __forceinline__ bool is_ally(int mode, int a, int b) { return mode == MODE_2V2 && a != b && ((a ^ b) & 1) == 0; }

// Decode one action (on the lane of its player): source and destination
// cells and the half flag packed as src | dst << 10 | half << 20, or -1 when
// the code can never be legal (out of range, k = 0, off the grid, into a
// mountain -- mountains never change during a step).
__device__ __forceinline__ int decode_action(const Lds &L, const Geom &g, int32_t a)
{
    if (a < 0 || a >= g.HW * 9) return -1;
    const int src = a / 9, k = a - src * 9;
    if (k == 0) return -1;
    const int dir = (k - 1) & 3;
    int r = div_w(src, g), c = src - r * g.W;
    r += dir == 0 ? -1 : dir == 1 ? 1 : 0;
    c += dir == 2 ? -1 : dir == 3 ? 1 : 0;
    if (r < 0 || r >= g.H || c < 0 || c >= g.W) return -1;
    const int dst = r * g.W + c;
    if (L.type[dst] == MOUNTAIN) return -1;
    return src | (dst << 10) | ((k >= 5 ? 1 : 0) << 20);
}

// Apply player i's decoded move (a wave-uniform value), re-validating
// ownership and army at application time (R4/R5).  The five LDS values the
// move can need are read at once and made scalar, the decision runs on the
// scalar unit, and lane 0 writes the cells that change.  Returns the player
// whose general was captured (-1 if none); the captured general becomes a
// castle here.
__device__ int apply_move(const Lds &L, const Geom &g, const EnvScalars &s, int i, int packed)
{
    if (packed < 0 || !((s.alive >> i) & 1)) return -1;
    const int src = packed & 1023, dst = (packed >> 10) & 1023;     // neighbours, never equal
    const bool half = (packed >> 20) & 1;
    const int o_src = readfirst(L.owner[src]);
    const int32_t have = readfirst(L.army[src]);
    const int o = readfirst(L.owner[dst]);
    const int32_t d = readfirst(L.army[dst]);
    const int t = readfirst(L.type[dst]);
    if (o_src != i || have <= 1) return -1;
    const int32_t m = half ? (have >> 1) : have - 1;
    int o_new = o, victim = -1;
    int32_t d_new;
    if (o == i) {
        d_new = sat_add(d, m);
    } else if (o >= 0 && is_ally(g.mode, o, i)) {
        d_new = sat_add(d, m);
        o_new = i;
    } else if (m > d) {
        o_new = i;
        d_new = m - d;
        if (t == GENERAL) {
#pragma unroll
            for (int v = 0; v < kMaxP; ++v) {
                if (v < g.P && victim < 0 && s.gpos[v] == dst && ((s.alive >> v) & 1) && v != i &&
                    !is_ally(g.mode, v, i))
                    victim = v;
            }
        }
    } else {
        d_new = d - m;
    }
    if (lane_id() == 0) {
        L.army[src] = have - m;
        L.army[dst] = d_new;
        L.owner[dst] = (int8_t)o_new;
        if (victim >= 0) L.type[dst] = CASTLE;
    }
    return readfirst(victim);
}

// All players' moves in rotating priority (reading R5), captures applied at
// once by the whole wave (Section IV-E transfer, reading R9 halving).
// Returns true if a general was captured (the type row then changed).
__device__ bool resolve_moves(const Lds &L, const Geom &g, EnvScalars &s, int32_t my_action)
{
    const int lane = lane_id();
    bool captured = false;
    const int my_move = lane < g.P ? decode_action(L, g, my_action) : -1;
    for (int j = 0; j < g.P; ++j) {
        const int i = (s.turn + j) % g.P;
        const int packed = readlane(my_move, i);
        const int victim = apply_move(L, g, s, i, packed);
        wave_sync();
        if (victim >= 0) {
            for (int c = lane; c < g.HW; c += kWave) {
                if (L.owner[c] == victim) {
                    L.owner[c] = (int8_t)i;
                    L.army[c] = L.army[c] >> 1;
                }
            }
            s.alive = (uint8_t)(s.alive & ~(1u << victim));
            captured = true;
            wave_sync();
        }
    }
    return captured;
}

// ---------------------------------------------------------------- random legal actor (reading R15)
// Lane (p, w) holds word w of player p's bitmaps.  The legal moves of one
// direction are the player's cells with more than one unit whose neighbour
// in that direction is on the grid and not a mountain: one AND with the
// shifted passable bitmap.  A cell with d legal directions contributes 2d
// entries (all-but-one, then half) to the list [pass, (cell, k)...]; the
// uniform pick is located by a prefix over words and a binary search over
// the bits of one word.  own: [P][16] words, pass/big: [16] words in LDS;
// blk: the actor's two Philox4x32 blocks if the caller computed them.
__device__ void actor_wave(const Geom &g, const uint64_t *own, const uint64_t *pass, const uint64_t *big,
                           uint32_t alive, uint64_t actor_seed, uint64_t step_idx, uint64_t env_id, int32_t *act_out,
                           const uint64_t *blk = nullptr)
{
    const int lane = lane_id();
    const int NW = g.NW, W = g.W;
    const int ppr = kWave / NW;
    const int lp = lane / NW, w = lane - lp * NW;
    const ColMasks cm = col_masks(w, g);
    const uint64_t pw = pass[w];
    const uint64_t pprev = w > 0 ? pass[w - 1] : 0ull, pnext = w < NW - 1 ? pass[w + 1] : 0ull;
    const uint64_t up_ok = (pw << W) | (pprev >> (64 - W));          // cell c with c - W passable
    const uint64_t dn_ok = (pw >> W) | (pnext << (64 - W));          // c + W passable
    const uint64_t lf_ok = ((pw << 1) | (pprev >> 63)) & ~cm.col0;   // c - 1 passable, same row
    const uint64_t rt_ok = ((pw >> 1) | (pnext << 63)) & ~cm.colL;   // c + 1 passable, same row
    const uint64_t bw = big[w];
    // the actor's draws (reading R15): player p takes 32-bit half p % 2 of
    // r[p / 2], r0 r1 from the block of players 0..3, r2 r3 from that of 4..7
    uint64_t r0, r1, r2, r3;
    if (blk != nullptr) {                        // computed earlier by the caller (in LDS)
        r0 = blk[0]; r1 = blk[1]; r2 = blk[2]; r3 = blk[3];
    } else {
        uint64_t w0, w1;
        actor_block(actor_seed, env_id, step_idx, w0, w1);
        r0 = shfl64(w0, 0); r1 = shfl64(w1, 0); r2 = shfl64(w0, 32); r3 = shfl64(w1, 32);
    }
    for (int p0 = 0; p0 < g.P; p0 += ppr) {
        const int p = p0 + lp;
        const bool valid = lp < ppr && p < g.P;
        const uint64_t src = (valid && ((alive >> p) & 1u)) ? (own[p * 16 + w] & bw) : 0ull;
        const uint64_t lu = src & up_ok, ld = src & dn_ok, ll = src & lf_ok, lr = src & rt_ok;
        const uint32_t cnt = 2u * (uint32_t)(__popcll(lu) + __popcll(ld) + __popcll(ll) + __popcll(lr));
        const uint32_t incl = wave_incl_scan(cnt);
        const int first = lp * NW;
        // every lane takes part in both shuffles (an inactive source lane would read as 0)
        const uint32_t below = shfl32(incl, first - 1);
        const uint32_t upto = shfl32(incl, first + NW - 1);
        const uint32_t before = first > 0 ? below : 0u;
        const uint32_t total = upto - before;
        const uint32_t excl = incl - cnt - before;
        const uint64_t rw = (p >> 1) == 0 ? r0 : (p >> 1) == 1 ? r1 : (p >> 1) == 2 ? r2 : r3;
        const uint32_t r = (p & 1) ? (uint32_t)(rw >> 32) : (uint32_t)rw;
        const uint32_t idx = pick(r, 1u + total);
        const bool mine = valid && idx > 0 && excl <= idx - 1 && idx - 1 < excl + cnt;
        if (mine) {
            // entry t of this word lies in the last cell b whose earlier cells
            // hold at most t entries.  A cell's move count n = lu + ld + ll + lr
            // (0..4) as three bit planes, n = s0 + 2 s1 + 4 s2 (full adders; a
            // carry of the second level excludes those of the first), so the
            // entries of a set of cells are 2 (|s0| + 2 |s1| + 4 |s2|); the
            // search halves the word, then works on 32-bit halves.
            uint32_t t = idx - 1 - excl;
            const uint64_t xa = lu ^ ld, xb = ll ^ lr, c1 = lu & ld, c2 = ll & lr;
            const uint64_t s0 = xa ^ xb, c3 = xa & xb;
            const uint64_t s1 = c1 ^ c2 ^ c3, s2 = c1 & c2;
            uint32_t h0 = (uint32_t)s0, h1 = (uint32_t)s1, h2 = (uint32_t)s2;
            const uint32_t lo = 2u * (uint32_t)(__popc(h0) + 2 * __popc(h1) + 4 * __popc(h2));
            int b = 0;
            if (lo <= t) {
                b = 32;
                t -= lo;
                h0 = (uint32_t)(s0 >> 32); h1 = (uint32_t)(s1 >> 32); h2 = (uint32_t)(s2 >> 32);
            }
            int bl = 0;
            for (int st = 16; st >= 1; st >>= 1) {
                const uint32_t m = (1u << (bl + st)) - 1u;
                const uint32_t pre = 2u * (uint32_t)(__popc(h0 & m) + 2 * __popc(h1 & m) + 4 * __popc(h2 & m));
                if (pre <= t) bl += st;
            }
            b += bl;
            const uint32_t ml = (1u << bl) - 1u;
            uint32_t j = t - 2u * (uint32_t)(__popc(h0 & ml) + 2 * __popc(h1 & ml) + 4 * __popc(h2 & ml));
            const uint32_t dirs = (uint32_t)((lu >> b) & 1ull) | ((uint32_t)((ld >> b) & 1ull) << 1) |
                                  ((uint32_t)((ll >> b) & 1ull) << 2) | ((uint32_t)((lr >> b) & 1ull) << 3);
            const uint32_t nd = (uint32_t)__popc(dirs);
            int kbase = 1;
            if (j >= nd) { j -= nd; kbase = 5; }
            int dir = 0;
            for (int d = 0, seen = 0; d < 4; ++d) {
                if ((dirs >> d) & 1u) {
                    if ((uint32_t)seen == j) { dir = d; break; }
                    ++seen;
                }
            }
            act_out[p] = (w * 64 + b) * 9 + kbase + dir;
        } else if (valid && w == 0 && idx == 0) {
            act_out[p] = 0;
        }
    }
}

// ---------------------------------------------------------------- fused env kernel
enum { K_STEP = 0, K_RESET = 1, K_OBSERVE = 2 };
// Observation writers: planes of a multiple of 4 cells (dword aligned), any
// other size, or planes padded to a multiple of 4 bytes (the layout of a
// pool's ragged observations, so envs of every shape take the dword writer).
enum { OBS_QUAD = 0, OBS_STREAM = 1, OBS_PADDED = 2 };

// Player-independent bits of the four cells of quad q, one 0x01 per cell
// byte (SWAR over the owner and type bytes).
struct QuadCells {
    uint32_t o4;        // owner bytes
    uint32_t neutral;   // no owner
    uint32_t plain_n;   // no owner and not a mountain
    uint32_t mtn, cas, gen;
};

__device__ __forceinline__ QuadCells quad_cells(const Lds &L, int q)
{
    QuadCells c;
    c.o4 = reinterpret_cast<const uint32_t *>(L.owner)[q];
    const uint32_t t4 = reinterpret_cast<const uint32_t *>(L.type)[q];
    c.neutral = (c.o4 >> 7) & 0x01010101u;
    c.mtn = t4 & ~(t4 >> 1) & 0x01010101u;
    c.cas = (t4 >> 1) & ~t4 & 0x01010101u;
    c.gen = t4 & (t4 >> 1) & 0x01010101u;
    c.plain_n = c.neutral & ~c.mtn;
    return c;
}

// The eight observation dwords of quad q for player p (reading R16): one
// byte per cell, channel k in v[k].  ac: the quad's army bytes clamped to
// 255.  In 2v2 `ally` is p's teammate, otherwise p itself.
__device__ __forceinline__ void quad_planes(const Lds &L, const QuadCells &c, uint32_t ac, int p, uint32_t ally,
                                            int q, uint32_t v[8])
{
    const uint32_t vb = (uint32_t)(L.vis[p * 16 + (q >> 4)] >> ((q & 15) * 4)) & 0xFu;
    const uint32_t visb = spread4(vb);
    const uint32_t eqp = bytes_eq(c.o4, (uint32_t)p);
    const uint32_t eqa = ally == (uint32_t)p ? eqp : bytes_eq(c.o4, ally);
    v[0] = eqp;
    v[1] = (c.neutral ^ 0x01010101u) & ~eqp & ~eqa & visb;
    v[2] = c.plain_n & visb;
    v[3] = c.mtn & visb;
    v[4] = c.cas & visb;
    v[5] = c.gen & visb;
    v[6] = visb ^ 0x01010101u;
    v[7] = ac & (visb * 0xFFu);
}

// Quad q's dwords of player p's eight planes into the env's observation
// block ([P][8] planes of PS bytes), nontemporal; `keep` masks the bytes of
// cells past the map in a padded plane's last quad to zero.
// ro: buffer descriptor of the env's block; the plane offset is a scalar
// operand and 4q the one vector offset of all eight stores.
// AUX: the stores' cache policy (nontemporal by default: every plane these
// stores write starts on a 32-byte sector, so no sector is shared by two
// planes written at different times).
template <int AUX = kAuxNT>
__device__ __forceinline__ void quad_store(const Lds &L, const Geom &g, const Rsrc &ro, const QuadCells &qc,
                                           uint32_t ac, int p, int q, int PS, uint32_t keep = ~0u)
{
    const uint32_t ally = g.mode == MODE_2V2 ? (uint32_t)(p ^ 2) : (uint32_t)p;
    uint32_t v[8];
    quad_planes(L, qc, ac, p, ally, q, v);
#pragma unroll
    for (int ch = 0; ch < 8; ++ch)
        __builtin_amdgcn_raw_buffer_store_b32(v[ch] & keep, ro, 4 * q, (p * 8 + ch) * PS, AUX);
}

// Code bytes of the four cells of quad q for player p (bit k = channel k,
// k < 7; bit 6 set = fog): one register per quad for the stream writer,
// which extracts the channels one at a time.
__device__ __forceinline__ uint32_t code_quad(const Lds &L, int p, uint32_t ally, int q)
{
    const QuadCells c = quad_cells(L, q);
    const uint32_t vb = (uint32_t)(L.vis[p * 16 + (q >> 4)] >> ((q & 15) * 4)) & 0xFu;
    const uint32_t visb = spread4(vb);
    const uint32_t eqp = bytes_eq(c.o4, (uint32_t)p);
    const uint32_t eqa = ally == (uint32_t)p ? eqp : bytes_eq(c.o4, ally);
    const uint32_t enemy = (c.neutral ^ 0x01010101u) & ~eqp & ~eqa;
    return eqp | ((enemy & visb) << 1) | ((c.plain_n & visb) << 2) | ((c.mtn & visb) << 3) | ((c.cas & visb) << 4) |
           ((c.gen & visb) << 5) | ((visb ^ 0x01010101u) << 6);
}

// Army bytes of a quad on the cells its code bytes mark visible.
__device__ __forceinline__ uint32_t army_visible(uint32_t ac, uint32_t code4)
{
    return ac & ((((code4 >> 6) & 0x01010101u) ^ 0x01010101u) * 0xFFu);
}

// Code byte of one cell for player p (bit k = channel k < 7, as quad_planes), for the few
// output dwords that hold bytes of two planes.
__device__ __forceinline__ uint32_t code_cell(const Lds &L, int p, uint32_t ally, int c)
{
    const int o = L.owner[c];
    const uint32_t t = L.type[c];
    const bool vis = (L.vis[p * 16 + (c >> 6)] >> (c & 63)) & 1ull;
    const bool neutral = o < 0;
    const bool enemy = !neutral && o != p && (uint32_t)o != ally;
    uint32_t code = (o == p) ? 1u : 0u;
    if (vis) {
        code |= (enemy ? 2u : 0u) | ((neutral && t != (uint32_t)MOUNTAIN) ? 4u : 0u) |
                (t == (uint32_t)MOUNTAIN ? 8u : 0u) | (t == (uint32_t)CASTLE ? 16u : 0u) |
                (t == (uint32_t)GENERAL ? 32u : 0u);
    } else {
        code |= 64u;
    }
    return code;
}

// Observation byte b of the env block (plane b / HW, cell b % HW).
__device__ __forceinline__ uint32_t obs_byte(const Lds &L, const Geom &g, uint32_t b)
{
    const uint32_t q = div_hw(b, g), c = b - q * g.HW, p = q >> 3, ch = q & 7;
    const uint32_t ally = g.mode == MODE_2V2 ? (p ^ 2u) : p;
    const uint32_t cd = code_cell(L, (int)p, ally, (int)c);
    return ch < 7 ? (cd >> ch) & 1u : (((cd >> 6) & 1u) ? 0u : L.armyc[c]);
}

// Two waves per env: wave 0 writes the planes of players 0 .. obs_split(P) - 1
// and then runs the actor, wave 1 the rest (3 of 8 and 5 of 8 players
// balance the two; measured against 4 and 4: FFA-8 25x25 226 -> 217 us).
__device__ __forceinline__ int obs_split(int P) { return (P * 3) >> 3; }

// The unaligned-plane writer's main pass for players p_begin .. p_end - 1
// (every lane of the wave; the dwords that hold bytes of two planes are left
// to the caller's byte-wise pass).
__device__ __forceinline__ void obs_stream_planes(const Lds &L, const Geom &g, uint8_t *obs, int p_begin, int p_end)
{
    const int lane = lane_id();
    const int nq = g.HW >> 2;                                   // whole quads
    const int rounds = (nq + 1 + kWave - 1) / kWave;            // quads 0 .. nq
    const Rsrc ro = buffer_rsrc(obs, (uint32_t)(g.P * 8 * g.HW));
    const uint32_t HWu = (uint32_t)g.HW;
    const uint32_t m1 = HWu & 3u, m2 = (2u * HWu) & 3u, m3 = (3u * HWu) & 3u;
    const uint32_t M = 0x01010101u;
    for (int p = p_begin; p < p_end; ++p) {
        const uint32_t ally = g.mode == MODE_2V2 ? (uint32_t)(p ^ 2) : (uint32_t)p;
        const uint32_t pbase = (uint32_t)p * 8u * HWu;         // byte offset of plane (p, 0), a multiple of 8
        uint32_t carry_c = 0u, carry_a = 0u;
        for (int r = 0; r < rounds; ++r) {
            const int j = r * kWave + lane;
            const int qj = j < (g.S >> 2) ? j : 0;              // stays inside the padded row
            const uint32_t code = code_quad(L, p, ally, qj);
            const uint32_t ac = reinterpret_cast<const uint32_t *>(L.armyc)[qj];
            const uint32_t pc = wave_shr1(code, carry_c), pa = wave_shr1(ac, carry_a);
            carry_c = (uint32_t)readlane((int)code, kWave - 1);
            carry_a = (uint32_t)readlane((int)ac, kWave - 1);
            const uint32_t c1 = m1 == 0u ? code : __builtin_amdgcn_alignbyte(code, pc, 4u - m1);
            const uint32_t c2 = m2 == 0u ? code : __builtin_amdgcn_alignbyte(code, pc, 4u - m2);
            const uint32_t c3 = m3 == 0u ? code : __builtin_amdgcn_alignbyte(code, pc, 4u - m3);
            const uint32_t a3 = m3 == 0u ? ac : __builtin_amdgcn_alignbyte(ac, pa, 4u - m3);
            // interior: bytes 4j - m .. 4j - m + 3 all inside the plane.
            // Plain (cached) stores: the 32-byte sectors at plane
            // boundaries are shared by two stores and the cache merges
            // them; nontemporal partial-sector writes measured 1.5x
            // slower on these shapes.
            const int vo = 4 * j;
            if (vo + 4 <= g.HW) {
                __builtin_amdgcn_raw_buffer_store_b32(code & M, ro, vo, (int)(pbase & ~3u), 0);
                __builtin_amdgcn_raw_buffer_store_b32((code >> 4) & M, ro, vo, (int)((pbase + 4u * HWu) & ~3u), 0);
            }
            if (vo >= (int)m1 && vo + 4 - (int)m1 <= g.HW) {
                __builtin_amdgcn_raw_buffer_store_b32((c1 >> 1) & M, ro, vo, (int)((pbase + HWu) & ~3u), 0);
                __builtin_amdgcn_raw_buffer_store_b32((c1 >> 5) & M, ro, vo, (int)((pbase + 5u * HWu) & ~3u), 0);
            }
            if (vo >= (int)m2 && vo + 4 - (int)m2 <= g.HW) {
                __builtin_amdgcn_raw_buffer_store_b32((c2 >> 2) & M, ro, vo, (int)((pbase + 2u * HWu) & ~3u), 0);
                __builtin_amdgcn_raw_buffer_store_b32((c2 >> 6) & M, ro, vo, (int)((pbase + 6u * HWu) & ~3u), 0);
            }
            if (vo >= (int)m3 && vo + 4 - (int)m3 <= g.HW) {
                __builtin_amdgcn_raw_buffer_store_b32((c3 >> 3) & M, ro, vo, (int)((pbase + 3u * HWu) & ~3u), 0);
                __builtin_amdgcn_raw_buffer_store_b32(army_visible(a3, c3), ro, vo, (int)((pbase + 7u * HWu) & ~3u),
                                                      0);
            }
        }
    }
}

// Padded planes (plane stride g.PS, a multiple of 32 bytes): the dword
// writer for players p_begin .. p_end - 1, quads outer (a quad's cells
// decoded once for all those players; measured on the mixed pool: 286 ->
// 273 us per step against players outer); the bytes of cells past the map
// in a plane's last quads are written as zero.
__device__ __forceinline__ void obs_padded_planes(const Lds &L, const Geom &g, uint8_t *obs, int p_begin, int p_end)
{
    const int lane = lane_id();
    const int PS = g.PS;
    const int nq = PS >> 2;
    const int nfull = ((g.HW + 3) >> 2) - 1;                          // last quad holding map cells
    const uint32_t tail = (g.HW & 3) ? (1u << (8 * (g.HW & 3))) - 1u : ~0u;
    const Rsrc ro = buffer_rsrc(obs, (uint32_t)(g.P * 8 * PS));
    for (int q = lane; q < nq; q += kWave) {
        const QuadCells qc = quad_cells(L, q);
        const uint32_t ac = reinterpret_cast<const uint32_t *>(L.armyc)[q];
        const uint32_t keep = q < nfull ? ~0u : q == nfull ? tail : 0u;
        for (int p = p_begin; p < p_end; ++p) quad_store(L, g, ro, qc, ac, p, q, PS, keep);
    }
}

// Per-env inputs and outputs of one step (pointers into this env's rows).
struct EnvIO {
    EnvScalars *sc;
    int8_t *owner;
    uint8_t *type;
    int32_t *army;
    const int32_t *actions;     // P actions of this step
    int32_t *next_actions;      // fused actor output (ACT)
    int32_t *rewards;
    uint8_t *done;
    uint8_t *obs;               // this env's [P][8][H][W] block, nullptr = no observation
    int32_t *land;              // scoreboard (SB)
    int64_t *army_tot;
    uint64_t env_id;            // global id (keys every draw)
    uint64_t actor_step;        // actor step index when the tick is not used
    bool use_tick;              // keep the per-env step counter; the actor draws with it
    int nwv = 1;                // waves of the workgroup sharing the unaligned observation planes
};

// One environment step (or reset / observation) on one wave.  OBSV selects
// the observation writer and layout at compile time (OBS_PADDED for the
// mixed shapes of a pool).
template <int KIND, int OBSV, bool SB, bool ACT>
__device__ __forceinline__ void env_body(uint8_t *smem, const Geom &g, const GenParamsDev &prm, uint64_t seed,
                                         uint64_t actor_seed, const EnvIO &io)
{
    const int lane = lane_id();
    const Lds L = carve(smem, g);
    const uint64_t env_id = io.env_id;

    EnvScalars s;
    bool write_type = false, grow2 = false, grow50 = false, done = false;
    uint32_t win = 0, lose = 0;

    if (KIND == K_RESET) {
        mapgen_wave(L, g, prm, seed, env_id, 0u, s);
        s.tick = 0;
        write_type = true;
    } else {
        s = *io.sc;
        const int n16 = g.S >> 4;
        const uint4 *go = reinterpret_cast<const uint4 *>(io.owner);
        const uint4 *gt = reinterpret_cast<const uint4 *>(io.type);
        const uint4 *ga = reinterpret_cast<const uint4 *>(io.army);
        int32_t act = 0;
        if constexpr (ACT) {
            // state HBM -> registers (16-byte loads; S <= 1024 cells, so one
            // owner and one type chunk and at most four army chunks per
            // lane; indexes are clamped rather than the loads predicated:
            // lanes past the end re-read the last chunk and skip the store)
            const int na = 4 * n16;
            // two-wave envs issue their state loads at raised wave priority,
            // so a new env's loads are not queued behind older waves' work
            // (FFA-8 25x25: 216 -> 211 us; one-wave shapes unchanged)
            if (io.nwv > 1) __builtin_amdgcn_s_setprio(3);
            const uint4 vo = go[min(lane, n16 - 1)];
            const uint4 vt = gt[min(lane, n16 - 1)];
            const uint4 va0 = ga[min(lane, na - 1)];
            const uint4 va1 = ga[min(lane + 64, na - 1)];
            const uint4 va2 = ga[min(lane + 128, na - 1)];
            const uint4 va3 = ga[min(lane + 192, na - 1)];
            if (KIND == K_STEP && lane < g.P) act = io.actions[lane];
            if (io.nwv > 1) __builtin_amdgcn_s_setprio(0);
            // the actor's Philox blocks do not depend on the state:
            // computing them while the loads are in flight hides their
            // latency; they wait in LDS until the actor runs
            if (io.next_actions != nullptr) {
                const uint64_t tick = (uint64_t)s.tick + ((KIND == K_STEP && io.use_tick) ? 1u : 0u);
                uint64_t w0, w1;
                actor_block(actor_seed, env_id, io.use_tick ? tick : io.actor_step, w0, w1);
                if ((lane & 31) == 0) {
                    uint64_t *pb = L.gbm + 52 + (lane >> 4);
                    pb[0] = w0;
                    pb[1] = w1;
                }
            }
            if (lane < n16) {
                reinterpret_cast<uint4 *>(L.owner)[lane] = vo;
                reinterpret_cast<uint4 *>(L.type)[lane] = vt;
            }
            uint4 *la = reinterpret_cast<uint4 *>(L.army);
            if (lane < na) la[lane] = va0;
            if (lane + 64 < na) la[lane + 64] = va1;
            if (lane + 128 < na) la[lane + 128] = va2;
            if (lane + 192 < na) la[lane + 192] = va3;
        } else {
            // state HBM -> LDS, 16-byte loads
            for (int i = lane; i < n16; i += kWave) {
                reinterpret_cast<uint4 *>(L.owner)[i] = go[i];
                reinterpret_cast<uint4 *>(L.type)[i] = gt[i];
            }
            for (int i = lane; i < 4 * n16; i += kWave) reinterpret_cast<uint4 *>(L.army)[i] = ga[i];
            if (KIND == K_STEP && lane < g.P) act = io.actions[lane];
        }
        wave_sync();
        if (KIND == K_STEP) {
            if (io.use_tick) s.tick += 1;
            if (!s.finished) {
                const uint32_t alive0 = s.alive;
                write_type = resolve_moves(L, g, s, act);
                s.turn += 1;
                grow2 = (s.turn & 1) == 0;
                grow50 = (s.turn % 50) == 0;
                // terminal and rewards (Section III, Section IV-E; reading R11)
                const uint32_t alive = s.alive;
                if (g.mode == MODE_2V2) {
                    const bool t0 = (alive & 0x5u) != 0, t1 = (alive & 0xAu) != 0;
                    if (!t0 || !t1) {
                        done = true;
                        const uint32_t winners = t0 ? 0x5u : 0xAu;
                        win = winners;
                        lose = 0xFu & ~winners;
                    }
                } else {
                    lose = alive0 & ~alive;
                    if (__popc(alive) == 1) { done = true; win = alive; }
                }
                if (done) {
                    if (prm.auto_reset) {
                        mapgen_wave(L, g, prm, seed, env_id, s.episode + 1u, s);
                        write_type = true;
                        grow2 = grow50 = false;
                    } else {
                        s.finished = 1;
                    }
                }
            } else {
                done = true;
            }
        }
    }

    // ---- growth (Section IV-C), state store, army clamp, scoreboard
    int land_acc[kMaxP];
    int64_t army_acc[kMaxP];
    if (SB) {
#pragma unroll
        for (int p = 0; p < kMaxP; ++p) { land_acc[p] = 0; army_acc[p] = 0; }
    }
    {
        const int nq = g.S >> 2;
        uint32_t *go = reinterpret_cast<uint32_t *>(io.owner);
        uint32_t *gt = reinterpret_cast<uint32_t *>(io.type);
        int4 *ga = reinterpret_cast<int4 *>(io.army);
        for (int q = lane; q < nq; q += kWave) {
            const uint32_t o4 = reinterpret_cast<const uint32_t *>(L.owner)[q];
            const uint32_t t4 = reinterpret_cast<const uint32_t *>(L.type)[q];
            int4 a4 = reinterpret_cast<const int4 *>(L.army)[q];
            int32_t av[4] = {a4.x, a4.y, a4.z, a4.w};
            // one 0x01 per growing cell byte, without branches: owned (the
            // owner byte's sign bit clear) and a castle or general (type bit
            // 1) on even turns or plain (type 0) on multiples of 50; the
            // army never wraps (saturating add, reading R12)
            const uint32_t gm2 = grow2 ? 0x01010101u : 0u, gm50 = grow50 ? 0x01010101u : 0u;
            const uint32_t inc = (~o4 >> 7) & (((t4 >> 1) & gm2) | (~(t4 | (t4 >> 1)) & gm50));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int o = (int8_t)(o4 >> (8 * k));
                av[k] = __builtin_elementwise_add_sat(av[k], (int32_t)((inc >> (8 * k)) & 1u));
                if (SB) {
#pragma unroll
                    for (int p = 0; p < kMaxP; ++p) {
                        if (o == p) { land_acc[p] += 1; army_acc[p] += av[k]; }
                    }
                }
            }
            if (KIND != K_OBSERVE) {
                st_nt(reinterpret_cast<uint4 *>(ga + q),
                      make_uint4((uint32_t)av[0], (uint32_t)av[1], (uint32_t)av[2], (uint32_t)av[3]));
                st_nt(go + q, o4);
                if (write_type) st_nt(gt + q, t4);
            }
            uint32_t ac = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) ac |= (uint32_t)(av[k] > 255 ? 255 : av[k]) << (8 * k);
            reinterpret_cast<uint32_t *>(L.armyc)[q] = ac;
        }
    }
    if (SB) {
        for (int p = 0; p < g.P; ++p) {
            int lp = 0;
            int64_t ap = 0;
#pragma unroll
            for (int t = 0; t < kMaxP; ++t) if (t == p) { lp = land_acc[t]; ap = army_acc[t]; }
            lp = (int)wave_sum_u32((uint32_t)lp);
            ap = wave_sum_i64(ap);
            if (lane == 0) {
                io.land[p] = lp;
                io.army_tot[p] = ap;
            }
        }
    }

    // ---- per-player owned-cell bitmaps (one ballot per player per 64 cells);
    // with the fused actor also the passable and army > 1 bitmaps
    // The reads of cells past the map (c >= H*W, up to 63 bytes past a row)
    // stay inside the env's LDS block; a scalar mask drops their bits.
    for (int w = 0; w < g.NW; ++w) {
        const int c = w * 64 + lane;
        const int rem = g.HW - 64 * w;
        const uint64_t real = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
        const int o = L.owner[c];
        for (int p = 0; p < g.P; ++p) {
            // (the player index as an opaque scalar: one compare per ballot
            // rather than a strength-reduced running difference)
            const uint64_t m = ballot(o == readfirst(p)) & real;
            if (lane == 0) L.obm[p * 16 + w] = m;
        }
        if (ACT) {
            const uint64_t pm = ballot(L.type[c] != MOUNTAIN) & real;
            const uint64_t bm = ballot(L.armyc[c] > 1) & real;
            if (lane == 0) { L.gbm[w] = pm; L.gbm[16 + w] = bm; }
        }
    }
    wave_sync();

    // ---- fog (Section IV-B, team vision R10)
    team_vision(L.obm, L.vis, g);
    wave_sync();
    // a second wave of the workgroup (FFA with unaligned planes) waits here
    // for the state and the vision, then writes the later players' planes
    if ((OBSV == OBS_STREAM || OBSV == OBS_PADDED) && io.nwv > 1) __syncthreads();

    // Planes of a multiple of 4 cells: each lane takes 4 cells, computes their
    // bytes of all 8 channel planes in registers and stores them directly
    // (4-byte stores, 256 contiguous bytes per wave store).  Other shapes
    // realign the same dwords with lane shuffles below.
    if (OBSV == OBS_QUAD || OBSV == OBS_PADDED) {
        if (io.obs != nullptr) {
            // Quads outer: a quad's owner and type bits decoded once for
            // all players.
            if (OBSV == OBS_QUAD) {
                const int nq = g.HW >> 2;
                const Rsrc ro = buffer_rsrc(io.obs, (uint32_t)(g.P * 8 * g.HW));
                for (int q = lane; q < nq; q += kWave) {
                    const QuadCells qc = quad_cells(L, q);
                    const uint32_t ac = reinterpret_cast<const uint32_t *>(L.armyc)[q];
                    for (int p = 0; p < g.P; ++p) quad_store(L, g, ro, qc, ac, p, q, g.HW);
                }
            } else {
                obs_padded_planes(L, g, io.obs, 0, io.nwv > 1 ? obs_split(g.P) : g.P);
            }
        }
    } else if (io.obs != nullptr) {
        // ---- other plane sizes: plane (p, ch) starts m = (8p + ch)·HW mod 4
        // bytes into a dword.  Channels ch and ch + 4 share m (4·HW is a
        // multiple of 4), so a player's planes fall into four alignment
        // classes k = ch mod 4 with m_k = k·HW mod 4 (m_0 = 0).  Lane j
        // computes quad j's code bytes (code_quad) and army bytes; output
        // dword j of a plane of class k is the last m_k bytes of quad j-1
        // (lane j-1's, by a wave shift, or carried over from the previous
        // round) followed by the first 4-m_k of quad j.  The realignment
        // moves whole bytes and the channels are bits of a byte, so each
        // class realigns the code dword once and masks its two channels out
        // of it.  Dwords that hold bytes of two planes are left to a
        // byte-wise pass after the loop.
        obs_stream_planes(L, g, io.obs, 0, io.nwv > 1 ? obs_split(g.P) : g.P);
        uint32_t *ob = reinterpret_cast<uint32_t *>(io.obs);
        // the dwords across plane boundaries: at most one per plane start
        const int n_planes = g.P * 8;
        for (int i = 1 + lane; i < n_planes; i += kWave) {
            const uint32_t B0 = (uint32_t)(i * g.HW);
            if ((B0 & 3u) == 0) continue;
            const uint32_t b = B0 & ~3u;
            uint32_t v = 0;
#pragma nounroll
            for (int k = 0; k < 4; ++k) v |= obs_byte(L, g, b + k) << (8 * k);
            ob[b >> 2] = v;
        }
    }
    wave_sync();

    // ---- fused random actor for the next step, on the final state
    if (ACT && io.next_actions != nullptr)
        actor_wave(g, L.obm, L.gbm, L.gbm + 16, s.alive, actor_seed, io.use_tick ? s.tick : io.actor_step, env_id,
                   io.next_actions, KIND != K_RESET ? L.gbm + 52 : nullptr);

    // ---- rewards, done, scalars
    if (KIND == K_STEP) {
        if (lane < g.P) io.rewards[lane] = ((win >> lane) & 1u) ? 1 : (((lose >> lane) & 1u) ? -1 : 0);
        if (lane == 0) *io.done = done ? 1 : 0;
    }
    if (KIND != K_OBSERVE && lane == 0) {
        EnvScalars *d = io.sc;
        d->turn = s.turn;
        d->episode = s.episode;
        d->alive = s.alive;
        d->finished = s.finished;
        if (io.use_tick || KIND == K_RESET) d->tick = s.tick;
        if (write_type) {
#pragma unroll
            for (int i = 0; i < kMaxP; ++i) d->gpos[i] = s.gpos[i];
        }
    }
}

// The step kernels for planes of a multiple of 4 cells without the
// scoreboard are limited to the registers of 8 waves per SIMD (the default
// budget of 106 scalar registers allows 7); the extra scalar spills go to
// vector-register lanes and cost less than the lost occupancy (measured).
// The scoreboard kernels would spill vector registers to scratch under that
// limit, and the other plane sizes measured slower at 25x25; they keep the
// default.
// NWV = 2 (steps of FFA boards with unaligned planes): a second wave per env
// writes the observation planes of the players from obs_split(P) on.
template <int KIND, int OBSV, bool SB, bool ACT, int NWV>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu((SB || OBSV != OBS_QUAD) ? 1 : 8, 8))) void k_env(EnvArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int e = (int)xcd_env(blockIdx.x, gridDim.x);
    const Geom g = a.g;
    const size_t cell0 = (size_t)e * g.S;
    EnvIO io;
    io.sc = a.sc + e;
    io.owner = a.owner + cell0;
    io.type = a.type + cell0;
    io.army = a.army + cell0;
    io.actions = a.actions + (size_t)e * g.P;
    io.next_actions = a.next_actions + (size_t)e * g.P;
    io.rewards = a.rewards + (size_t)e * g.P;
    io.done = a.dones + e;
    io.obs = a.obs != nullptr ? a.obs + (size_t)e * (size_t)(g.P * 8 * g.PS) : nullptr;
    io.land = a.land + (size_t)e * g.P;
    io.army_tot = a.army_tot + (size_t)e * g.P;
    io.env_id = a.env_base + (uint64_t)e;
    io.actor_step = a.step_idx;
    io.use_tick = false;
    if (NWV > 1) {
        static_assert(NWV == 1 || OBSV == OBS_STREAM || OBSV == OBS_PADDED,
                      "a second wave only shares the unaligned- and padded-plane writers");
        const int wv = readfirst((int)(threadIdx.x >> 6));
        if (wv > 0) {
            // exactly one barrier, matching the one wave 0 passes after the vision
            const Lds L = carve(smem, g);
            __syncthreads();
            if (io.obs != nullptr) {
                if (OBSV == OBS_STREAM) obs_stream_planes(L, g, io.obs, obs_split(g.P), g.P);
                else obs_padded_planes(L, g, io.obs, obs_split(g.P), g.P);
            }
            return;
        }
        io.nwv = NWV;
    }
    env_body<KIND, OBSV, SB, ACT>(smem, g, a.prm, a.seed, a.actor_seed, io);
}

// ---------------------------------------------------------------- batched pool (mixed shapes)
// One wave per env, `wpg` envs per workgroup, envs taken in the order of a
// work list (slots slot_begin .. slot_end - 1 of it: a launch covers one
// segment of envs that share a packing); each env's shape, mode, generator
// settings and buffer offsets come from its 32-byte descriptor.  With a
// grid smaller than the segment the workgroups loop (persistent form).
// With two waves per env (NWV = 2, one env per workgroup) the second wave
// writes the observation planes of the later players, as in the plain
// two-wave step.
// One pool env on the calling wave (slot = position in the work list;
// wave = the wave's index within the env, of nwv).
template <int KIND, bool ACT>
__device__ __forceinline__ void pool_env_d(const PoolArgs &a, uint8_t *smem, const PoolDesc &d, int nwv = 1,
                                           int wave = 0)
{
    const uint32_t e = d.env;
    Geom g;
    g.H = d.H;
    g.W = d.W;
    g.HW = d.H * d.W;
    g.S = (g.HW + 15) & ~15;
    g.P = d.P;
    g.mode = d.mode;
    g.NW = (g.HW + 63) >> 6;
    g.magic_w = d.magic_w;
    g.magic_hw = d.magic_hw;
    g.PS = pool_plane_stride(g.HW, g.P);
    uint8_t *obs = a.obs != nullptr ? a.obs + (size_t)d.obs_off16 * 16 : nullptr;
    if (wave > 0) {
        // exactly one barrier, matching the one wave 0 passes after the vision
        const Lds L = carve(smem, g);
        __syncthreads();
        if (obs != nullptr) obs_padded_planes(L, g, obs, obs_split(g.P), g.P);
        return;
    }
    GenParamsDev prm = a.prm;
    prm.cmin = d.cmin;
    prm.cmax = d.cmax;
    prm.dmin = d.dmin;
    EnvIO io;
    io.sc = a.sc + e;
    io.owner = a.owner + d.cell_off;
    io.type = a.type + d.cell_off;
    io.army = a.army + d.cell_off;
    io.actions = a.actions + d.act_off;
    io.next_actions = a.actor ? a.actions + d.act_off : nullptr;
    io.rewards = a.rewards + d.act_off;
    io.done = a.dones + e;
    io.obs = obs;
    io.land = nullptr;
    io.army_tot = nullptr;
    io.env_id = a.env_base + e;
    io.actor_step = 0;
    io.use_tick = true;
    io.nwv = nwv;
    env_body<KIND, OBS_PADDED, false, ACT>(smem, g, prm, a.seed, a.actor_seed, io);
}

template <int KIND, bool ACT>
__device__ __forceinline__ void pool_env(const PoolArgs &a, uint8_t *smem, uint32_t slot, int nwv = 1, int wave = 0)
{
    pool_env_d<KIND, ACT>(a, smem, a.desc[slot], nwv, wave);
}

// PERSIST = false: one env per wave (per workgroup with NWV = 2), the grid
// covers the segment.  PERSIST = true (NWV = 1 only: the two waves of an env
// would need a second barrier before reusing the LDS for the next env): a
// smaller grid whose waves stride over the segment.
template <int KIND, bool ACT, bool PERSIST, int NWV>
__global__ __launch_bounds__(256) void k_pool(PoolArgs a)
{
    static_assert(NWV == 1 || !PERSIST, "two waves per env only in the one-shot grid");
    extern __shared__ __align__(16) uint8_t smem[];
    // wave index as a scalar: everything derived from the env id stays wave-uniform
    const uint32_t wave = (uint32_t)readfirst((int)(threadIdx.x >> 6));
    if (NWV == 2) {
        const uint32_t slot = a.slot_begin + blockIdx.x;
        if (slot < a.slot_end) pool_env<KIND, ACT>(a, smem, slot, 2, (int)wave);
        return;
    }
    uint8_t *mine = smem + wave * a.lds_per_wave;
    if (PERSIST) {
        for (uint32_t slot = a.slot_begin + blockIdx.x * a.wpg + wave; slot < a.slot_end; slot += gridDim.x * a.wpg)
            pool_env<KIND, ACT>(a, mine, slot);
    } else {
        const uint32_t slot = a.slot_begin + xcd_chunk32(blockIdx.x, gridDim.x) * a.wpg + wave;
        if (slot < a.slot_end) pool_env<KIND, ACT>(a, mine, slot);
    }
}

// ---------------------------------------------------------------- standalone actor
__global__ __launch_bounds__(64) void k_sample(SampleArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = lane_id();
    const int e = blockIdx.x;
    const Geom g = a.g;
    const Lds L = carve(smem, g);
    const uint64_t env_id = a.env_base + (uint64_t)e;
    const size_t cell0 = (size_t)e * g.S;
    const uint32_t alive = a.sc[e].alive;
    // owner and type rows into LDS; army only as the "more than one unit" bit
    const int n16 = g.S >> 4;
    for (int i = lane; i < n16; i += kWave) {
        reinterpret_cast<uint4 *>(L.owner)[i] = reinterpret_cast<const uint4 *>(a.owner + cell0)[i];
        reinterpret_cast<uint4 *>(L.type)[i] = reinterpret_cast<const uint4 *>(a.type + cell0)[i];
    }
    wave_sync();
    for (int w = 0; w < g.NW; ++w) {
        const int c = w * 64 + lane;
        const bool real = c < g.HW;
        const int o = real ? (int)L.owner[c] : -1;
        const bool many = real && a.army[cell0 + c] > 1;
        for (int p = 0; p < g.P; ++p) {
            const uint64_t m = ballot(o == readfirst(p));
            if (lane == 0) L.obm[p * 16 + w] = m;
        }
        const uint64_t pm = ballot(real && L.type[c] != MOUNTAIN);
        const uint64_t bm = ballot(many);
        if (lane == 0) { L.gbm[w] = pm; L.gbm[16 + w] = bm; }
    }
    wave_sync();
    actor_wave(g, L.obm, L.gbm, L.gbm + 16, alive, a.actor_seed, a.step_idx, env_id, a.actions + (size_t)e * g.P);
}

// ---------------------------------------------------------------- launchers
uint32_t lds_bytes(const Geom &g) { return lds_bytes_for(g.S, g.P); }

int obs_variant(int HW, int P)
{
    (void)P;
    return HW % 4 == 0 ? OBS_QUAD : OBS_STREAM;
}

static int obs_variant(const Geom &g) { return obs_variant(g.HW, g.P); }

template <int KIND, bool SB, bool ACT>
static hipError_t launch_kind(const EnvArgs &a, int n_envs, hipStream_t stream)
{
    const dim3 grid((unsigned)n_envs), block(kWave);
    const uint32_t lds = lds_bytes(a.g);
    if (a.g.PS != a.g.HW) {
        // planes padded to 32 bytes: the dword writer for every shape; more
        // than 4 players share it between two waves, as the unaligned writer
        if constexpr (KIND == K_STEP) {
            if (a.g.P > 4 && a.obs != nullptr && n_envs <= 16384) {
                hipLaunchKernelGGL((k_env<KIND, OBS_PADDED, SB, ACT, 2>), grid, dim3(2 * kWave), lds, stream, a);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_env<KIND, OBS_PADDED, SB, ACT, 1>), grid, block, lds, stream, a);
        return hipGetLastError();
    }
    switch (obs_variant(a.g)) {
    case OBS_QUAD: hipLaunchKernelGGL((k_env<KIND, OBS_QUAD, SB, ACT, 1>), grid, block, lds, stream, a); break;
    default:
        // steps of boards with more than 4 players and unaligned planes: the
        // observation (most of the work) is shared by two waves per env when
        // the batch leaves room for the second wave (measured: FFA-8 25x25
        // with 16,384 envs 249 -> 226 us; 17x19 with 32,768 envs a little
        // slower, so larger batches keep one wave)
        if constexpr (KIND == K_STEP) {
            if (a.g.P > 4 && a.obs != nullptr && n_envs <= 16384) {
                hipLaunchKernelGGL((k_env<KIND, OBS_STREAM, SB, ACT, 2>), grid, dim3(2 * kWave), lds, stream, a);
                break;
            }
        }
        hipLaunchKernelGGL((k_env<KIND, OBS_STREAM, SB, ACT, 1>), grid, block, lds, stream, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_step(const EnvArgs &a, int n_envs, hipStream_t stream)
{
    if (a.next_actions != nullptr)
        return (a.land != nullptr) ? launch_kind<K_STEP, true, true>(a, n_envs, stream)
                                   : launch_kind<K_STEP, false, true>(a, n_envs, stream);
    return (a.land != nullptr) ? launch_kind<K_STEP, true, false>(a, n_envs, stream)
                               : launch_kind<K_STEP, false, false>(a, n_envs, stream);
}

hipError_t launch_reset(const EnvArgs &a, int n_envs, hipStream_t stream)
{
    return launch_kind<K_RESET, false, false>(a, n_envs, stream);
}

hipError_t launch_observe(const EnvArgs &a, int n_envs, hipStream_t stream)
{
    return launch_kind<K_OBSERVE, false, false>(a, n_envs, stream);
}

// ---------------------------------------------------------------- served batches
// One launch steps the envs of many requests (each request = one step of a
// group, a pool of its own), one workgroup per env of the launch; a
// workgroup finds its request by a binary search over the requests' first
// workgroups (at most 9 scalar loads from the argument segment), so no
// workgroup is launched for nothing when request sizes differ.
// Buffers are addressed as arena + offset so that every pointer derives from
// a kernel argument (global address space, scalar base + vector offset).
// The request list travels in the kernel argument (scalar loads from the
// argument segment), the group records stay resident in the arena.
// UNI: every request of the launch is a uniform group (its record says so),
// whose descriptors the kernel derives instead of loading; a launch with any
// other group loads every descriptor (one copy of the step per kernel: with
// both forms in one kernel the served mix ran 5-13% slower).
// The uniform instance budgets registers for 8 waves per SIMD (uniform 24x24
// 1v1 groups fit 8 in LDS); the other keeps the default budget, since the
// LDS of its largest board limits it to fewer waves anyway (served mix
// 401.5 -> 410 M frames/s without the 8-wave budget's spills).
template <bool UNI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(UNI ? 8 : 1, 8))) void k_serve(ServeLaunch la)
{
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t *const arena = la.arena;
    // the request holding this workgroup: binary search over the ascending
    // first[] (wave-uniform, scalar loads), first[lo] <= b < first[hi]
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = la.n_req;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (la.first[mid] <= b) lo = mid;
        else hi = mid;
    }
    const ServeReq &r = la.groups[la.idx[lo]];
    const uint32_t slot = b - la.first[lo];
    if (slot >= r.n_envs) return;
    PoolArgs a;
    a.prm = r.prm;
    a.seed = r.seed;
    a.env_base = r.env_base;
    a.actor_seed = r.actor_seed;
    a.n_envs = r.n_envs;
    a.slot_begin = 0;
    a.slot_end = r.n_envs;
    a.wpg = 1;
    a.lds_per_wave = 0;
    a.actor = r.actor;
    a.desc = reinterpret_cast<const PoolDesc *>(arena + r.off_desc);
    a.sc = reinterpret_cast<EnvScalars *>(arena + r.off_sc);
    a.owner = reinterpret_cast<int8_t *>(arena + r.off_owner);
    a.type = arena + r.off_type;
    a.army = reinterpret_cast<int32_t *>(arena + r.off_army);
    a.actions = reinterpret_cast<int32_t *>(arena + r.off_actions);
    a.rewards = reinterpret_cast<int32_t *>(arena + r.off_rewards);
    a.dones = arena + r.off_dones;
    a.obs = r.off_obs != ~0ull ? arena + r.off_obs : nullptr;
    if (UNI) {
        // every env of a uniform group has the template's shape and
        // settings: its descriptor follows from the slot
        PoolDesc d = r.tmpl;
        d.cell_off = slot * r.cells_per_env;
        d.obs_off16 = slot * r.obs16_per_env;
        d.act_off = slot * d.P;
        d.env = slot;
        pool_env_d<K_STEP, true>(a, smem, d);
    } else {
        pool_env<K_STEP, true>(a, smem, slot);
    }
}

hipError_t launch_serve(const ServeLaunch &la, uint32_t total_envs, uint32_t lds, bool all_uniform, hipStream_t stream)
{
    if (la.n_req == 0 || la.n_req > kServeMaxReqs || total_envs == 0) return hipErrorInvalidValue;
    if (all_uniform) hipLaunchKernelGGL(k_serve<true>, dim3(total_envs), dim3(kWave), lds, stream, la);
    else hipLaunchKernelGGL(k_serve<false>, dim3(total_envs), dim3(kWave), lds, stream, la);
    return hipGetLastError();
}

template <int KIND, bool ACT, bool PERSIST, int NWV>
static hipError_t launch_pool_kind(const PoolArgs &a, uint32_t grid, hipStream_t stream)
{
    const uint32_t threads = NWV == 2 ? 2 * kWave : kWave * a.wpg;
    const uint32_t lds = NWV == 2 ? a.lds_per_wave : a.lds_per_wave * a.wpg;
    hipLaunchKernelGGL((k_pool<KIND, ACT, PERSIST, NWV>), dim3(grid), dim3(threads), lds, stream, a);
    return hipGetLastError();
}

template <int KIND, bool ACT>
static hipError_t launch_pool_act(const PoolArgs &a, uint32_t grid, uint32_t nwv, hipStream_t stream)
{
    const uint32_t n = a.slot_end - a.slot_begin;
    if (nwv == 2) return launch_pool_kind<KIND, ACT, false, 2>(a, n, stream);
    const uint32_t full = (n + a.wpg - 1) / a.wpg;
    if (grid == 0 || grid >= full) return launch_pool_kind<KIND, ACT, false, 1>(a, full, stream);
    return launch_pool_kind<KIND, ACT, true, 1>(a, grid, stream);
}

// One segment of the work list [a.slot_begin, a.slot_end): grid == 0 one
// wave (nwv waves) per env, else persistent (nwv == 1 only).
hipError_t launch_pool(const PoolArgs &a, int kind, bool act, uint32_t grid, uint32_t nwv, hipStream_t stream)
{
    if (a.slot_end <= a.slot_begin) return hipSuccess;
    if (kind == K_RESET)
        return act ? launch_pool_act<K_RESET, true>(a, grid, 1, stream) : launch_pool_act<K_RESET, false>(a, grid, 1, stream);
    return act ? launch_pool_act<K_STEP, true>(a, grid, nwv, stream) : launch_pool_act<K_STEP, false>(a, grid, nwv, stream);
}

hipError_t launch_sample(const SampleArgs &a, int n_envs, hipStream_t stream)
{
    hipLaunchKernelGGL(k_sample, dim3((unsigned)n_envs), dim3(kWave), lds_bytes(a.g), stream, a);
    return hipGetLastError();
}

}  // namespace gen
