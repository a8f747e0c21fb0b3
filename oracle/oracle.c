/*
 * oracle.c -- plain, slow, single-threaded CPU reference simulator of the
 * Generals.io environment step (arxiv 2606.23348, Section IV "Game
 * Description", subsections IV-A..IV-E, and Appendix A for the observation).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg use it.  It shares no code, header, table or constant
 * generator with the HIP library; the two meet only through the public
 * host-state format (plain arrays) and the seeds.
 *
 * The paper leaves many details open.  Every such gap is filled by a numbered
 * reading (R1..R18) that the HIP path follows too; the readings are listed,
 * with the passage each one rests on, in the design notes at the repository
 * root.  Parts of this file that no external fact pins carry the marker
 * "parity unpinned" below: the move order (R5), the per-cell halving on
 * capture (R9), team vision (R10), reward timing in FFA/2v2 (R11), the
 * auto-reset convention (R13), the map generator's draw order (R14) and the
 * army bucket of the observation (R16).
 *
 * Style: straight loops over row-major cells, one environment at a time, no
 * bit tricks, no precomputed tables.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ---- cell types (Section IV-A: plain, mountain, general, castle) ---- */
enum { T_PLAIN = 0, T_MOUNTAIN = 1, T_CASTLE = 2, T_GENERAL = 3 };
/* ---- game modes (Section IV-E) ---- */
enum { M_1V1 = 0, M_2V2 = 1, M_FFA = 2 };
/* ---- Philox key domains (second key word) ---- */
enum { D_MAPGEN = 1, D_ACTIONS = 2, D_PREGROW = 3, D_POOLSPEC = 4, D_ARRIVALS = 5 };

#define ORC_MAX_CELLS 1024
#define ORC_MAX_P 8

/* Configuration of one batch of environments (all the same shape and mode). */
typedef struct orc_cfg {
    int32_t H, W, mode, P;
    uint32_t mountain_thresh;      /* cell is a mountain iff draw < thresh */
    int32_t cities_min, cities_max;
    int32_t city_army_min, city_army_max;
    int32_t min_general_dist;      /* Manhattan */
    int32_t auto_reset;            /* R13 */
    int32_t pregrow;               /* pre-grown generals on env%4==0, episode 0 */
    uint64_t seed;                 /* map seed */
    uint64_t env_base;             /* global id of env 0 of the batch */
    int32_t generator;             /* 0: synthetic generator (R14); 1: official rules (R18) */
    int32_t max_general_dist;      /* R18: cap on the BFS spawn distance (0 = none; curriculum) */
    int32_t castle_radius;         /* R18: a castle within this BFS distance of every general */
    int32_t pad;
    const uint64_t *env_ids;       /* NULL: env e of a batch has global id env_base + e;
                                      else env_ids[e] (envs of one shape scattered over a pool) */
} orc_cfg;

/* Public host-state format: env-major plain arrays. */
typedef struct orc_batch {
    int8_t   *owner;     /* [E][H*W], -1 neutral */
    int32_t  *army;      /* [E][H*W] */
    uint8_t  *type;      /* [E][H*W] */
    int32_t  *turn;      /* [E] */
    uint32_t *episode;   /* [E] */
    uint8_t  *alive;     /* [E] bit p = player p alive */
    uint8_t  *finished;  /* [E] terminal and frozen (auto-reset off) */
    int16_t  *gpos;      /* [E][P] cell of each player's general */
} orc_batch;

/* One environment, unpacked. */
typedef struct orc_env {
    int H, W, P, mode;
    int8_t owner[ORC_MAX_CELLS];
    int32_t army[ORC_MAX_CELLS];
    uint8_t type[ORC_MAX_CELLS];
    int32_t turn;
    uint32_t episode;
    uint8_t alive;
    uint8_t finished;
    int16_t gpos[ORC_MAX_P];
} orc_env;

/* ======================================================================
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies words 0 and 2
 * by the two round multipliers, swaps the products' halves into place and
 * mixes in the key; the key is bumped by the two Weyl constants between
 * rounds.
 * ==================================================================== */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;  /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;  /* sqrt(3) - 1 */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Draw number j (a 32-bit word) of the stream keyed (seed, domain) with
 * counter prefix (c0, c1, c2): block j/8 is counter word 3; inside a block
 * the 64-bit word is (j/2)%4 and the low half comes first (R14). */
uint32_t orc_draw(uint64_t seed, uint64_t domain, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t j)
{
    uint64_t ctr[4] = { c0, c1, c2, j / 8 };
    uint64_t key[2] = { seed, domain };
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t w = out[(j / 2) % 4];
    return (j % 2 == 0) ? (uint32_t)(w & 0xFFFFFFFFu) : (uint32_t)(w >> 32);
}

/* ======================================================================
 * Philox4x32-10 (same paper as above): the 32-bit member of the family.
 * Four 32-bit counter words and two key words; each round multiplies words
 * 0 and 2 by the round multipliers, swaps the products' halves into place
 * and mixes in the key; the key is bumped by the two 32-bit Weyl constants
 * between rounds.
 * ==================================================================== */
static const uint32_t PHILOX32_M0 = 0xD2511F53u;
static const uint32_t PHILOX32_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX32_W0 = 0x9E3779B9u;  /* golden ratio */
static const uint32_t PHILOX32_W1 = 0xBB67AE85u;  /* sqrt(3) - 1 */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += PHILOX32_W0; k1 += PHILOX32_W1; }
        uint64_t p0 = (uint64_t)PHILOX32_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX32_M1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The random actor's draw for player p of env `env_id` at actor step `step`
 * (R15): word p mod 4 of Philox4x32-10 keyed by the two halves of the actor
 * seed, counter (step low, step high, env low, env high), with the top bit
 * of the last word flipped for players 4..7 (env ids stay below 2^63). */
uint32_t orc_actor_draw(uint64_t seed_act, uint64_t env_id, uint64_t step, int p)
{
    uint32_t ctr[4] = { (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)env_id,
                        (uint32_t)(env_id >> 32) ^ (p >= 4 ? 0x80000000u : 0u) };
    uint32_t key[2] = { (uint32_t)seed_act, (uint32_t)(seed_act >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[p % 4];
}

/* Uniform pick in [0, n) from a 32-bit draw: floor(r * n / 2^32). */
static uint32_t pick(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }

static int iabs(int x) { return x < 0 ? -x : x; }

/* Saturating addition at INT32_MAX (R12: army never wraps). */
static int32_t sat_add(int32_t a, int32_t b)
{
    int64_t s = (int64_t)a + (int64_t)b;
    if (s > INT32_MAX) return INT32_MAX;
    return (int32_t)s;
}

/* Allies exist only in 2v2, where team(i) = i mod 2 (Section IV-E). */
static int is_ally(const orc_env *s, int a, int b)
{
    return s->mode == M_2V2 && a != b && (a % 2) == (b % 2);
}

static int in_team(const orc_env *s, int owner, int p)
{
    return owner == p || (owner >= 0 && is_ally(s, owner, p));
}

/* BFS distance from src over non-mountain cells, 4-connected (-1: not
 * reachable). */
static void bfs_dist(const orc_env *s, int src, int *dist)
{
    const int H = s->H, W = s->W, HW = H * W;
    int queue[ORC_MAX_CELLS];
    for (int c = 0; c < HW; c++) dist[c] = -1;
    int qh = 0, qt = 0;
    dist[src] = 0;
    queue[qt++] = src;
    while (qh < qt) {
        int c = queue[qh++];
        int r = c / W, col = c % W;
        int nb[4][2] = { { r - 1, col }, { r + 1, col }, { r, col - 1 }, { r, col + 1 } };
        for (int k = 0; k < 4; k++) {
            int nr = nb[k][0], nc = nb[k][1];
            if (nr < 0 || nr >= H || nc < 0 || nc >= W) continue;
            int d = nr * W + nc;
            if (s->type[d] == T_MOUNTAIN || dist[d] >= 0) continue;
            dist[d] = dist[c] + 1;
            queue[qt++] = d;
        }
    }
}

/* ======================================================================
 * The official generator (Section IV-A: 20% mountains, 9..11 neutral castles
 * of 40..50 units, generals at least 17 steps apart, a neutral castle within
 * radius 6 of every general) with the spawn-distance cap of the curriculum
 * (Section V-C); reading R18.  Same stream and attempt structure as the
 * synthetic generator: G1 and G2 unchanged; every distance is a BFS over
 * non-mountain cells; each further general is a pick over the cells whose
 * distance to every earlier general lies in [min, max]; after the castle
 * count, every general in order that has no castle within the radius gets
 * one picked among the plain cells within it, then the remaining castles go
 * anywhere.  Returns 1 on success (state filled), 0 if this attempt fails.
 * parity unpinned: the draw order is a reading.
 * ==================================================================== */
static int mapgen_official_attempt(orc_env *s, const orc_cfg *cfg, uint64_t env_id, uint32_t episode, int attempt)
{
    const int H = cfg->H, W = cfg->W, HW = H * W, P = cfg->P;
    int list[ORC_MAX_CELLS];
    int dist[ORC_MAX_P][ORC_MAX_CELLS];
    int g[ORC_MAX_P];
    const uint32_t T = attempt < 64 ? cfg->mountain_thresh : 0u;
    uint64_t j = 0;
    for (int c = 0; c < HW; c++) {
        uint32_t r = orc_draw(cfg->seed, D_MAPGEN, env_id, episode, (uint64_t)attempt, j++);
        s->type[c] = (r < T) ? T_MOUNTAIN : T_PLAIN;
        s->owner[c] = -1;
        s->army[c] = 0;
    }
    int n = 0;
    for (int c = 0; c < HW; c++)
        if (s->type[c] != T_MOUNTAIN) list[n++] = c;
    if (n == 0) return 0;
    g[0] = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
    bfs_dist(s, g[0], dist[0]);
    for (int i = 1; i < P; i++) {
        n = 0;
        for (int c = 0; c < HW; c++) {
            int good = 1;
            for (int k = 0; k < i; k++) {
                const int d = dist[k][c];
                if (d < 0 || d < cfg->min_general_dist || c == g[k] ||
                    (cfg->max_general_dist > 0 && d > cfg->max_general_dist)) { good = 0; break; }
            }
            if (good) list[n++] = c;
        }
        if (n == 0) return 0;
        g[i] = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
        bfs_dist(s, g[i], dist[i]);
    }
    for (int i = 0; i < P; i++) s->type[g[i]] = T_GENERAL;
    int ncastles = cfg->cities_min + (int)pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++),
                                               (uint32_t)(cfg->cities_max - cfg->cities_min + 1));
    int placed = 0;
    for (int i = 0; i < P; i++) {
        int near = 0;
        for (int c = 0; c < HW; c++)
            if (s->type[c] == T_CASTLE && dist[i][c] >= 0 && dist[i][c] <= cfg->castle_radius) near = 1;
        if (near) continue;
        n = 0;
        for (int c = 0; c < HW; c++)
            if (s->type[c] == T_PLAIN && dist[i][c] >= 1 && dist[i][c] <= cfg->castle_radius) list[n++] = c;
        if (n == 0) return 0;
        int c = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
        s->type[c] = T_CASTLE;
        s->army[c] = cfg->city_army_min + (int32_t)pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++),
                                                         (uint32_t)(cfg->city_army_max - cfg->city_army_min + 1));
        placed++;
    }
    for (int t = placed; t < ncastles; t++) {
        n = 0;
        for (int c = 0; c < HW; c++)
            if (s->type[c] == T_PLAIN) list[n++] = c;
        if (n == 0) break;
        int c = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
        s->type[c] = T_CASTLE;
        s->army[c] = cfg->city_army_min + (int32_t)pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++),
                                                         (uint32_t)(cfg->city_army_max - cfg->city_army_min + 1));
    }
    for (int i = 0; i < P; i++) {
        s->owner[g[i]] = (int8_t)i;
        s->army[g[i]] = 1;
        s->gpos[i] = (int16_t)g[i];
    }
    return 1;
}

/* ======================================================================
 * Map generation (Section IV-A, with the generator parameters of the
 * synthetic workloads; reading R14).  Returns the attempt that succeeded
 * (0..127) or 128 for the deterministic last resort.
 * parity unpinned: the draw order below is a reading, not printed anywhere.
 * ==================================================================== */
static int mapgen(orc_env *s, const orc_cfg *cfg, uint64_t env_id, uint32_t episode)
{
    const int H = cfg->H, W = cfg->W, HW = H * W, P = cfg->P;
    int list[ORC_MAX_CELLS];
    int comp[ORC_MAX_CELLS];
    int queue[ORC_MAX_CELLS];
    int g[ORC_MAX_P];

    s->H = H; s->W = W; s->P = P; s->mode = cfg->mode;
    for (int attempt = 0; attempt < 128; attempt++) {
        if (cfg->generator == 1) {
            if (!mapgen_official_attempt(s, cfg, env_id, episode, attempt)) continue;
            s->turn = 0;
            s->episode = episode;
            s->alive = (uint8_t)((1u << P) - 1u);
            s->finished = 0;
            return attempt;
        }
        uint32_t T = attempt < 64 ? cfg->mountain_thresh : 0u;
        uint64_t j = 0;
        /* G1: mountains, one draw per cell in row-major order */
        for (int c = 0; c < HW; c++) {
            uint32_t r = orc_draw(cfg->seed, D_MAPGEN, env_id, episode, (uint64_t)attempt, j++);
            s->type[c] = (r < T) ? T_MOUNTAIN : T_PLAIN;
            s->owner[c] = -1;
            s->army[c] = 0;
        }
        /* G2: first general uniform over non-mountain cells */
        int n = 0;
        for (int c = 0; c < HW; c++)
            if (s->type[c] != T_MOUNTAIN) list[n++] = c;
        if (n == 0) continue;
        g[0] = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
        /* G3: 4-connected component of g[0] over non-mountain cells (BFS) */
        for (int c = 0; c < HW; c++) comp[c] = 0;
        int qh = 0, qt = 0;
        comp[g[0]] = 1; queue[qt++] = g[0];
        while (qh < qt) {
            int c = queue[qh++];
            int r = c / W, col = c % W;
            int nb[4][2] = { { r - 1, col }, { r + 1, col }, { r, col - 1 }, { r, col + 1 } };
            for (int k = 0; k < 4; k++) {
                int nr = nb[k][0], nc = nb[k][1];
                if (nr < 0 || nr >= H || nc < 0 || nc >= W) continue;
                int d = nr * W + nc;
                if (s->type[d] == T_MOUNTAIN || comp[d]) continue;
                comp[d] = 1; queue[qt++] = d;
            }
        }
        /* G4: other generals in the component, Manhattan >= d_min from all earlier ones */
        int ok = 1;
        for (int i = 1; i < P && ok; i++) {
            n = 0;
            for (int c = 0; c < HW; c++) {
                if (!comp[c]) continue;
                int good = 1;
                for (int k = 0; k < i; k++) {
                    int dist = iabs(c / W - g[k] / W) + iabs(c % W - g[k] % W);
                    if (c == g[k] || dist < cfg->min_general_dist) { good = 0; break; }
                }
                if (good) list[n++] = c;
            }
            if (n == 0) { ok = 0; break; }
            g[i] = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
        }
        if (!ok) continue;
        /* G5: neutral cities anywhere on free plain cells, army uniform in range */
        int ncities = cfg->cities_min + (int)pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++),
                                                  (uint32_t)(cfg->cities_max - cfg->cities_min + 1));
        for (int t = 0; t < ncities; t++) {
            n = 0;
            for (int c = 0; c < HW; c++) {
                if (s->type[c] != T_PLAIN) continue;
                int is_gen = 0;
                for (int k = 0; k < P; k++) if (g[k] == c) is_gen = 1;
                if (!is_gen) list[n++] = c;
            }
            if (n == 0) break;
            int c = list[pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++), (uint32_t)n)];
            s->type[c] = T_CASTLE;
            s->army[c] = cfg->city_army_min +
                (int32_t)pick(orc_draw(cfg->seed, D_MAPGEN, env_id, episode, attempt, j++),
                              (uint32_t)(cfg->city_army_max - cfg->city_army_min + 1));
        }
        /* G6: generals */
        for (int i = 0; i < P; i++) {
            s->owner[g[i]] = (int8_t)i;
            s->army[g[i]] = 1;
            s->type[g[i]] = T_GENERAL;
            s->gpos[i] = (int16_t)g[i];
        }
        s->turn = 0;
        s->episode = episode;
        s->alive = (uint8_t)((1u << P) - 1u);
        s->finished = 0;
        return attempt;
    }
    /* deterministic last resort: no mountains, no cities, generals on fixed cells */
    const int fr[8] = { 0, H - 1, 0, H - 1, 0, H - 1, H / 2, H / 2 };
    const int fc[8] = { 0, W - 1, W - 1, 0, W / 2, W / 2, 0, W - 1 };
    for (int c = 0; c < HW; c++) { s->type[c] = T_PLAIN; s->owner[c] = -1; s->army[c] = 0; }
    for (int i = 0; i < P; i++) {
        int c = fr[i] * W + fc[i];
        s->owner[c] = (int8_t)i; s->army[c] = 1; s->type[c] = T_GENERAL; s->gpos[i] = (int16_t)c;
    }
    s->turn = 0; s->episode = episode; s->alive = (uint8_t)((1u << P) - 1u); s->finished = 0;
    return 128;
}

/* Pre-grown generals for the overflow-stress workload: at episode 0 only, on
 * envs whose global id is a multiple of 4, general i gets 100000 + U{0..900000}
 * from draw i of the (seed, PREGROW) stream with counter prefix (env, 0, 0). */
static void pregrow(orc_env *s, const orc_cfg *cfg, uint64_t env_id)
{
    if (!cfg->pregrow || s->episode != 0 || env_id % 4 != 0) return;
    for (int i = 0; i < s->P; i++) {
        uint32_t r = orc_draw(cfg->seed, D_PREGROW, env_id, 0, 0, (uint64_t)i);
        s->army[s->gpos[i]] = 100000 + (int32_t)pick(r, 900001u);
    }
}

/* ======================================================================
 * Moves and combat (Section IV-D; team rule Section IV-E).
 * ==================================================================== */
static void capture(orc_env *s, int captor, int victim)
{
    /* Section IV-E: all of the victim's cells go to the captor with half of
     * their army (R9: floor per cell); the general becomes a castle. */
    int HW = s->H * s->W;
    for (int c = 0; c < HW; c++) {
        if (s->owner[c] == victim) {
            s->owner[c] = (int8_t)captor;
            s->army[c] = s->army[c] / 2;
        }
    }
    s->type[s->gpos[victim]] = T_CASTLE;
    s->alive = (uint8_t)(s->alive & ~(1u << victim));
}

/* Apply one player's action (encoding cell*9+k; k=0 pass, 1..4 all-but-one
 * toward up/down/left/right, 5..8 half toward the same).  Illegal actions are
 * passes (R4). */
static void apply_move(orc_env *s, int i, int32_t a)
{
    const int H = s->H, W = s->W, HW = H * W;
    if (!((s->alive >> i) & 1)) return;
    if (a < 0 || a >= HW * 9) return;
    int src = a / 9, k = a % 9;
    if (k == 0) return;
    int dir = (k - 1) % 4, half = (k >= 5);
    int r = src / W, c = src % W;
    if (dir == 0) r -= 1;
    else if (dir == 1) r += 1;
    else if (dir == 2) c -= 1;
    else c += 1;
    if (r < 0 || r >= H || c < 0 || c >= W) return;
    int dst = r * W + c;
    if (s->type[dst] == T_MOUNTAIN) return;
    if (s->owner[src] != i) return;
    int32_t have = s->army[src];
    if (have <= 1) return;
    int32_t m = half ? have / 2 : have - 1;
    s->army[src] = have - m;

    int o = s->owner[dst];
    int32_t d = s->army[dst];
    if (o == i) {
        s->army[dst] = sat_add(d, m);                  /* own cell: merge */
    } else if (o >= 0 && is_ally(s, o, i)) {
        s->army[dst] = sat_add(d, m);                  /* ally: pool and take */
        s->owner[dst] = (int8_t)i;
    } else if (m > d) {                                /* combat won */
        s->owner[dst] = (int8_t)i;
        s->army[dst] = m - d;
        if (s->type[dst] == T_GENERAL) {
            for (int v = 0; v < s->P; v++) {
                if (s->gpos[v] == dst && ((s->alive >> v) & 1) && v != i && !is_ally(s, v, i)) {
                    capture(s, i, v);
                    break;
                }
            }
        }
    } else {
        s->army[dst] = d - m;                          /* lost or tied: owner kept */
    }
}

/* Army growth (Section IV-C, readings R1-R2), applied after turn += 1. */
static void growth(orc_env *s)
{
    int HW = s->H * s->W;
    int every2 = (s->turn % 2 == 0), every50 = (s->turn % 50 == 0);
    for (int c = 0; c < HW; c++) {
        if (s->owner[c] < 0) continue;
        if (every2 && (s->type[c] == T_GENERAL || s->type[c] == T_CASTLE))
            s->army[c] = sat_add(s->army[c], 1);
        if (every50 && s->type[c] == T_PLAIN)
            s->army[c] = sat_add(s->army[c], 1);
    }
}

static int popcount8(unsigned x)
{
    int n = 0;
    for (int b = 0; b < 8; b++) n += (x >> b) & 1;
    return n;
}

/* One environment step.  Moves in rotating priority (R5, parity unpinned),
 * growth, terminal rewards (R11, parity unpinned), auto-reset (R13). */
static void step_env(orc_env *s, const orc_cfg *cfg, uint64_t env_id, const int32_t *actions,
                     int32_t *rewards, uint8_t *done)
{
    const int P = s->P;
    for (int p = 0; p < P; p++) rewards[p] = 0;
    *done = 0;
    if (s->finished) { *done = 1; return; }

    uint8_t alive_before = s->alive;
    for (int j = 0; j < P; j++) {
        int i = (s->turn + j) % P;
        apply_move(s, i, actions[i]);
    }
    s->turn += 1;
    growth(s);

    uint8_t lost = (uint8_t)(alive_before & ~s->alive);
    int over = 0;
    if (s->mode == M_2V2) {
        int team0 = 0, team1 = 0;
        for (int p = 0; p < P; p++) {
            if ((s->alive >> p) & 1) { if (p % 2 == 0) team0++; else team1++; }
        }
        if (team0 == 0 || team1 == 0) {
            over = 1;
            int winner = team0 == 0 ? 1 : 0;
            for (int p = 0; p < P; p++) rewards[p] = (p % 2 == winner) ? 1 : -1;
        }
    } else {
        for (int p = 0; p < P; p++) if ((lost >> p) & 1) rewards[p] = -1;
        if (popcount8(s->alive) == 1) {
            over = 1;
            for (int p = 0; p < P; p++) if ((s->alive >> p) & 1) rewards[p] = 1;
        }
    }
    if (over) {
        *done = 1;
        if (cfg->auto_reset) {
            mapgen(s, cfg, env_id, s->episode + 1);
        } else {
            s->finished = 1;
        }
    }
}

/* Observation of player p (8 channels, reading R16; vision Section IV-B). */
static void observe_env(const orc_env *s, uint8_t *obs /* [P][8][H*W] */)
{
    const int H = s->H, W = s->W, HW = H * W, P = s->P;
    for (int p = 0; p < P; p++) {
        uint8_t *o = obs + (size_t)p * 8 * HW;
        for (int r = 0; r < H; r++) {
            for (int c = 0; c < W; c++) {
                int cell = r * W + c;
                int vis = 0;
                for (int dr = -1; dr <= 1; dr++) {
                    for (int dc = -1; dc <= 1; dc++) {
                        int nr = r + dr, nc = c + dc;
                        if (nr < 0 || nr >= H || nc < 0 || nc >= W) continue;
                        if (in_team(s, s->owner[nr * W + nc], p)) vis = 1;
                    }
                }
                int own = s->owner[cell], t = s->type[cell];
                o[0 * HW + cell] = (own == p);
                o[1 * HW + cell] = vis && own >= 0 && !in_team(s, own, p);
                o[2 * HW + cell] = vis && own == -1 && t != T_MOUNTAIN;
                o[3 * HW + cell] = vis && t == T_MOUNTAIN;
                o[4 * HW + cell] = vis && t == T_CASTLE;
                o[5 * HW + cell] = vis && t == T_GENERAL;
                o[6 * HW + cell] = !vis;
                o[7 * HW + cell] = vis ? (uint8_t)(s->army[cell] > 255 ? 255 : s->army[cell]) : 0;
            }
        }
    }
}

/* Legality of (cell, k) for player p (R4), used by the random actor. */
static int legal(const orc_env *s, int p, int cell, int k)
{
    const int H = s->H, W = s->W;
    if (!((s->alive >> p) & 1)) return 0;
    if (s->owner[cell] != p || s->army[cell] <= 1) return 0;
    int dir = (k - 1) % 4;
    int r = cell / W, c = cell % W;
    if (dir == 0) r -= 1;
    else if (dir == 1) r += 1;
    else if (dir == 2) c -= 1;
    else c += 1;
    if (r < 0 || r >= H || c < 0 || c >= W) return 0;
    return s->type[r * W + c] != T_MOUNTAIN;
}

/* Random legal actor (R15): uniform over {pass} + legal (cell, k) listed by
 * cell in row-major order and then k = 1..8.  Player p uses its actor draw
 * (orc_actor_draw): one Philox4x32 block serves four players. */
static void sample_env(const orc_env *s, uint64_t seed_act, uint64_t step_idx, uint64_t env_id, int32_t *actions)
{
    int32_t L[ORC_MAX_CELLS * 8 + 1];
    const int HW = s->H * s->W;
    for (int p = 0; p < s->P; p++) {
        int n = 0;
        L[n++] = 0;
        for (int cell = 0; cell < HW; cell++)
            for (int k = 1; k <= 8; k++)
                if (legal(s, p, cell, k)) L[n++] = cell * 9 + k;
        uint32_t r = orc_actor_draw(seed_act, env_id, step_idx, p);
        actions[p] = ((s->alive >> p) & 1) ? L[pick(r, (uint32_t)n)] : 0;
    }
}

/* ---------------- conversion to and from the public host format ---------------- */
static void load_env(orc_env *s, const orc_cfg *cfg, const orc_batch *b, int e)
{
    const int HW = cfg->H * cfg->W, P = cfg->P;
    s->H = cfg->H; s->W = cfg->W; s->P = P; s->mode = cfg->mode;
    memcpy(s->owner, b->owner + (size_t)e * HW, (size_t)HW);
    memcpy(s->army, b->army + (size_t)e * HW, (size_t)HW * 4);
    memcpy(s->type, b->type + (size_t)e * HW, (size_t)HW);
    s->turn = b->turn[e];
    s->episode = b->episode[e];
    s->alive = b->alive[e];
    s->finished = b->finished[e];
    for (int p = 0; p < ORC_MAX_P; p++) s->gpos[p] = p < P ? b->gpos[(size_t)e * P + p] : -1;
}

static void store_env(const orc_env *s, const orc_cfg *cfg, orc_batch *b, int e)
{
    const int HW = cfg->H * cfg->W, P = cfg->P;
    memcpy(b->owner + (size_t)e * HW, s->owner, (size_t)HW);
    memcpy(b->army + (size_t)e * HW, s->army, (size_t)HW * 4);
    memcpy(b->type + (size_t)e * HW, s->type, (size_t)HW);
    b->turn[e] = s->turn;
    b->episode[e] = s->episode;
    b->alive[e] = s->alive;
    b->finished[e] = s->finished;
    for (int p = 0; p < P; p++) b->gpos[(size_t)e * P + p] = s->gpos[p];
}

/* Global id of env e of a batch: every random draw of the env is keyed by it. */
static uint64_t env_id_of(const orc_cfg *cfg, int e)
{
    return cfg->env_ids ? cfg->env_ids[e] : cfg->env_base + (uint64_t)e;
}

static int cfg_ok(const orc_cfg *cfg)
{
    if (cfg->H < 3 || cfg->W < 3 || cfg->H * cfg->W > ORC_MAX_CELLS) return 0;
    if (cfg->P < 2 || cfg->P > ORC_MAX_P) return 0;
    if (cfg->mode == M_1V1 && cfg->P != 2) return 0;
    if (cfg->mode == M_2V2 && cfg->P != 4) return 0;
    return 1;
}

/* ---------------- exported batch entry points (ctypes) ---------------- */

/* Fresh maps for envs env_base..env_base+E-1 at episode 0.  attempts[e] gets
 * the generator attempt used (128 = deterministic last resort).  Returns -1 on
 * a bad configuration. */
int orc_reset_batch(const orc_cfg *cfg, int32_t E, orc_batch *b, int32_t *attempts)
{
    orc_env s;
    if (!cfg_ok(cfg)) return -1;
    for (int e = 0; e < E; e++) {
        uint64_t id = env_id_of(cfg, e);
        int a = mapgen(&s, cfg, id, 0);
        pregrow(&s, cfg, id);
        if (attempts) attempts[e] = a;
        store_env(&s, cfg, b, e);
    }
    return 0;
}

/* One step of every env: actions [E][P] -> rewards [E][P], done [E]. */
int orc_step_batch(const orc_cfg *cfg, int32_t E, orc_batch *b, const int32_t *actions,
                   int32_t *rewards, uint8_t *done)
{
    orc_env s;
    if (!cfg_ok(cfg)) return -1;
    for (int e = 0; e < E; e++) {
        load_env(&s, cfg, b, e);
        step_env(&s, cfg, env_id_of(cfg, e), actions + (size_t)e * cfg->P,
                 rewards + (size_t)e * cfg->P, done + e);
        store_env(&s, cfg, b, e);
    }
    return 0;
}

/* Observation of every env: obs [E][P][8][H][W]. */
int orc_observe_batch(const orc_cfg *cfg, int32_t E, const orc_batch *b, uint8_t *obs)
{
    orc_env s;
    if (!cfg_ok(cfg)) return -1;
    const size_t per = (size_t)cfg->P * 8 * cfg->H * cfg->W;
    for (int e = 0; e < E; e++) {
        load_env(&s, cfg, b, e);
        observe_env(&s, obs + (size_t)e * per);
    }
    return 0;
}

/* Public scoreboard (Section IV-B): land [E][P] and army [E][P]. */
int orc_scoreboard_batch(const orc_cfg *cfg, int32_t E, const orc_batch *b, int32_t *land, int64_t *army)
{
    if (!cfg_ok(cfg)) return -1;
    const int HW = cfg->H * cfg->W, P = cfg->P;
    for (int e = 0; e < E; e++) {
        for (int p = 0; p < P; p++) { land[(size_t)e * P + p] = 0; army[(size_t)e * P + p] = 0; }
        for (int c = 0; c < HW; c++) {
            int o = b->owner[(size_t)e * HW + c];
            if (o < 0) continue;
            land[(size_t)e * P + o] += 1;
            army[(size_t)e * P + o] += b->army[(size_t)e * HW + c];
        }
    }
    return 0;
}

/* Random legal actions for every env (R15). */
int orc_sample_batch(const orc_cfg *cfg, int32_t E, const orc_batch *b, uint64_t seed_act,
                     uint64_t step_idx, int32_t *actions)
{
    orc_env s;
    if (!cfg_ok(cfg)) return -1;
    for (int e = 0; e < E; e++) {
        load_env(&s, cfg, b, e);
        sample_env(&s, seed_act, step_idx, env_id_of(cfg, e), actions + (size_t)e * cfg->P);
    }
    return 0;
}

/* The whole loop the GPU path runs per step -- sample, step, observe -- for
 * n_steps starting at global step step0.  Used to time the oracle. */
int orc_run(const orc_cfg *cfg, int32_t E, orc_batch *b, uint64_t seed_act, uint64_t step0,
            int32_t n_steps, int32_t *actions, int32_t *rewards, uint8_t *done, uint8_t *obs)
{
    for (int t = 0; t < n_steps; t++) {
        if (orc_sample_batch(cfg, E, b, seed_act, step0 + (uint64_t)t, actions) != 0) return -1;
        if (orc_step_batch(cfg, E, b, actions, rewards, done) != 0) return -1;
        if (orc_observe_batch(cfg, E, b, obs) != 0) return -1;
    }
    return 0;
}

/* ======================================================================
 * The paper's full feature tensor (Appendix A, table of observation
 * channels; reading R17): C = 24 + 2 * 7 = 38 float32 maps per player.
 *
 * Per env the oracle keeps, for the current episode, a running memory of
 * what each player has seen (the persistent channels 4..8, 20, 21) and the
 * own- and enemy-army channel values of the last 8 recorded frames (for the
 * delta stacks 24..37).  A frame is the state after a step, keyed by its
 * turn; recording the same turn twice changes nothing, and a turn with no
 * recorded frame (before the episode, or skipped by the caller) counts as
 * an empty board.  A state of another episode starts a fresh memory.
 * parity unpinned for the readings themselves (R17): the channel
 * definitions below are how this implementation reads the table.
 * ==================================================================== */
#define ORC_FEAT_C 38
#define ORC_HIST 7           /* H_hist, the delta stack depth */
#define ORC_FRAMES 8         /* frames t-7 .. t */
#define ORC_WINDOW 512       /* scoreboard window of the two temporal tokens */

typedef struct orc_fmem {
    int32_t valid;                                /* 0: no frame recorded yet */
    uint32_t episode;
    uint8_t seen[ORC_MAX_P][ORC_MAX_CELLS];       /* ever visible */
    uint8_t enemy_seen[ORC_MAX_P][ORC_MAX_CELLS]; /* ever visible while enemy-owned */
    uint8_t gen_seen[ORC_MAX_P][ORC_MAX_CELLS];   /* ever visible as a general */
    uint8_t castle_seen[ORC_MAX_P][ORC_MAX_CELLS];
    uint8_t mtn_seen[ORC_MAX_P][ORC_MAX_CELLS];
    int32_t last_army[ORC_MAX_P][ORC_MAX_CELLS];  /* enemy army at the last visible frame (0 if none) */
    int32_t last_enemy_turn[ORC_MAX_P][ORC_MAX_CELLS]; /* turn of the last enemy sighting, if enemy_seen */
    int32_t n_frames;                             /* kept frames, oldest first */
    int32_t frame_turn[ORC_FRAMES];
    int32_t own[ORC_FRAMES][ORC_MAX_P][ORC_MAX_CELLS];   /* channel 1 of that frame */
    int32_t enemy[ORC_FRAMES][ORC_MAX_P][ORC_MAX_CELLS]; /* channel 2 of that frame */
    int32_t n_score;                              /* kept scoreboard records, oldest first */
    int32_t score_turn[ORC_WINDOW];
    int32_t opp_land[ORC_WINDOW][ORC_MAX_P];      /* land of all of p's enemies at that turn */
    int64_t opp_army[ORC_WINDOW][ORC_MAX_P];      /* their army total */
} orc_fmem;

/* An enemy of player p owns the cell: owned, and not by p's team. */
static int enemy_of(const orc_env *s, int owner, int p)
{
    return owner >= 0 && !in_team(s, owner, p);
}

/* Team vision (Section IV-B, R10): a cell is visible to p if a cell of p's
 * team lies in its 3 x 3 neighbourhood. */
static int visible(const orc_env *s, int p, int cell)
{
    const int H = s->H, W = s->W, r = cell / W, c = cell % W;
    for (int dr = -1; dr <= 1; dr++) {
        for (int dc = -1; dc <= 1; dc++) {
            int nr = r + dr, nc = c + dc;
            if (nr < 0 || nr >= H || nc < 0 || nc >= W) continue;
            if (in_team(s, s->owner[nr * W + nc], p)) return 1;
        }
    }
    return 0;
}

/* Index of the kept frame with turn t (the latest such), or -1. */
static int frame_at(const orc_fmem *m, int64_t t)
{
    for (int i = m->n_frames - 1; i >= 0; i--)
        if (m->frame_turn[i] == t) return i;
    return -1;
}

/* Record the current frame into the memory and write the 38 channels of
 * every player, feat [P][38][H*W], and, if tok is not NULL, the two
 * temporal tokens of every player (Section V-A, network architecture):
 * tok [P][2][512], row 0 the enemies' army total and row 1 their land for
 * the turns t-511 .. t (oldest first; 0 for a turn with no record). */
static void features_env(const orc_env *s, orc_fmem *m, float *feat, float *tok)
{
    const int H = s->H, W = s->W, HW = H * W, P = s->P;
    int vis[ORC_MAX_P][ORC_MAX_CELLS];
    int32_t land[ORC_MAX_P];
    int64_t army[ORC_MAX_P];

    if (!m->valid || m->episode != s->episode) {
        memset(m, 0, sizeof(*m));
        m->valid = 1;
        m->episode = s->episode;
    }
    for (int p = 0; p < P; p++) {
        land[p] = 0;
        army[p] = 0;
        for (int c = 0; c < HW; c++) vis[p][c] = visible(s, p, c);
    }
    for (int c = 0; c < HW; c++) {
        if (s->owner[c] >= 0) {
            land[s->owner[c]] += 1;
            army[s->owner[c]] += s->army[c];
        }
    }

    /* the running memory takes this frame first: "ever seen" includes now */
    for (int p = 0; p < P; p++) {
        for (int c = 0; c < HW; c++) {
            if (!vis[p][c]) continue;
            const int en = enemy_of(s, s->owner[c], p);
            m->seen[p][c] = 1;
            if (en) {
                m->enemy_seen[p][c] = 1;
                m->last_enemy_turn[p][c] = s->turn;
            }
            if (s->type[c] == T_GENERAL) m->gen_seen[p][c] = 1;
            if (s->type[c] == T_CASTLE) m->castle_seen[p][c] = 1;
            if (s->type[c] == T_MOUNTAIN) m->mtn_seen[p][c] = 1;
            m->last_army[p][c] = en ? s->army[c] : 0;
        }
    }

    /* keep the frame (a repeated turn replaces its own entry) */
    int slot;
    if (m->n_frames > 0 && m->frame_turn[m->n_frames - 1] == s->turn) {
        slot = m->n_frames - 1;
    } else {
        if (m->n_frames == ORC_FRAMES) {
            memmove(&m->frame_turn[0], &m->frame_turn[1], sizeof(int32_t) * (ORC_FRAMES - 1));
            memmove(&m->own[0], &m->own[1], sizeof(m->own[0]) * (ORC_FRAMES - 1));
            memmove(&m->enemy[0], &m->enemy[1], sizeof(m->enemy[0]) * (ORC_FRAMES - 1));
            m->n_frames--;
        }
        slot = m->n_frames++;
    }
    m->frame_turn[slot] = s->turn;
    for (int p = 0; p < P; p++) {
        for (int c = 0; c < HW; c++) {
            m->own[slot][p][c] = s->owner[c] == p ? s->army[c] : 0;
            m->enemy[slot][p][c] = (vis[p][c] && enemy_of(s, s->owner[c], p)) ? s->army[c] : 0;
        }
    }

    for (int p = 0; p < P; p++) {
        int32_t opp_land = 0;
        int64_t opp_army = 0;
        for (int q = 0; q < P; q++) {
            if (q != p && !in_team(s, q, p)) {
                opp_land += land[q];
                opp_army += army[q];
            }
        }
        float *f = feat + (size_t)p * ORC_FEAT_C * HW;
        for (int c = 0; c < HW; c++) {
            const int r = c / W, col = c % W;
            const int o = s->owner[c], t = s->type[c], v = vis[p][c];
            const int32_t a = s->army[c];
            const int en = enemy_of(s, o, p);
            f[0 * HW + c] = (float)(v ? a : 0);
            f[1 * HW + c] = (float)(o == p ? a : 0);
            f[2 * HW + c] = (float)(v && en ? a : 0);
            f[3 * HW + c] = (float)(v && o < 0 ? a : 0);
            f[4 * HW + c] = (float)m->seen[p][c];
            f[5 * HW + c] = (float)m->enemy_seen[p][c];
            f[6 * HW + c] = (float)m->gen_seen[p][c];
            f[7 * HW + c] = (float)m->castle_seen[p][c];
            f[8 * HW + c] = (float)m->mtn_seen[p][c];
            f[9 * HW + c] = (float)(v && o < 0 && t != T_MOUNTAIN);
            f[10 * HW + c] = (float)(o == p);
            f[11 * HW + c] = (float)(v && en);
            f[12 * HW + c] = (float)(!v);
            f[13 * HW + c] = (float)(!v && (t == T_MOUNTAIN || t == T_CASTLE || m->gen_seen[p][c]));
            f[14 * HW + c] = (float)s->turn;
            f[15 * HW + c] = (float)((double)(s->turn % 50) / 50.0);
            f[16 * HW + c] = (float)land[p];
            f[17 * HW + c] = (float)army[p];
            f[18 * HW + c] = (float)opp_land;
            f[19 * HW + c] = (float)opp_army;
            f[20 * HW + c] = (float)m->last_army[p][c];
            f[21 * HW + c] = (v || !m->enemy_seen[p][c])
                                 ? 0.0f
                                 : (float)(log1p((double)(s->turn - m->last_enemy_turn[p][c])) / 5.0);
            f[22 * HW + c] = (float)((double)col / (double)(W - 1));
            f[23 * HW + c] = (float)((double)r / (double)(H - 1));
            for (int k = 0; k < ORC_HIST; k++) {
                const int i0 = frame_at(m, (int64_t)s->turn - k), i1 = frame_at(m, (int64_t)s->turn - k - 1);
                const int64_t own0 = i0 >= 0 ? m->own[i0][p][c] : 0, own1 = i1 >= 0 ? m->own[i1][p][c] : 0;
                const int64_t en0 = i0 >= 0 ? m->enemy[i0][p][c] : 0, en1 = i1 >= 0 ? m->enemy[i1][p][c] : 0;
                f[(24 + k) * HW + c] = (float)(own0 - own1);
                f[(24 + ORC_HIST + k) * HW + c] = (float)(en0 - en1);
            }
        }
    }

    /* scoreboard record of this turn (a repeated turn replaces its entry) */
    int rs;
    if (m->n_score > 0 && m->score_turn[m->n_score - 1] == s->turn) {
        rs = m->n_score - 1;
    } else {
        if (m->n_score == ORC_WINDOW) {
            memmove(&m->score_turn[0], &m->score_turn[1], sizeof(int32_t) * (ORC_WINDOW - 1));
            memmove(&m->opp_land[0], &m->opp_land[1], sizeof(m->opp_land[0]) * (ORC_WINDOW - 1));
            memmove(&m->opp_army[0], &m->opp_army[1], sizeof(m->opp_army[0]) * (ORC_WINDOW - 1));
            m->n_score--;
        }
        rs = m->n_score++;
    }
    m->score_turn[rs] = s->turn;
    for (int p = 0; p < P; p++) {
        m->opp_land[rs][p] = 0;
        m->opp_army[rs][p] = 0;
        for (int q = 0; q < P; q++) {
            if (q != p && !in_team(s, q, p)) {
                m->opp_land[rs][p] += land[q];
                m->opp_army[rs][p] += army[q];
            }
        }
    }
    if (tok == NULL) return;
    const int64_t first = (int64_t)s->turn - (ORC_WINDOW - 1);
    for (int p = 0; p < P; p++) {
        float *tp = tok + (size_t)p * 2 * ORC_WINDOW;
        for (int j = 0; j < 2 * ORC_WINDOW; j++) tp[j] = 0.0f;
        for (int i = 0; i < m->n_score; i++) {
            const int64_t j = (int64_t)m->score_turn[i] - first;
            if (j < 0 || j >= ORC_WINDOW) continue;
            tp[j] = (float)m->opp_army[i][p];
            tp[ORC_WINDOW + j] = (float)m->opp_land[i][p];
        }
    }
}

/* Size of one env's feature memory; the caller zero-fills E of them once. */
int64_t orc_fmem_bytes(void) { return (int64_t)sizeof(orc_fmem); }

/* Features of every env: mem [E] orc_fmem (updated), feat [E][P][38][H*W],
 * tok [E][P][2][512] or NULL. */
int orc_features_batch(const orc_cfg *cfg, int32_t E, const orc_batch *b, void *mem, float *feat, float *tok)
{
    orc_env s;
    if (!cfg_ok(cfg)) return -1;
    const size_t per = (size_t)cfg->P * ORC_FEAT_C * cfg->H * cfg->W;
    for (int e = 0; e < E; e++) {
        load_env(&s, cfg, b, e);
        features_env(&s, (orc_fmem *)mem + e, feat + (size_t)e * per,
                     tok ? tok + (size_t)e * cfg->P * 2 * ORC_WINDOW : NULL);
    }
    return 0;
}
