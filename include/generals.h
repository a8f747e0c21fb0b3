/*
 * generals.h -- C ABI of the MI355X (gfx950) batched Generals.io environment
 * step, after arxiv 2606.23348 ("Superhuman AI for Generals.io Using
 * Self-Play Reinforcement Learning"), Section IV (game description) and
 * Section IV-G (the batched environment, Table I).
 *
 * Conventions for every entry point:
 *  - Returns a gen_status; GEN_OK == 0.  On any other value a message is
 *    available from gen_last_error() on the calling thread.  Nothing is
 *    launched when an argument check fails.
 *  - "d_" pointers are device pointers (HIP device memory) owned by the
 *    caller; "h_" pointers are host memory owned by the caller.  The library
 *    never frees caller memory and allocates no device memory in the plain
 *    entry points (gen_get_envs keeps one staging block of its own per
 *    device, see there).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Launches are asynchronous on that stream unless a call says it blocks.
 *    Asynchronous kernel faults surface as GEN_EHIP on a later call.
 *  - Action codes follow the paper's H x W x 9 action space (Section IV-G):
 *    a = cell * 9 + k, cell = row * W + col; k = 0 pass, k = 1..4 send
 *    all-but-one unit up/down/left/right, k = 5..8 send half (rounded down)
 *    up/down/left/right.  Any code that is out of range, has k = 0, or is
 *    illegal under the rules (Section IV-D) is a pass, never an error.
 *  - Players: 2 in 1v1, 4 in 2v2 (team = id mod 2), 2..8 in free-for-all.
 *  - All arithmetic is exact integer arithmetic; army additions saturate at
 *    INT32_MAX.
 */
#ifndef GENERALS_H
#define GENERALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEN_LAYOUT_VERSION 1
#define GEN_MAX_PLAYERS 8
#define GEN_MIN_SIDE 3
#define GEN_MAX_SIDE 32
#define GEN_MAX_CELLS 1024
#define GEN_OBS_CHANNELS 8

typedef enum gen_status {
    GEN_OK = 0,
    GEN_EINVAL = -1,    /* bad argument, shape, mode or state contents */
    GEN_ENOMEM = -2,    /* a caller buffer is too small, or a host allocation failed */
    GEN_EHIP = -3,      /* the HIP runtime reported an error */
    GEN_EBUDGET = -4,   /* admission refused: the device-memory budget is exhausted */
    GEN_EBUSY = -5,     /* not finished yet (wait with a timeout) */
    GEN_ENOTFOUND = -6  /* unknown handle or ticket */
} gen_status;

/* Game formats (Section IV-E). */
typedef enum gen_mode { GEN_1V1 = 0, GEN_2V2 = 1, GEN_FFA = 2 } gen_mode;

/* Cell types (Section IV-A: plain, mountain, castle, general). */
enum { GEN_PLAIN = 0, GEN_MOUNTAIN = 1, GEN_CASTLE = 2, GEN_GENERAL = 3 };

/* Observation channels, uint8 [E][P][8][H][W] (8-channel reduction of the
 * paper's Appendix A feature tensor; fog as in Section IV-B): */
enum {
    GEN_OBS_OWN = 0,       /* cell owned by the observing player */
    GEN_OBS_ENEMY = 1,     /* visible, owned by a player outside the observer's team */
    GEN_OBS_NEUTRAL = 2,   /* visible, unowned, not a mountain */
    GEN_OBS_MOUNTAIN = 3,  /* visible mountain */
    GEN_OBS_CASTLE = 4,    /* visible castle (city) */
    GEN_OBS_GENERAL = 5,   /* visible general */
    GEN_OBS_FOG = 6,       /* not visible */
    GEN_OBS_ARMY = 7       /* visible army, clamped to 255; 0 under fog */
};

/* Map-generator and episode parameters (Section IV-A generator family). */
typedef struct gen_params {
    int32_t n_players;          /* FFA: 2..8.  Ignored for 1v1 (2) and 2v2 (4). */
    uint32_t mountain_thresh;   /* a cell is a mountain iff its 32-bit draw < thresh
                                   (floor(2^32 * density); 858993459 for 20%) */
    int32_t cities_min, cities_max;       /* neutral castles per map, inclusive */
    int32_t city_army_min, city_army_max; /* their starting armies, inclusive */
    int32_t min_general_dist;   /* Manhattan distance between any two generals */
    int32_t auto_reset;         /* 1: a finished game restarts on the next map in the same step */
    int32_t pregrow;            /* 1: at episode 0, envs with global id % 4 == 0 start
                                   each general at 100000 + U{0..900000} */
    int32_t generator;          /* 0: synthetic generator (Manhattan spacing, cities
                                   anywhere); 1: the official rules (Section IV-A):
                                   spacing in BFS steps over non-mountain cells and a
                                   castle within castle_radius steps of every general */
    int32_t max_general_dist;   /* generator 1: cap on the BFS distance between generals
                                   (the spawn-distance curriculum, Section V-C); 0 = none */
    int32_t castle_radius;      /* generator 1: BFS radius of the guaranteed castle (6) */
    int32_t obs_layout;         /* observation layout of the plain-batch calls (gen_step,
                                   gen_step_sample, gen_observe, gen_reset): 0 = dense
                                   uint8 [E][P][8][H][W]; 1 = each plane H*W bytes then
                                   zero bytes up to a multiple of 32 (of 64 with more
                                   than 2 players), uint8 [E][P][8][PS] with
                                   PS = (H*W + 31) & ~31, or (H*W + 63) & ~63 when P > 2
                                   (the same as 0 when H*W is a multiple of that).  1 lets
                                   every env's planes be written with aligned streaming
                                   stores.  Pools always use 1. */
    int32_t reserved[3];        /* must be zero */
} gen_params;

/* Descriptor of one batch of identical envs living in one device buffer.
 * Filled by gen_layout() / gen_reset(); the caller keeps it and passes it to
 * every later call.  It holds no device resources. */
typedef struct gen_state {
    uint32_t version;           /* GEN_LAYOUT_VERSION */
    int32_t n_envs, H, W, mode, n_players;
    int32_t stride;             /* cells per env in the grid arrays: H*W rounded up to 16 */
    int32_t reserved0;
    uint64_t seed;              /* map seed: draws of every (re)generated map */
    uint64_t env_base;          /* global id of env 0 (keys every random draw) */
    gen_params params;
    /* Device buffer layout (bytes from d_buf), struct-of-arrays, env-major:
     *   scalars [n_envs] 32-byte records {int32 turn; uint32 episode;
     *           uint8 alive_mask; uint8 finished; uint8 pad[2]; uint32 tick;
     *           int16 gpos[8]; }
     *   owner   int8  [n_envs][stride]  (-1 neutral)
     *   type    uint8 [n_envs][stride]
     *   army    int32 [n_envs][stride]
     * Cells past H*W in a row are padding (neutral plain, 0 units). */
    uint64_t off_scalars, off_owner, off_type, off_army;
    uint64_t bytes;             /* device bytes the buffer must hold */
    void *d_buf;                /* device buffer (set by gen_reset) */
} gen_state;

/* Host copy of a batch in the public host-state format (all C-contiguous,
 * caller-owned):  owner int8 [E][H*W], army int32 [E][H*W], type uint8
 * [E][H*W], turn int32 [E], episode uint32 [E], alive uint8 [E] (bit p set
 * while player p has a general), finished uint8 [E] (1 once a game ended
 * with auto_reset off; such an env is frozen), gpos int16 [E][P]. */
typedef struct gen_host_state {
    int8_t *owner;
    int32_t *army;
    uint8_t *type;
    int32_t *turn;
    uint32_t *episode;
    uint8_t *alive;
    uint8_t *finished;
    int16_t *gpos;
} gen_host_state;

/* Library version (GEN_LAYOUT_VERSION of the build). */
int gen_version(void);

/* Message of the last non-OK return on this thread ("" if none).  The
 * pointer stays valid until the next call on the same thread. */
const char *gen_last_error(void);

/* Defaults (Section IV-A): 20% mountains, 9..11 castles of 40..50 units,
 * auto-reset on, the synthetic generator with generals at least 9 apart
 * (Manhattan); castle_radius 6.  For the official rules set generator = 1
 * and min_general_dist = 17; for a curriculum stage, min_general_dist = 1
 * and max_general_dist = the stage's cap. */
int gen_default_params(int32_t mode, int32_t n_players, gen_params *out);

/* Compute the device layout of n_envs envs of H x W (3..32 each side) in
 * `mode` without touching the device.  params NULL = defaults.  Fills *out
 * (d_buf = NULL).  GEN_EINVAL on a bad shape (n_envs < 1 included: an empty
 * batch has no layout), mode or parameter. */
int gen_layout(int32_t n_envs, int32_t H, int32_t W, int32_t mode, const gen_params *params,
               uint64_t seed, gen_state *out);

/* Device bytes needed for such a batch (0 on invalid input). */
uint64_t gen_state_bytes(int32_t n_envs, int32_t H, int32_t W, int32_t mode, const gen_params *params);

/* Generate fresh maps (Section IV-A; randomness only in the initial state,
 * Section III) for envs env_base .. env_base+n_envs-1 at episode 0 into
 * d_buf (buf_bytes >= gen_state_bytes, 256-byte aligned), fill *out, and, if
 * d_obs is not NULL, write the initial observation uint8 [E][P][8][H][W].
 * GEN_ENOMEM if buf_bytes is too small. */
int gen_reset(uint64_t seed, uint64_t env_base, int32_t n_envs, int32_t H, int32_t W, int32_t mode,
              const gen_params *params, void *d_buf, uint64_t buf_bytes, uint8_t *d_obs, void *stream,
              gen_state *out);

/* One environment step of every env (Sections IV-B..IV-E): moves in
 * rotating priority, combat, general capture and land transfer, growth,
 * terminal rewards, optional auto-reset, fog and observation.
 *   d_actions  int32 [E][P]   (read)
 *   d_obs      uint8 [E][P][8][H][W]  (written; after an auto-reset this is
 *              the new map's observation)
 *   d_rewards  int32 [E][P]   (written: +1 win, -1 loss, else 0)
 *   d_dones    uint8 [E]      (written: 1 when the game ended on this step,
 *              or was already over and frozen)
 *   d_land     int32 [E][P]   (nullable; scoreboard land, Section IV-B)
 *   d_army     int64 [E][P]   (nullable; scoreboard army total) */
int gen_step(const gen_state *st, const int32_t *d_actions, uint8_t *d_obs, int32_t *d_rewards,
             uint8_t *d_dones, int32_t *d_land, int64_t *d_army, void *stream);

/* Random legal actor (the action source of the benchmarks; the paper fixes no generator):
 * for every env, player p takes 32-bit word p mod 4 of the Philox4x32-10
 * block with key (actor_seed low, actor_seed high) and counter (step_idx
 * low, step_idx high, env low, env high), env = env_base + e, the counter's
 * top bit flipped for players 4..7 (env ids below 2^63), and picks
 * uniformly, floor(word * n / 2^32), among the n entries of [pass] + the
 * legal (cell, k) moves listed by cell in row-major order, then k = 1..8.
 * Dead players pass.  d_actions int32 [E][P]. */
int gen_sample_actions(const gen_state *st, uint64_t actor_seed, uint64_t step_idx, int32_t *d_actions,
                       void *stream);

/* gen_step followed by gen_sample_actions in one launch: the step consumes
 * d_actions, then the random legal actor samples the next step's actions
 * (Philox counter step index `next_step_idx`) from the post-step state --
 * after growth and any auto-reset -- and writes them back into d_actions.
 * Results are identical to the two separate calls; the state is read from
 * HBM once instead of twice. */
int gen_step_sample(const gen_state *st, int32_t *d_actions, uint64_t actor_seed, uint64_t next_step_idx,
                    uint8_t *d_obs, int32_t *d_rewards, uint8_t *d_dones, int32_t *d_land, int64_t *d_army,
                    void *stream);

/* Observation of the current state (no state change). */
int gen_observe(const gen_state *st, uint8_t *d_obs, void *stream);

/* ------------------------------------------------------------------------
 * The paper's full feature tensor (Appendix A, table of observation
 * channels): float32 [E][P][38][H][W] per call, for every player of every
 * env, from the current state and a per-env memory that the calls keep.
 *   0 army on visible cells          1 army on the player's own cells
 *   2 army on visible enemy cells    3 army on visible neutral cells
 *   4 ever visible                   5 ever seen enemy-owned
 *   6 general ever seen              7 castle ever seen
 *   8 mountain ever seen             9 visible neutral non-mountain
 *  10 own cell                      11 visible enemy cell
 *  12 fog                           13 fog over a mountain, castle or a general seen before
 *  14 turn                          15 (turn mod 50) / 50
 *  16 own land                      17 own army total
 *  18 land of all enemies           19 army of all enemies
 *  20 enemy army at the cell's last visible frame
 *  21 log(1 + turns since an enemy was last seen there) / 5 (0 while visible)
 *  22 col / (W - 1)                 23 row / (H - 1)
 *  24+k, 31+k (k = 0..6): own (channel 1), resp. visible-enemy (channel 2)
 *     army of the frame of turn t-k minus that of turn t-k-1.
 * "Enemy" = owned by a player outside the observer's team; vision is the
 * team's (as in gen_step).  A frame is the state after a step, keyed by its
 * turn: call gen_features once after gen_reset and after every step.  A turn
 * that was not recorded counts as an empty board in the delta stacks; the
 * first call on a state of a new episode (auto-reset) starts a fresh memory;
 * calling twice on the same state returns the same tensor.  Values are
 * exact integers converted to float32 (round to nearest even), except 15,
 * 21, 22 and 23 (computed in double, rounded once to float32).
 * The two temporal tokens of the network input (Section V-A) come with the
 * same call: float32 [E][P][2][512], for each player the army total (row 0)
 * and the land (row 1) of all its enemies at turns t-511 .. t, oldest
 * first, 0 for a turn that was not recorded.
 * ---------------------------------------------------------------------- */
#define GEN_FEAT_CHANNELS 38
#define GEN_FEAT_HISTORY 7
#define GEN_TOKEN_WINDOW 512

/* Device bytes of the feature memory of the batch `st` (0 if st is invalid).
 * The caller allocates it (256-byte aligned) and zero-fills it once before
 * the first gen_features call; after that only gen_features writes it. */
uint64_t gen_feat_mem_bytes(const gen_state *st);

/* Record the current state of every env into d_mem and write the features
 * d_feat float32 [E][P][38][H][W] and, if d_tokens is not NULL, the temporal
 * tokens d_tokens float32 [E][P][2][512].  GEN_ENOMEM if mem_bytes is too
 * small. */
int gen_features(const gen_state *st, void *d_mem, uint64_t mem_bytes, float *d_feat, float *d_tokens,
                 void *stream);

/* A rollout for a learner (Appendix D, training hyperparameters: 512 envs x
 * 512 steps per iteration),
 * driven by the random actor in place of a policy: for t = 0 .. n_steps-1,
 *   features of the current state  -> d_feat   [t][E][P][38][H][W]
 *   (and tokens if not NULL)       -> d_tokens [t][E][P][2][512]
 *   actor draws, step index step0+t -> d_actions [t][E][P]
 *   one step                        -> d_rewards [t][E][P], d_dones [t][E]
 * exactly as gen_features, gen_sample_actions and gen_step called in that
 * order (no 8-channel observation is written).  2 launches per step on
 * `stream` (capture the stream into a HIP graph to replay whole rollouts).
 * The batch and d_mem advance by n_steps steps. */
int gen_rollout(const gen_state *st, void *d_mem, uint64_t mem_bytes, int32_t n_steps, uint64_t actor_seed,
                uint64_t step0, float *d_feat, float *d_tokens, int32_t *d_actions, int32_t *d_rewards, uint8_t *d_dones,
                void *stream);

/* Blocking copies between the device buffer and the public host format
 * (synchronises `stream`).  gen_set_state rejects (GEN_EINVAL) contents the
 * kernels cannot take: owner outside [-1, P), type outside [0, 3], negative
 * army, gpos outside the grid, alive bits beyond P, negative turn. */
int gen_get_state(const gen_state *st, gen_host_state *h, void *stream);
int gen_set_state(const gen_state *st, const gen_host_state *h, void *stream);

/* ------------------------------------------------------------------------
 * Batched pool: envs of different shapes and modes stepped by one launch.
 * Each env keeps its own shape (3..32 per side), mode, player count and
 * generator settings; the state lives in one caller-provided device buffer
 * (layout private to the library), observations, actions and rewards in
 * ragged caller buffers at the offsets gen_pool_offsets reports.  An env's
 * observation block holds its [P][8] planes (channels as in gen_step), each
 * plane H*W bytes row-major followed by zero bytes up to a multiple of 32,
 * or of 64 for envs of more than 2 players (plane stride PS = (H*W + 31) & ~31,
 * or (H*W + 63) & ~63 when P > 2, so plane (p, ch) starts at byte
 * (8p + ch) * PS of the block): every plane starts on a 32-byte sector and
 * the whole block is written with aligned 4-byte streaming stores.  The random
 * actor of a pool draws with each env's own step counter (0 at reset, +1
 * per step) as its step index, so a captured graph can be replayed any
 * number of times and keeps drawing fresh actions.
 * ---------------------------------------------------------------------- */
typedef struct gen_env_spec {
    int32_t H, W, mode, n_players;        /* n_players: FFA only (2..8) */
    int32_t cities_min, cities_max;       /* <= 255 */
    int32_t min_general_dist;             /* <= 255 */
    int32_t reserved;                     /* must be zero */
} gen_env_spec;

typedef struct gen_pool gen_pool;        /* opaque host object; owns no device memory */

typedef struct gen_pool_info {
    int32_t n_envs;
    int32_t max_cells;          /* largest H*W in the pool */
    uint64_t state_bytes;       /* device state buffer to pass to gen_pool_reset */
    uint64_t obs_bytes;         /* ragged observation buffer (each env block P*8*PS bytes, 16-byte aligned) */
    uint64_t n_actions;         /* int32 entries of the ragged actions and rewards buffers (sum of P) */
    uint64_t work_list_off;     /* the work list inside the state buffer: the only bytes */
    uint64_t work_list_bytes;   /* of the state that depend on the packing (gen_pool_tuning) */
} gen_pool_info;

/* Packing of envs onto the GPU (chosen by the autotuner):
 *   waves_per_group 1, 2 or 4 envs (one wave each) per workgroup;
 *   grid            0 = one wave per env, else that many workgroups whose
 *                   waves stride over the work list;
 *   order           0 = env id order, 1 = largest envs (P*H*W) first. */
typedef struct gen_pool_tuning {
    int32_t waves_per_group, grid, order, reserved;
} gen_pool_tuning;

/* Packing of one size bucket of a pool: the envs with n_players players
 * whose map takes `words` 64-cell words (ceil(H*W / 64)).  Envs of buckets
 * that share a packing are stepped by one launch; a pool with several
 * packings takes one launch per distinct packing each step.
 *   waves_per_group  1, 2 or 4 envs (one wave each) per workgroup;
 *   waves_per_env    1, or 2: a second wave of the env's workgroup writes
 *                    the observation planes of players floor(3P/8) .. P-1
 *                    (then waves_per_group must be 1). */
typedef struct gen_pool_bucket {
    int32_t n_players, words;
    int32_t n_envs;             /* envs of the pool in the bucket (filled by gen_pool_buckets; ignored on set) */
    int32_t waves_per_group, waves_per_env;
    int32_t reserved[3];        /* must be zero */
} gen_pool_bucket;

/* Plan a pool of n_envs envs described by h_specs[n_envs] (host).  `common`
 * supplies the mountain threshold, city armies, auto_reset and pregrow
 * (NULL: defaults); its city counts, spawn distance and n_players are
 * ignored in favour of each spec.  GEN_EINVAL for n_envs < 1 or a bad spec. */
int gen_pool_create(uint64_t seed, uint64_t env_base, int32_t n_envs, const gen_env_spec *h_specs,
                    const gen_params *common, gen_pool **out);
int gen_pool_destroy(gen_pool *pool);
int gen_pool_query(const gen_pool *pool, gen_pool_info *out);
/* Byte offset of each env's observation block and index of its first action
 * (host arrays of n_envs entries; either may be NULL). */
int gen_pool_offsets(const gen_pool *pool, uint64_t *h_obs_off, uint32_t *h_act_off);
int gen_pool_get_tuning(const gen_pool *pool, gen_pool_tuning *out);
/* Takes effect at the next launch (uploads the work list if the pool is bound;
 * blocking on `stream`).  Results never depend on the packing.  The
 * pool-wide waves_per_group applies to the buckets gen_pool_set_buckets does
 * not list (and to the reset launch); grid applies to every one-wave-per-env
 * launch. */
int gen_pool_set_tuning(gen_pool *pool, const gen_pool_tuning *tuning, void *stream);
/* The pool's size buckets (in order of n_players, then words) with their
 * env counts and current packing: *n_out = number of buckets; up to
 * `capacity` of them are written to out (NULL allowed to query the count). */
int gen_pool_buckets(const gen_pool *pool, gen_pool_bucket *out, int32_t capacity, int32_t *n_out);
/* Set the packing of the listed buckets (others keep the pool-wide one);
 * n = 0 clears the table.  Same effect rules as gen_pool_set_tuning.  A
 * captured graph keeps the launches it captured: capture again after. */
int gen_pool_set_buckets(gen_pool *pool, const gen_pool_bucket *table, int32_t n, void *stream);
/* Bind the state buffer (>= state_bytes, 256-byte aligned), generate every
 * env's first map, write observations (d_obs nullable) and, if d_actions is
 * not NULL, the random actor's actions for step 0. */
int gen_pool_reset(gen_pool *pool, void *d_state, uint64_t state_bytes, uint8_t *d_obs, int32_t *d_actions,
                   uint64_t actor_seed, void *stream);
/* One step of every env.  actor != 0: afterwards draw the next actions into
 * d_actions with the random actor (fused, same launch). */
int gen_pool_step(gen_pool *pool, int32_t *d_actions, int32_t actor, uint64_t actor_seed, uint8_t *d_obs,
                  int32_t *d_rewards, uint8_t *d_dones, void *stream);
/* Capture k_steps fused steps (actor on) on `stream` (not the null stream)
 * into a HIP graph held by the pool; replay it with gen_pool_replay. */
int gen_pool_capture(gen_pool *pool, int32_t k_steps, int32_t *d_actions, uint64_t actor_seed, uint8_t *d_obs,
                     int32_t *d_rewards, uint8_t *d_dones, void *stream);
int gen_pool_replay(gen_pool *pool, void *stream);
/* Blocking copy of one env in the public host format (one row of H*W cells). */
int gen_pool_get_env(const gen_pool *pool, int32_t env, gen_host_state *h, void *stream);

/* Blocking copy of every env of a pool in the public host format, ragged
 * (for checkpoints and whole-pool parity checks): owner, army and type hold
 * the envs' H*W cells back to back in env order (env i starts at the sum of
 * H*W over envs 0 .. i-1); turn, episode, alive and finished hold one entry
 * per env; gpos holds GEN_MAX_PLAYERS entries per env, -1 past its players.
 * The caller sizes the arrays; GEN_ENOMEM if the host copy of the state
 * buffer cannot be allocated. */
int gen_pool_get_state(const gen_pool *pool, gen_host_state *h, void *stream);

/* ------------------------------------------------------------------------
 * Served form: an environment server with continuous batching.
 * The caller hands the server one device arena; its size is the memory
 * budget.  Each opened group (a pool of envs of any shapes and modes) gets
 * its state, observations, actions, rewards and done flags carved out of the
 * arena, or GEN_EBUDGET when they do not fit.  Step requests from any number
 * of client threads are queued; a scheduler thread gathers the requests of
 * every group that is not already on the GPU into one launch (envs of
 * different groups and sizes side by side), keeps up to n_launch_streams
 * launches in flight, and completes tickets when their launch finishes.
 * A group is never in two launches at once, and every env is independent,
 * so results do not depend on how requests were batched.
 * ---------------------------------------------------------------------- */
typedef struct gen_server gen_server;

typedef struct gen_group_buffers {
    uint64_t state_off;         /* byte offsets into the arena */
    uint64_t obs_off;           /* ragged observations, per-env offsets from gen_pool_offsets(pool) */
    uint64_t actions_off, rewards_off, dones_off;
    uint64_t obs_bytes, n_actions;
    int32_t n_envs, reserved;
    gen_pool *pool;             /* the group's plan (offsets, gen_pool_get_env); owned by the server */
} gen_group_buffers;

typedef struct gen_server_stats {
    uint64_t requests, frames, launches;
    uint64_t groups_open;       /* admitted groups */
    uint64_t groups_queued;     /* opens that had to wait for memory (since the last reset) */
    uint64_t arena_bytes, bytes_in_use;
    /* step latency, submit -> completion seen by the server, over the
     * requests since the last reset: p50 and p99 from a histogram of 32
     * log-spaced buckets per power of two (within 1.6% of the sample),
     * mean and max exact */
    double lat_p50_us, lat_p99_us, lat_mean_us;
    double envs_per_launch;
    double wall_s;              /* gen_server_drive: length of the measured window */
    uint64_t groups_pending;    /* groups waiting for memory now */
    uint64_t lat_samples;
    double lat_max_us;
} gen_server_stats;

/* d_arena: device buffer of arena_bytes (256-byte aligned) the server may
 * use; n_launch_streams: launches in flight (1..4); max_batch_envs: cap on
 * envs per launch (0 = no cap).  Starts the scheduler thread.  The server
 * keeps one record per open group in a table carved from the arena at
 * creation (16,384 records of 192 bytes); a launch carries at most 512
 * requests, the list itself passed as the kernel argument (no copy). */
int gen_server_create(void *d_arena, uint64_t arena_bytes, int32_t n_launch_streams, int32_t max_batch_envs,
                      gen_server **out);
/* Finishes the work in flight, stops the scheduler, releases host objects. */
int gen_server_destroy(gen_server *srv);
/* Open a group: plan it (GEN_EBUSY when 16,384 groups are open or queued
 * already), and if its buffers fit in the arena now (and no
 * earlier group is waiting), carve them and generate its maps (blocking):
 * GEN_OK, *group is steppable.  If they do not fit, the group is queued:
 * GEN_EBUDGET with *group set, and it is admitted (buffers carved, maps
 * generated) in order of arrival as soon as closes free enough memory; a
 * group larger than the whole arena is refused with GEN_EINVAL.  Requests
 * may be submitted to a queued group: they run once it is admitted.
 * actor != 0: every step also draws the group's next actions with the random
 * actor (seed actor_seed, each env's own step counter); else the caller
 * writes actions into the group's action buffer before each request. */
int gen_server_open(gen_server *srv, uint64_t seed, uint64_t env_base, int32_t n_envs, const gen_env_spec *h_specs,
                    const gen_params *common, int32_t actor, uint64_t actor_seed, uint64_t *group);
/* Wait until a queued group is admitted: GEN_OK (at once for an admitted
 * group), GEN_EBUSY if timeout_us passed first (timeout_us < 0: wait
 * forever), GEN_ENOTFOUND if it was closed, GEN_EHIP if its admission failed. */
int gen_server_wait_admitted(gen_server *srv, uint64_t group, int64_t timeout_us);
/* Buffers of an admitted group (GEN_EBUSY while it is queued). */
int gen_server_buffers(gen_server *srv, uint64_t group, gen_group_buffers *out);
/* Queue one step of every env of the group; *ticket identifies it. */
int gen_server_submit(gen_server *srv, uint64_t group, uint64_t *ticket);
/* GEN_OK when the step is done (its outputs are in the group's buffers),
 * GEN_EBUSY if timeout_us passed first (timeout_us < 0: wait forever),
 * GEN_ENOTFOUND for an unknown or already collected ticket (a finished
 * ticket is kept until it is collected or 2^18 newer tickets were issued;
 * a pending one is never dropped: submit returns GEN_EBUSY instead). */
int gen_server_wait(gen_server *srv, uint64_t ticket, int64_t timeout_us);
/* Waits for the group's work in flight, drops its queued requests (their
 * tickets fail with GEN_ENOTFOUND) and returns its memory to the arena,
 * then admits the queued groups that now fit.  A queued group is simply
 * taken off the queue. */
int gen_server_close(gen_server *srv, uint64_t group);
int gen_server_report(gen_server *srv, gen_server_stats *out, int32_t reset);

/* Batching window: a launch starts when every open group is either on the
 * GPU or has a request waiting, or when the waiting requests hold
 * min_batch_envs envs (0 = a quarter of the envs of the open groups), or
 * when the oldest of them has waited max_wait_us (default 100).  Larger
 * batches spread the per-launch host cost over more envs; max_wait_us
 * bounds the latency it adds. */
int gen_server_set_batching(gen_server *srv, int64_t min_batch_envs, int64_t max_wait_us);

/* Synthetic clients for measuring the server (load generator, not part of
 * the step): n_clients logical clients (run as state machines by up to 8
 * threads), each owning groups_per_client groups opened from h_specs (env
 * specs of all groups back to back, group g has h_group_envs[g] envs), each
 * issuing, when its arrival timer fires, one request for its next group in
 * turn once that group's previous request has completed (closed loop per
 * group); the timer follows the arrival gaps h_gaps_us[client][k]
 * (microseconds; all zero = back to back) until duration_us has passed.  A group that reached steps_per_group steps is
 * closed and reopened (same specs, next env ids) when steps_per_group > 0.
 * Returns the stats of the run. */
int gen_server_drive(gen_server *srv, int32_t n_clients, int32_t groups_per_client, const int32_t *h_group_envs,
                     const gen_env_spec *h_specs, const gen_params *common, uint64_t seed, uint64_t actor_seed,
                     const double *h_gaps_us, int32_t gaps_per_client, int64_t duration_us, int32_t steps_per_group,
                     gen_server_stats *out);

/* Blocking copy of selected envs only: env h_env_ids[i] (0 <= id < n_envs)
 * goes to row i of each host array, which therefore hold n_ids rows.  For
 * checkpoints of part of a batch and for sampled parity checks.  One gather
 * kernel packs the envs into a device staging block in the host format, then
 * one copy per field comes down; the staging block is the library's own (one
 * per device, allocated on first use, grown when a larger gather needs it,
 * held until the process ends), and calls on one device take turns on it. */
int gen_get_envs(const gen_state *st, const int32_t *h_env_ids, int32_t n_ids, gen_host_state *h, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): gen_get_envs with its staging block in
 * the library's static device array of GEN_STATIC_STAGING_BYTES per device
 * (8 MiB, held by every device the library runs on until the process ends)
 * instead of a buffer the library allocates.  It allocates no device memory.
 * The state must live on the current device (GEN_EINVAL otherwise);
 * GEN_ENOMEM when the gather needs more than the array holds (n_ids * (6 *
 * H * W + 10 + 2 * P) bytes plus 256-byte alignment of each of 9 sections).
 * Every call on one device stages through that device's one array: calls
 * that overlap on one device race and must be serialised by the caller.
 * Blocking on `stream`, as gen_get_envs. */
#define GEN_STATIC_STAGING_BYTES (8u << 20)
int gen_get_envs_static(const gen_state *st, const int32_t *h_env_ids, int32_t n_ids, gen_host_state *h,
                        void *stream);

/* Measurement helper, not part of the step: copy `bytes` (a multiple of 16)
 * from d_src to d_dst (both 16-byte aligned device buffers, not overlapping)
 * with a plain streaming kernel (one 16-byte element per thread, plain
 * loads, nontemporal stores).  Timed next to the step kernels, it gives the
 * practical HBM ceiling of a read-once / write-once stream.  GEN_EINVAL on
 * a null or misaligned buffer or a size not a multiple of 16. */
int gen_stream_copy(void *d_dst, const void *d_src, uint64_t bytes, void *stream);

/* Measurement helper, not part of the step: write `dst_bytes` (a multiple of
 * 16, fewer than 2^32 16-byte chunks) to d_dst, chunk i being chunk
 * floor(i / k) of d_src, which must hold ceil(dst_bytes / 16 / k) chunks
 * (the caller owns both buffers: 16-byte aligned, on the current device, not
 * overlapping).  k = 1 is the copy above; the kernel has the copy's form.  A
 * stream writing k bytes per byte read: an env step writes 3.5 (1v1 24x24)
 * to 11 (FFA-8 25x25) times what it reads, so timed at the step's ratio it
 * gives the practical HBM ceiling of the step's mix of reads and writes.
 * k = 0 writes zeros and reads nothing (d_src may be NULL): a write-only
 * stream.  GEN_EINVAL on a null or misaligned buffer or a bad size.
 * Asynchronous on `stream`. */
int gen_stream_spread(void *d_dst, const void *d_src, uint64_t dst_bytes, uint32_t k, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GENERALS_H */
