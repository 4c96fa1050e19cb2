/*
 * jx_oracle.h -- plain, slow, single-threaded FP64 CPU oracle for the batched
 * first-person grid-world step and its raycast render.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library under paper_2605_19926_amd/) never links, imports or calls it,
 * and shares no source, header, table or helper with it.
 *
 * What it follows (JAXenstein, Tao & Konidaris):
 *   - Sec. 2.1 "Ray casting": one ray per image column, first wall hit, found by
 *     DDA marching along tile boundaries.
 *   - Sec. 2.2: the world is a tile map (2-D occupancy grid).
 *   - Fig. 1 caption: objects are fixed billboard sprites as in Wolfenstein 3D.
 *   - Sec. 3.2 and Table 2: common tile-map format with walls, coloured walls,
 *     keys, locked doors and goal; Table 1 key-door task (red key opens a red
 *     door, then reach the goal).
 * Everything the paper leaves open (camera, movement, collision, rewards, RNG,
 * maze generation, colours, sprite size) follows the readings written next to
 * each function in jx_oracle.c.
 */
#ifndef JX_ORACLE_H
#define JX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_SIDE 64
#define ORC_MAX_DECOR 2

/* Environment configuration, the oracle's own copy of the fields it needs.
 * Floating fields hold the float32 value the configuration was given in,
 * widened exactly to double by the caller. */
typedef struct {
  int32_t side;          /* N: tile-grid side */
  int32_t n_colors;      /* K: wall palette size (1..8) */
  double loop_frac;      /* fraction of standing separator walls removed */
  int32_t key_door;      /* 1: locked door + key per episode */
  int32_t goal_sprite;   /* 1: goal drawn as a billboard */
  int32_t max_decor;     /* 0..2 decorative billboards per episode */
  int32_t obs_h, obs_w;  /* frame size */
  double fov_deg;        /* horizontal field of view */
  int32_t n_actions;     /* 4 or 6 */
  int32_t episode_cap;   /* truncation length */
  double move, turn, pickup_radius, r_goal, r_key;
  int32_t shade_levels;  /* S: distance-shading levels, 0 = off */
  double shade_dist;     /* D: distance at which the last level starts */
  const char* ascii_map; /* NULL: generated maze; else an ASCII map (Table 2 symbols) */
} orc_cfg;

/* Per-environment state.  Positions in tile units, heading in radians from +x
 * toward +y (y grows "south"). */
typedef struct {
  double x, y, theta;
  int32_t t, episode;
  int32_t goal, door, key;     /* tile ids y*N+x, -1 when absent */
  int32_t key_taken, door_open;
  int32_t n_decor;
  int32_t decor[ORC_MAX_DECOR];
  /* ASCII maps: tiles of the red, blue and yellow keys (-1 absent), the keys
   * taken (bit c), and the doors open (bit = door index) */
  int32_t akey[3];
  int32_t akey_taken;
  int32_t doors_open;
} orc_state;

/* Tile bytes of a grid.  0 floor; low nibble 1 = default wall ('#', colour
 * palette[id mod K]); 2..10 = coloured wall '1'..'9'; bit 7 = door, with its
 * type in bits 4..6 (ORC_DOOR_*) and its index (0..15) in bits 0..3.  On floor
 * tiles bit 5 marks a spawn candidate ('S') and bit 6 a goal candidate ('G'). */
#define ORC_TILE_DOOR   0x80
#define ORC_TILE_SPAWN  0x20
#define ORC_TILE_GOAL   0x40
#define ORC_DOOR_RED_LOCKED      0
#define ORC_DOOR_BLUE_LOCKED     1
#define ORC_DOOR_YELLOW_LOCKED   2
#define ORC_DOOR_BLUE_UNLOCKED   3
#define ORC_DOOR_YELLOW_UNLOCKED 4
#define ORC_MAX_DOORS 16

/* Step event bits (identical meaning on every implementation of the rules). */
#define ORC_EV_BLOCKED_X 0x01
#define ORC_EV_BLOCKED_Y 0x02
#define ORC_EV_KEY       0x04
#define ORC_EV_GOAL      0x08
#define ORC_EV_TRUNC     0x10
#define ORC_EV_INVALID   0x20
#define ORC_EV_RESET     0x40
#define ORC_EV_DOOR      0x80   /* a door opened (bumped, or unlocked by a key) */

/* Step decision flags: the outcome sits within 1e-5 of a decision boundary. */
#define ORC_SF_MOVE  0x01   /* S1: collision boundary */
#define ORC_SF_KEY   0x02   /* S2: pickup radius */
#define ORC_SF_GOAL  0x04   /* S3: goal-cell boundary */

/* Column flags. */
#define ORC_CF_DDA    0x01  /* F1: near-tie between x and y crossings next to a blocker */
#define ORC_CF_SPAN   0x02  /* F2: wall span boundary within the window of a pixel centre */
#define ORC_CF_SPRITE 0x04  /* F3: a sprite comparison within its window */
#define ORC_CF_MULTI  0x08  /* more than one F1 tie on the walk */
#define ORC_CF_SHADE  0x10  /* F4: t* S / D within the window of a shading level boundary */

/* ---- random numbers ---------------------------------------------------- */
uint64_t orc_rng_next(uint64_t* s);                 /* SplitMix64 step */
uint64_t orc_mix64(uint64_t v);                     /* SplitMix64 finaliser of v + golden gamma */
uint32_t orc_rng_range(uint64_t* s, uint32_t n);    /* uniform draw in [0, n) */

/* ---- layout ----------------------------------------------------------- */
/* Writes the N*N tile grid (0 floor, 1 wall) for `seed`.  Returns the number
 * of separator walls removed for loops, or -1 on bad arguments. */
int32_t orc_maze(uint64_t seed, int32_t N, double loop_frac, uint8_t* grid);

/* Parses an ASCII map (Table 2 symbols, rows separated by '\n') into the N*N
 * grid (tile bytes above); keys3 receives the red, blue and yellow key tiles
 * (-1 absent).  Returns the number of doors or a negative error. */
int32_t orc_ascii(const char* text, int32_t N, uint8_t* grid, int32_t* keys3);

/* ---- episodes ---------------------------------------------------------- */
int32_t orc_reset(const uint8_t* grid, const orc_cfg* cfg, uint64_t seed,
                  int32_t episode, orc_state* out);

/* One transition from `in` under `action`.  On done the returned state is the
 * first state of the next episode.  Returns 0 or -1 on bad arguments. */
int32_t orc_step(const uint8_t* grid, const orc_cfg* cfg, uint64_t seed,
                 const orc_state* in, int32_t action, orc_state* out,
                 double* reward, int32_t* done, int32_t* events, int32_t* sflags);

/* Same transition; the step flags use `window` instead of 1e-5 (for comparing
 * trajectories whose positions have drifted apart by rounding). */
int32_t orc_step_w(const uint8_t* grid, const orc_cfg* cfg, uint64_t seed,
                   const orc_state* in, int32_t action, orc_state* out,
                   double* reward, int32_t* done, int32_t* events, int32_t* sflags,
                   double window);

/* ---- render ------------------------------------------------------------ */
/* Renders `st` into obs[H][W][3].  Per column: hit tile id, side (0: x-face,
 * 1: y-face), perpendicular distance, flags, and the alternative (hit, side,
 * t) obtained by taking the other branch at the first flagged DDA tie
 * (alt_hit = -1 when there is none).  Any per-column pointer may be NULL. */
int32_t orc_render(const uint8_t* grid, const orc_cfg* cfg, const orc_state* st,
                   uint8_t* obs, int32_t* hit, int32_t* side, double* tstar,
                   int32_t* cflags, int32_t* alt_hit, int32_t* alt_side, double* alt_t);

/* The same render with the acceptance data of a frame whose decisions sit
 * inside their windows (several results are then correct, Sec. 2.1 DDA):
 *   branch 0: the frame of orc_render; branch 1: every column with a flagged
 *     DDA tie takes the other side of its first tie (the column's second valid
 *     result: hit, side and t* of that walk, sprites z-tested against that t*);
 *     the per-column outputs then describe that walk (alt_* still the walk
 *     not taken by branch 0).
 *   tie (nullable) [H][W]: 1 on every pixel whose value is decided by a
 *     comparison inside its window on this frame: the row pair of a tied span
 *     edge (F2), every wall row of a column whose shading level is tied (F4),
 *     every row of a billboard whose horizontal edge, z-test or near clip is
 *     tied on that column, or whose depth ties another's, and the row pair of
 *     its tied vertical edge (F3).  Every other pixel has one correct value.
 * Returns 0, or -1 on bad arguments. */
int32_t orc_render_ex(const uint8_t* grid, const orc_cfg* cfg, const orc_state* st, int32_t branch,
                      uint8_t* obs, int32_t* hit, int32_t* side, double* tstar, int32_t* cflags,
                      int32_t* alt_hit, int32_t* alt_side, double* alt_t, uint8_t* tie);

/* Single-ray query used by the closed-form tests: casts from (x, y) along
 * (rx, ry) and reports the first blocking tile.  Returns the hit tile id. */
int32_t orc_cast(const uint8_t* grid, int32_t N, int32_t door, int32_t door_open,
                 double x, double y, double rx, double ry,
                 int32_t* side, double* tstar, int32_t* flags);

/* ---- training-buffer formats ------------------------------------------- */
/* The frames a recurrent-PPO learner consumes (the paper trains on 64x64
 * frames with 128-step rollouts and the previous action fed to the policy):
 * layout 0 = NHWC (obs[H][W][3]), 1 = NCHW (obs[3][H][W]); dtype 0 = the
 * byte itself, 1 = bfloat16, 2 = float32, where the floating types hold the
 * byte divided by 255 rounded to nearest (ties to even) in that type. */
#define ORC_OBS_NHWC 0
#define ORC_OBS_NCHW 1
#define ORC_OBS_U8   0
#define ORC_OBS_BF16 1
#define ORC_OBS_F32  2
float orc_norm_f32(int32_t b);     /* b / 255 rounded to float32 */
uint16_t orc_norm_bf16(int32_t b); /* b / 255 rounded to bfloat16 (bit pattern) */
/* Converts one rendered frame hwc[H][W][3] into `out` in the given format;
 * returns the bytes written or -1 on bad arguments. */
int64_t orc_format_frame(const uint8_t* hwc, int32_t H, int32_t W, int32_t layout,
                         int32_t dtype, void* out);
/* The previous action stored beside the frame a step returns: the action
 * taken, or n_actions ("none") when that frame starts an episode or the
 * action was not a valid one. */
int32_t orc_prev_action(const orc_cfg* cfg, int32_t action, int32_t done);

/* Runs `n_steps` steps of `n_envs` environments, each from episode 0, with
 * actions[t*n_envs+i], rendering every frame into a scratch buffer.  This is
 * the timed CPU baseline; returns the number of env-steps done.  counts
 * (nullable) [4] receives the columns rendered, the columns flagged (any of
 * F1-F4), the F1 columns and the steps flagged (S1-S3). */
int64_t orc_rollout(const orc_cfg* cfg, int32_t n_envs, const uint64_t* seeds,
                    int32_t n_steps, const uint8_t* actions, uint8_t* last_obs,
                    int64_t* counts);

#ifdef __cplusplus
}
#endif
#endif
