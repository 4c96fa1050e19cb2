/*
 * jx.h -- C-ABI of libjx: batched first-person grid-world environments with a
 * raycast renderer, running as hand-written HIP kernels on one AMD Instinct
 * MI355X (gfx950).
 *
 * The method (JAXenstein, Tao & Konidaris): every environment is a partially
 * observable first-person task on a tile map with discrete actions and pixel
 * observations (abstract, Sec. 1; partial observability, Sec. 1).  Each frame is drawn by casting one
 * ray per image column to its first wall, found by DDA marching along tile
 * boundaries (Sec. 2.1), over a tile-map world (Sec. 2.2, Sec. 3.2, Table 2);
 * objects are fixed billboard sprites (Fig. 1).  Frames are rendered natively
 * at the training resolution (Sec. 3.1, App. A.1).  Environments are stepped in
 * batches (Sec. 1, Sec. 3.1); here a batch is one kernel launch.
 *
 * Conventions used by every entry point
 *   - All functions returning jx_status return JX_OK (0) or a negative code;
 *     jx_last_error() then holds a message (thread-local).
 *   - "_dev" pointers are device (HBM) addresses on the context's device, owned
 *     by the caller; "_host" pointers are host memory owned by the caller.
 *   - Step, render and rollout are asynchronous on the context's stream and
 *     return after enqueueing; device faults surface as JX_EDEVICE on a later
 *     call or on jx_sync().  A context serves one stream and is not thread-safe.
 *   - Observations are RGB, row 0 at the top, by default uint8 row-major
 *     [row][col][channel]; jx_env_cfg.obs_layout / obs_dtype select the other
 *     training-buffer formats (JX_OBS_*).  With one configuration for all envs
 *     the batch is [n][frame]; with several configurations env i starts at byte
 *     offset jx_obs_offsets()[i].  Observation pointers and strides are in
 *     bytes whatever the element type.
 *   - Reward is float32 per env, done is uint8 per env; both belong to the
 *     transition.  When done = 1 the env has been reset inside the step and its
 *     observation is the first frame of the next episode.
 */
#ifndef JX_H
#define JX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JX_ABI_VERSION 5

typedef int32_t jx_status;
#define JX_OK 0
#define JX_EINVAL (-1)   /* bad argument */
#define JX_ENOMEM (-2)   /* workspace or budget too small */
#define JX_EDEVICE (-3)  /* HIP runtime or device error */
#define JX_ESTATE (-4)   /* call not valid in the current state (e.g. step before reset) */
#define JX_EBUSY (-5)    /* serving: not admitted yet / result not ready */

/* Per-environment configuration.  Limits: side 5..64 (tile-grid side N),
 * n_colors 1..8, loop_frac 0..1, max_decor 0..2, obs_h even and 2..128,
 * obs_w a multiple of 4 in 4..128, n_actions 4 or 6, episode_cap >= 1,
 * shade_levels 0..16 (shade_dist > 0 when shading is on).
 * Values used by the workloads: fov 60, move 0.1, turn pi/16, pickup 0.3. */
typedef struct {
  int32_t side;          /* N: the map is N x N tiles, border tiles are walls */
  int32_t n_colors;      /* K: wall colour = palette[tile id mod K] */
  float loop_frac;       /* fraction of standing maze separator walls removed */
  int32_t key_door;      /* 1: a locked door and its key are placed per episode */
  int32_t goal_sprite;   /* 1: the goal is drawn as a billboard sprite */
  int32_t max_decor;     /* 0..2 decorative sprites per episode */
  int32_t obs_h, obs_w;  /* frame height and width in pixels */
  float fov_deg;         /* horizontal field of view */
  int32_t n_actions;     /* 4: fwd, back, turn-L, turn-R; 6: fwd, back, strafe-L, strafe-R, turn-L, turn-R */
  int32_t episode_cap;   /* truncation length in steps */
  float move;            /* distance per move action, tiles */
  float turn;            /* radians per turn action */
  float pickup_radius;   /* key pickup radius, tiles */
  float r_goal, r_key;   /* rewards */
  /* Distance shading of walls (the paper's ray-casting section allows a shading
   * colour by the hit distance; the rule is this library's reading).  With
   * S = shade_levels > 0 a column hit at perpendicular distance t* is drawn at
   * level l = min(floor(t* * S / shade_dist), S - 1): each channel of its wall
   * colour (after the side darkening) becomes floor(c * (S - l) / S).
   * Sprites, ceiling and floor are not shaded.  0 = off. */
  int32_t shade_levels;
  float shade_dist;
  /* Layout source: NULL = a seeded maze (the env seed; loop_frac applies).
   * Otherwise a NUL-terminated ASCII map with the paper's Table 2 symbols, rows
   * separated by '\n', placed at the top-left of the side x side grid (tiles it
   * does not cover are walls): '#' wall (colour palette[id mod K]), '1'..'9'
   * coloured walls, '.' or ' ' floor, 'S' spawn candidate, 'G' goal candidate,
   * 'r' 'b' 'y' red, blue, yellow key (at most one per colour), '"' and '\'
   * blue and yellow unlocked doors, 'R' 'B' 'Y' red, blue and yellow locked
   * doors (at most 16 doors).  Border tiles must be walls.  Rules (the
   * library's reading): each episode draws the spawn among the 'S' tiles (every
   * floor tile if none) and the goal among the 'G' tiles (the tile farthest from
   * the spawn, doors passable, if none); an unlocked door opens when the agent
   * walks into it (that move is refused); picking up a key (reward r_key) opens
   * every locked door of its colour; keys are drawn as billboards.  key_door
   * and max_decor must be 0.  The text is read by the call that takes the
   * configuration and need not outlive it. */
  const char* ascii_map;
  /* Frame format, for writing frames straight into a learner's rollout buffer
   * (the paper trains a recurrent PPO agent on 64x64 frames over 128-step
   * rollouts, Sec. 3.1 and the training hyperparameters of the appendix).
   * obs_layout: JX_OBS_NHWC ([H][W][3]) or JX_OBS_NCHW ([3][H][W]).
   * obs_dtype: JX_OBS_U8 (the byte), JX_OBS_BF16 or JX_OBS_F32 (the byte / 255
   * rounded to nearest-even in that type; the paper leaves normalisation open,
   * this is the library's reading).  Every configuration of one context must
   * use the same format.  Frame bytes = H * W * 3 * element size.  The serving
   * API takes the default format (NHWC, U8) only. */
  int32_t obs_layout;
  int32_t obs_dtype;
} jx_env_cfg;

#define JX_OBS_NHWC 0
#define JX_OBS_NCHW 1
#define JX_OBS_U8 0
#define JX_OBS_BF16 1
#define JX_OBS_F32 2

typedef struct jx_ctx jx_ctx;

/* Launch mapping (results are bit-identical under every mapping). */
#define JX_FORM_PLAIN 0       /* one wave per env, one workgroup slot per env */
#define JX_FORM_PERSISTENT 1  /* persistent waves pull envs from device work queues */
#define JX_FORM_PIPELINE 2    /* persistent producer/writer wave pairs, double-buffered */
typedef struct {
  int32_t form;            /* JX_FORM_PLAIN, JX_FORM_PERSISTENT or JX_FORM_PIPELINE */
  int32_t waves_per_group; /* waves (plain, persistent: 1, 2, 4, 8) or wave pairs
                              (pipelined: 1, 2, 4) per workgroup */
  int32_t groups_per_cu;   /* persistent and pipelined forms: workgroups per compute unit, 1..16 */
  int32_t store_mode;      /* 0: ordinary stores, 1: non-temporal observation stores */
  int32_t waves_per_env;   /* plain form: 1, 2 or 4 waves share one env (at most
                              waves_per_group; other forms: 1).  Each runs the same
                              step and cast and writes its share of the frame's
                              rows, so small batches of large frames use more of
                              the chip; results do not change. */
} jx_launch;

/* Per-column record of the last render (tests and tools).  hit = tile id of the
 * first blocking tile, side 0 = x-face (vertical grid line), 1 = y-face,
 * t = perpendicular distance, cell = 1 wall, 2 locked door. */
typedef struct {
  int32_t hit;
  int32_t side;
  float t;
  int32_t cell;
} jx_col_debug;

/* One named array of the state image returned by jx_get_state(). */
typedef struct {
  char name[24];
  int64_t offset;   /* byte offset in the state image */
  int64_t bytes;    /* size in bytes */
  int32_t elem;     /* element size in bytes */
  int32_t count;    /* number of elements */
} jx_field;

/* ABI version of the library (JX_ABI_VERSION it was built with) and the
 * calling thread's last error message (library plumbing; not in the paper). */
int32_t jx_abi_version(void);
const char* jx_last_error(void);

/* Bytes of device workspace needed for n_envs environments (the library's
 * memory plan; not in the paper).  cfg_index[i]
 * selects cfgs[cfg_index[i]]; cfg_index may be NULL when n_cfgs == 1.
 * Returns 0 on invalid arguments. */
size_t jx_workspace_bytes(int32_t n_envs, const jx_env_cfg* cfgs, int32_t n_cfgs,
                          const int32_t* cfg_index);

/* Creates a context (library plumbing; not in the paper) on `device`,
 * enqueueing on `hip_stream` (a hipStream_t;
 * NULL = the default stream).  `workspace_dev` is caller-owned device memory of
 * ws_bytes bytes, 256-byte aligned; it holds all environment state (SoA), maps
 * and tables and must outlive the context. */
jx_status jx_create(jx_ctx** out, int32_t device, void* hip_stream, void* workspace_dev,
                    size_t ws_bytes);
void jx_destroy(jx_ctx* ctx);

/* Starts episode 0 of every env (the paper's tasks: tile-map worlds of
 * Sec. 2.2 and Sec. 3.2, the navigation and key-door tasks of Table 1, the
 * ASCII symbols of Table 2; the per-episode spawn, goal, door and key draws
 * are this library's reading).  Generates each env's maze from seeds_host[i]
 * on the host, uploads maps and tables, and runs the episode reset on the
 * device.  cfgs_host[n_cfgs] are the configurations, cfg_index_host[n] (NULL
 * when n_cfgs == 1) picks env i's.  Errors: JX_EINVAL for a bad configuration
 * or ASCII map (message in jx_last_error), JX_ENOMEM when the context's
 * workspace is smaller than jx_workspace_bytes(), JX_EDEVICE on a HIP error.
 * When obs_dev is not NULL the first frames are rendered into it.
 * n_envs may be 0 (every later call is then a no-op).  Synchronous: returns
 * after the reset kernel has finished. */
jx_status jx_reset(jx_ctx* ctx, int32_t n_envs, const uint64_t* seeds_host,
                   const jx_env_cfg* cfgs_host, int32_t n_cfgs, const int32_t* cfg_index_host,
                   uint8_t* obs_dev);

/* Sizes of the batch (library plumbing; not in the paper). */
int32_t jx_num_envs(const jx_ctx* ctx);
/* Total observation bytes of one step (sum over envs). */
int64_t jx_obs_bytes(const jx_ctx* ctx);
/* offsets_host[0..n]: byte offset of env i's frame in a step's observation
 * buffer; offsets_host[n] = jx_obs_bytes(). */
jx_status jx_obs_offsets(const jx_ctx* ctx, int64_t* offsets_host);

/* One batched transition and render of every env: a first-person task with
 * discrete actions and pixel observations (Sec. 1, Sec. 3.2), stepped as one
 * batch (the paper vectorises envs with vmap, Sec. 1, Sec. 3.1); each frame is
 * drawn by one DDA ray per image column (Sec. 2.1) at the training resolution
 * (Sec. 3.1, App. A.1).  The action rules, rewards and auto-reset are this
 * library's readings.  actions_dev[n] uint8 (values >= n_actions
 * are counted no-ops); obs_dev receives jx_obs_bytes() bytes (4-byte aligned;
 * 16-byte aligned for the floating formats); reward_dev[n] float32; done_dev[n]
 * uint8.  prev_action_dev (nullable) [n] uint8 receives the previous action to
 * feed the policy beside the returned frame (the paper's agent concatenates
 * it): the action taken, or n_actions ("none") when the frame starts a new
 * episode (done = 1) or the action was out of range.  A caller may capture the
 * call into a graph of its own under any launch mapping: every launch leaves
 * the work-queue counters it used at zero, so replays find them clean. */
jx_status jx_step(jx_ctx* ctx, const uint8_t* actions_dev, uint8_t* obs_dev, float* reward_dev,
                  uint8_t* done_dev, uint8_t* prev_action_dev);

/* T consecutive steps (the paper's learner collects 128-step rollouts of
 * vmapped envs, Sec. 3.1, App. A.2 and the PPO hyperparameter table; graph
 * capture and the fused launch are this library's).  actions_dev[T][n]; step t
 * writes its frames at
 * obs_dev + t*obs_stride (obs_stride >= jx_obs_bytes(), or 0 to write every
 * step into the same frame buffer), rewards at reward_dev + t*n, dones at
 * done_dev + t*n and, when prev_action_dev is not NULL, previous actions (as in
 * jx_step) at prev_action_dev + t*n.  flags & JX_ROLLOUT_GRAPH: the T
 * launches are captured once per (T, launch mapping) into a hipGraph and
 * replayed with one graph launch;
 * the buffers of each call reach the captured kernels through a descriptor in
 * the workspace, so a captured graph serves any buffers.  Without the flag the
 * T launches are enqueued one by one. */
#define JX_ROLLOUT_GRAPH 1
/* flags & JX_ROLLOUT_FUSED: one launch runs all T steps; each wave keeps its
 * env's state on chip between steps and writes it back after the last step.
 * Outputs (frames, rewards, dones, final state) equal T single-step launches
 * bit for bit.  Takes precedence over JX_ROLLOUT_GRAPH.  Under the plain
 * mapping, waves take envs by a static stride (waves_per_group waves per
 * workgroup, waves_per_env of them sharing each env); under the persistent
 * mapping, groups_per_cu workgroups per compute unit claim envs one at a time
 * from device work queues, costliest
 * first (uneven shapes); the pipelined mapping and the training-buffer formats
 * run the static stride with 4 waves per workgroup (those formats also run
 * every per-step launch in the plain form). */
#define JX_ROLLOUT_FUSED 2
jx_status jx_rollout(jx_ctx* ctx, int32_t T, const uint8_t* actions_dev, uint8_t* obs_dev,
                     int64_t obs_stride, float* reward_dev, uint8_t* done_dev,
                     uint8_t* prev_action_dev, int32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same T
 * steps as jx_rollout(ctx, T, ..., flags), with the same arguments, buffers
 * and results bit for bit, under the context's launch mapping.  The persistent
 * form's work-queue counters live in a static device array of the library
 * (16 KiB, one copy per device, resolved by jx_create and held until the
 * process ends) instead of the context's workspace; no input size can exceed
 * it, since a launch uses at most 32 queues whatever the batch.  The call
 * allocates nothing (no hipMalloc, hipFree, graph or host buffer) and only
 * enqueues kernels on the context's stream: a kernel first clears the counters
 * the previous call left in the array, so a captured call replays correctly.
 * flags: 0 (T launches) or JX_ROLLOUT_FUSED (one launch); JX_ROLLOUT_GRAPH is
 * rejected with JX_EINVAL (instantiating a graph allocates).  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * streams, threads or contexts) race and must be serialised by the caller.
 * JX_EDEVICE if the array could not be resolved when the context was created. */
jx_status jx_rollout_noalloc(jx_ctx* ctx, int32_t T, const uint8_t* actions_dev, uint8_t* obs_dev,
                             int64_t obs_stride, float* reward_dev, uint8_t* done_dev,
                             uint8_t* prev_action_dev, int32_t flags);

/* Renders the current state without stepping: one ray per image column to
 * the first blocking tile by DDA over tile boundaries, perpendicular distance,
 * column fill by hit tile and side (Sec. 2.1), billboard sprites (Fig. 1
 * caption).  obs_dev may be NULL;
 * column_debug_dev (nullable) receives jx_col_debug[n][max obs_w]. */
jx_status jx_render(jx_ctx* ctx, uint8_t* obs_dev, jx_col_debug* column_debug_dev);

/* State image (checkpoint format of this library; not in the paper): every
 * per-env array, the maps and the configuration table, as
 * one host buffer of jx_state_bytes() bytes.  jx_set_state() accepts only an
 * image taken from a context reset with the same envs and configurations.
 * Both synchronise the context's stream. */
size_t jx_state_bytes(const jx_ctx* ctx);
jx_status jx_state_layout(const jx_ctx* ctx, jx_field* fields, int32_t cap, int32_t* n_fields);
jx_status jx_get_state(const jx_ctx* ctx, void* host_buf, size_t bytes);
jx_status jx_set_state(jx_ctx* ctx, const void* host_buf, size_t bytes);

/* Launch mapping of later steps (this library's batching forms; results do
 * not depend on it).  JX_EINVAL for a mapping outside the limits above. */
jx_status jx_set_launch(jx_ctx* ctx, const jx_launch* launch);
jx_status jx_get_launch(const jx_ctx* ctx, jx_launch* launch);

/* Autotuner (this library's; the paper's batching is jit + vmap, Sec. 1,
 * Sec. 3.1): times every candidate mapping over `iters` steps driven by
 * actions_dev[iters][n], writing frames into obs_scratch_dev (jx_obs_bytes()
 * bytes), checks that each candidate's frames, rewards, dones and state are
 * bit-identical to the default mapping's, and selects the fastest.  The env
 * state is restored afterwards.  cache_path (nullable) is a text file of
 * previous choices keyed by device and workload shape.  *chosen (nullable)
 * receives the pick.  Synchronous. */
jx_status jx_autotune(jx_ctx* ctx, const uint8_t* actions_dev, int32_t iters,
                      uint8_t* obs_scratch_dev, const char* cache_path, jx_launch* chosen);

/* Waits for the context's stream; JX_EDEVICE reports a device fault of any
 * earlier call (library plumbing; not in the paper). */
jx_status jx_sync(jx_ctx* ctx);

/* Host only (no device): the N x N tile grid (0 floor, 1 wall; tile bytes of
 * an ASCII map) that jx_reset builds for `seed` under `cfg` (the tile-map
 * worlds of Sec. 2.2 and Table 2; the seeded maze is this library's reading). */
jx_status jx_make_layout(uint64_t seed, const jx_env_cfg* cfg, uint8_t* grid_host);

/* ---------------------------------------------------------------------------
 * Serving (not in the paper: this library's serving form of the same step and
 * render; the paper measures steps/s and training throughput only, Sec. 3.1).
 * A request loop holding many clients' environments resident on one
 * device.  Clients open env batches of any size and configuration; requests
 * (one step of one client) that are ready are coalesced into shared persistent
 * launches spread over n_streams streams, so that requests arriving while
 * others run are admitted and overlap on the device (continuous batching).
 * Clients are admitted while their device memory fits the HBM budget; others
 * wait in FIFO order.  All functions are thread-safe.  For latency two of the
 * server's threads poll rather than sleep: the scheduler for up to 1 ms when
 * the device falls idle, the completion thread every 2 us while launches are
 * in flight, so a busy server keeps up to two host cores busy.
 * ------------------------------------------------------------------------- */
typedef struct jx_server jx_server;

#define JX_SERVE_COALESCE 0  /* mode: coalesce ready requests into shared launches */
#define JX_SERVE_PLAIN 1     /* mode: one launch per request, FIFO, one stream */

/* hbm_budget_bytes bounds the device memory of admitted clients' state and
 * maps.  Testing hook: when the environment variable JX_SERVER_FAIL_LAUNCH
 * holds an integer k >= 0 at creation, the server's k-th launch (0-based, in
 * issue order) is treated as failed without any HIP call being made for it, so
 * the failure path below can be exercised with every kernel exiting normally.
 * Each stream also holds a 128 MiB device staging buffer for its launches'
 * descriptors and actions, and the server a pinned host arena of
 * min(budget, 2 GiB) from which they are copied and into which the serving
 * kernels write host clients' results directly; one step of a client must
 * fit both.
 * n_streams 1..8.  max_batch_envs bounds envs per launch (0 = no bound). */
jx_status jx_server_create(jx_server** out, int32_t device, size_t hbm_budget_bytes,
                           int32_t n_streams, int32_t mode, int32_t max_batch_envs);
void jx_server_destroy(jx_server* srv);

/* Opens a client of n_envs envs (one configuration for all; the default frame
 * format only).  Returns JX_OK when admitted, JX_EBUSY when queued for
 * admission (the id is valid either way; requests submitted meanwhile wait),
 * JX_ENOMEM when the client's state alone exceeds the budget or one step of it
 * does not fit the launch staging, JX_EINVAL for a bad configuration. */
jx_status jx_server_open(jx_server* srv, int32_t n_envs, const uint64_t* seeds_host,
                         const jx_env_cfg* cfg, int32_t* client);

/* Opens a client whose results stay on the device (the step's consumer, such
 * as a learner on the same GPU, reads them there; nothing is copied to the
 * host): obs_dev [slots][n_envs][H][W][3] uint8, reward_dev [slots][n_envs]
 * float32 and done_dev [slots][n_envs] uint8 are caller-owned device memory on
 * the server's device (obs and reward 4-byte aligned) that must stay valid
 * until the client's last request has been collected.  The client's requests
 * run in submission order and the k-th of them (0-based) writes slot
 * k mod slots, so a caller that keeps at most `slots` requests uncollected
 * never has a slot overwritten before it has read it.  jx_server_wait on such a
 * request takes no host buffers (JX_EINVAL otherwise).  Admission and errors as
 * jx_server_open; JX_EINVAL for null rings or slots < 1. */
jx_status jx_server_open_dev(jx_server* srv, int32_t n_envs, const uint64_t* seeds_host, const jx_env_cfg* cfg,
                             uint8_t* obs_dev, float* reward_dev, uint8_t* done_dev, int32_t slots,
                             int32_t* client);

/* Queues one step of `client` with actions_host[n_envs] (copied).  *ticket
 * identifies the request.  JX_EDEVICE if the client has failed (a launch
 * holding one of its steps failed). */
jx_status jx_server_submit(jx_server* srv, int32_t client, const uint8_t* actions_host,
                           uint64_t* ticket);

/* Waits for a request (timeout_s < 0: forever; 0: poll, JX_EBUSY if not done)
 * and copies its frames (n_envs * H * W * 3 bytes), rewards and dones into
 * host buffers (each nullable; all NULL for a client opened with
 * jx_server_open_dev).  latency_s (nullable) = submit-to-complete seconds.
 * A failed launch fails its own requests only: they return JX_EDEVICE, their
 * clients fail (their queued and later requests return JX_EDEVICE too, since
 * their state is unknown) and every other client is served on. */
jx_status jx_server_wait(jx_server* srv, uint64_t ticket, double timeout_s, uint8_t* obs_host,
                         float* reward_host, uint8_t* done_host, double* latency_s);

/* Completion queue: waits (timeout_s < 0: forever; 0: poll, JX_EBUSY if none)
 * for a completed request not yet collected and returns its ticket and client
 * (client nullable), in completion order, each once.  It does not collect the
 * request: pass the ticket to jx_server_wait.  A launch's results occupy the
 * server's pinned staging arena (min(budget, 2 GiB)) until every request of
 * that launch is collected, and a launch is issued only when its results fit,
 * so callers should collect what completes. */
jx_status jx_server_wait_any(jx_server* srv, double timeout_s, uint64_t* ticket, int32_t* client);

/* Releases the client once its queued requests have completed; a client still
 * waiting for admission is admitted first if it has queued requests, else it
 * leaves the admission queue at once.  Results of its requests stay
 * collectable with jx_server_wait after the close.  No request may be
 * submitted to a closed client. */
jx_status jx_server_close(jx_server* srv, int32_t client);

/* Counters: launches, requests, envs stepped, admission waits, bytes in use,
 * failed launches. */
typedef struct {
  int64_t launches;
  int64_t requests;
  int64_t env_steps;
  int64_t admission_waits;
  int64_t bytes_in_use;
  int64_t clients_active;
  int64_t clients_pending;
  int64_t failed_launches;
} jx_server_stats;
jx_status jx_server_get_stats(jx_server* srv, jx_server_stats* out);

/* Load generator (native threads, so the caller's interpreter does not limit
 * the offered load): replays an arrival trace against srv.  Request k is
 * submitted t_arrival_s[k] seconds after the call starts (the trace must be in
 * arrival order) for client[k] with actions_host[k] (that client's n actions);
 * if close_after is not NULL and close_after[k] != 0 the client is closed right
 * after that submit.  n_collectors threads (1..64) take completed requests in
 * completion order (jx_server_wait_any) and collect them (jx_server_wait) into
 * buffers of their own.  latency_s[k] receives request k's submit-to-ready
 * latency; submitted_s (nullable) the time the submits took; wall_s (nullable)
 * the time until the last result was collected.  Every client of the trace must
 * be open (admitted or queued), and no other requests may be submitted to srv
 * while the replay runs.  Returns JX_EDEVICE if a request fails, a request not
 * of the trace completes, or the replay exceeds timeout_s (> 0). */
jx_status jx_server_replay(jx_server* srv, int32_t n, const double* t_arrival_s, const int32_t* client,
                           const uint8_t* const* actions_host, const uint8_t* close_after,
                           int32_t n_collectors, double timeout_s, double* latency_s,
                           double* submitted_s, double* wall_s);

#ifdef __cplusplus
}
#endif
#endif /* JX_H */
