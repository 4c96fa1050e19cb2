// jx_internal.h -- structures shared by the host runtime and the device kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace jx {

constexpr int kMaxSide = 64;     // one map row fits a 64-bit mask; one row per lane in BFS
constexpr int kMaxW = 128;       // column records per wave in LDS
constexpr int kMaxH = 128;
constexpr int kMaxDecor = 2;
constexpr int kMaxShadeLevels = 16;
// Frame formats: obs_layout * 3 + obs_dtype (layout 0 NHWC, 1 NCHW; dtype 0
// byte, 1 bfloat16, 2 float32 of byte / 255).
constexpr int kObsFormats = 6;
constexpr int obs_elem_bytes(int fmt) { return fmt % 3 == 0 ? 1 : (fmt % 3 == 1 ? 2 : 4); }
constexpr uint32_t kStateMagic = 0x4A585331u;  // "JXS1"

// Event bits written per env and step.
constexpr uint32_t EV_BLOCKED_X = 0x01, EV_BLOCKED_Y = 0x02, EV_KEY = 0x04, EV_GOAL = 0x08,
                   EV_TRUNC = 0x10, EV_INVALID = 0x20, EV_RESET = 0x40, EV_DOOR = 0x80;
// Per-env flag bits.
constexpr uint32_t FL_KEY = 0x01, FL_DOOR_OPEN = 0x02;
// ASCII maps: key c (0 red, 1 blue, 2 yellow) taken
constexpr uint32_t FL_AKEY0 = 0x04;

enum Mode : int32_t { MODE_STEP = 0, MODE_RESET = 1, MODE_RENDER = 2 };

// Per-configuration constants, derived on the host from jx_env_cfg.
struct DevCfg {
  int32_t side, n_colors, key_door, goal_sprite;
  int32_t max_decor, obs_h, obs_w, n_actions;
  int32_t cap, shade_levels;
  float shade_scale;   // shade_levels / shade_dist, rounded to float
  uint32_t shade_mul;  // ceil(2^16 / shade_levels): x / S == (x * shade_mul) >> 16 for x < 4096
  float move, turn, pr2, r_goal;
  float r_key, tanH, inv_tanH, inv_w;  // 1/tanH and 1/obs_w, rounded to float
  int32_t ascii;  // 1: the layout is an ASCII map (doors, keys, candidates)
  // tan(fov/2) / obs_w in double, split into two floats (hi + lo, 48 bits):
  // column c's ray is dir + (2c + 1 - obs_w) * ray_q * right
  float ray_q_hi, ray_q_lo;
  int32_t pad3;
};
static_assert(sizeof(DevCfg) == 96, "DevCfg layout");

// First 256 bytes of every workspace.
struct WsHeader {
  uint32_t queue;      // persistent form: next work item
  uint32_t exited;     // persistent form: waves that left the queue
  uint32_t magic;
  int32_t n_envs;
  int64_t state_bytes;
  int32_t n_cfgs;
  int32_t pad[57];
};
static_assert(sizeof(WsHeader) == 256, "header size");

// Device-resident I/O of a captured rollout: step t uses act + t*n,
// obs + t*obs_stride, rew + t*n, done + t*n.  Written by a one-thread kernel
// before each graph replay, so one captured graph serves any buffers.
struct RolloutDesc {
  const uint8_t* act;
  uint8_t* obs;
  float* rew;
  uint8_t* done;
  uint8_t* prev;  // nullable: previous actions, prev + t*n
  int64_t obs_stride;
  int32_t n;
  int32_t store_mode;
};

// Device view of one batch of environments (pointers into one workspace).
struct DevState {
  float* x;
  float* y;
  float* th;
  uint32_t* t;
  uint32_t* ep;
  int32_t* goal;
  int32_t* door;
  int32_t* key;
  int32_t* decor;     // [n][2]
  int32_t* akey;      // [n][3] ASCII maps: red, blue, yellow key tiles (-1 absent)
  uint32_t* doors;    // ASCII maps: doors open (bit = door index)
  uint8_t* flags;
  uint8_t* events;
  uint8_t* ndecor;
  uint32_t* invalid;  // counted invalid actions per env
  const uint64_t* seed;
  const int32_t* cfg_idx;
  const uint32_t* map_off;
  const int64_t* obs_off;  // [n+1]
  const int32_t* order;    // persistent work order (costliest first)
  RolloutDesc* rdesc;      // rollout I/O descriptor
  uint32_t* queues;        // persistent form: [4 slots][32 queues][32] counters
  const DevCfg* cfgs;
  const uint8_t* maps;
  WsHeader* hdr;
  int32_t n;
  // One configuration for every env: the kernels take it from here and derive
  // map and frame offsets from the env index (no dependent loads).
  int32_t uniform;
  int32_t any_ascii;  // some configuration is an ASCII map (host-set; picks the kernel variant)
  int32_t obs_fmt;    // frame format, obs_layout * 3 + obs_dtype (the same for every env)
  DevCfg ucfg;
  int64_t map_stride;
  int64_t obs_stride;
};

// Per-launch I/O.
struct DevIo {
  const uint8_t* act;
  uint8_t* obs;
  float* rew;
  uint8_t* done;
  uint8_t* prev;      // nullable: previous action per env
  void* dbg;          // jx_col_debug[n][dbg_stride]
  int32_t dbg_stride;
  int32_t mode;
  int32_t store_mode;
  int32_t pad;
};

// Serving: one work item = (batch descriptor index, env).
struct ServeItem {
  int32_t desc;
  int32_t env;
};

// Workspace layout: byte offsets of every array.
struct Layout {
  int64_t hdr, x, y, th, t, ep, goal, door, key, decor, akey, doors, flags, events, ndecor, invalid, seed,
      cfg_idx, map_off, obs_off, order, rdesc, queues, cfgs, maps, total;
};

// Launch entry points implemented in jx_kernels.hip.
struct LaunchCfg {
  int32_t form, waves_per_group, groups_per_cu, store_mode;
  int32_t waves_per_env = 1;  // plain form: waves sharing one env (1, 2, 4; at most waves_per_group)
};
// Persistent queues: kQueueSlots counter sets of kQueues queues each, one
// 128-byte line per counter.  Launch `seq` uses set seq % kQueueSlots and clears
// set (seq + 1) % kQueueSlots for the launch after it.
constexpr int kQueues = 32, kQueueSlots = 4, kQueueStride = 32;
constexpr int kQueueWords = kQueues * kQueueSlots * kQueueStride;
// Static device scratch of the rollout entry point that allocates nothing: one
// full set of queue counters (16 KiB).  Every batch size fits it: a launch uses
// at most kQueues queues whatever the number of envs.
constexpr int kScratchWords = kQueueWords;
static_assert(kScratchWords * 4 == 16384, "scratch size");

// rd != nullptr: the I/O of step t is taken from the device descriptor rd.
// seq: launch sequence number (persistent form).
int launch_batch(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t,
                 const LaunchCfg& lc, int max_side, int n_cu, uint32_t seq, void* stream);
int launch_clear_queues(uint32_t* queues, void* stream);
// Device address of the static scratch array on `device`, looked up on the
// first call for that device, which must be made with the device current.
// 0 or a hipError_t code.
int scratch_device_address(int device, uint32_t** out);
// One launch for T steps of every env (actions for all steps given up front).
// lc.form 1 (persistent, byte frames): persistent waves claim envs from the
// queue counters of launch `seq`, as launch_batch does; otherwise a static
// stride of lc.waves_per_group-wave workgroups.
int launch_rollout_fused(const DevState& s, const uint8_t* act, uint8_t* obs, int64_t obs_stride,
                         float* rew, uint8_t* dn, uint8_t* prev, int T, const LaunchCfg& lc, int max_side, int n_cu,
                         uint32_t seq, void* stream);
int launch_set_desc(RolloutDesc* rd_dev, const RolloutDesc& value, void* stream);
int launch_serve(const DevState* states_dev, const DevIo* ios_dev, const ServeItem* items_dev,
                 int n_items, uint32_t* queues_dev, uint32_t seq, int waves_per_group,
                 int n_groups, void* stream);
const char* kernel_error_string(int code);

}  // namespace jx
