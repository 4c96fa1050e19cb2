// jx_abi.cpp -- host runtime behind include/jx.h: validation, workspace layout,
// reset (host maze generation + device episode reset), step, hipGraph rollouts,
// state import/export and the launch-mapping autotuner.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <array>
#include <fstream>
#include <map>
#include <numeric>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "jx.h"
#include "jx_common.h"
#include "jx_internal.h"
#include "jx_layout.h"

using namespace jx;

struct jx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  int n = -1;  // -1 until reset
  Layout L{};
  DevState S{};
  std::vector<jx_env_cfg> cfgs;
  std::vector<std::string> ascii_texts;  // copies of the configurations' ASCII maps
  std::vector<int32_t> cfg_idx;
  std::vector<int64_t> obs_off;
  std::vector<DevCfg> dev_cfgs;
  int max_side = 0, max_w = 0;
  int n_cu = 1;
  LaunchCfg launch{0, 1, 4, 0};
  uint32_t seq = 0;  // persistent launches enqueued on this context's stream
  // static scratch of jx_rollout_noalloc on this device (looked up at create)
  uint32_t* scratch = nullptr;
  int scratch_err = 0;
  // captured rollouts, keyed by (T, launch mapping)
  std::map<std::array<int32_t, 6>, hipGraphExec_t> graphs;
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_error(JX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Enqueues one step/render launch.  seq_override >= 0 fixes the persistent
// queue sequence number (graph capture); otherwise the context's counter runs.
static jx_status launch_or_fail(jx_ctx* c, const DevIo& io, hipStream_t st,
                                const RolloutDesc* rd = nullptr, int t = 0,
                                int64_t seq_override = -1) {
  const uint32_t seq = seq_override >= 0 ? (uint32_t)seq_override : c->seq;
  int rc = launch_batch(c->S, io, rd, t, c->launch, c->max_side, c->n_cu, seq, st);
  if (rc == 0 && seq_override < 0 && c->launch.form == JX_FORM_PERSISTENT) c->seq += 1;
  if (rc != 0) return set_error(JX_EDEVICE, std::string("kernel launch: ") + kernel_error_string(rc));
  return JX_OK;
}

static jx_status check_ready(const jx_ctx* c) {
  if (!c) return set_error(JX_EINVAL, "null context");
  if (c->n < 0) return set_error(JX_ESTATE, "context not reset");
  return JX_OK;
}

extern "C" {

int32_t jx_abi_version(void) { return JX_ABI_VERSION; }

const char* jx_last_error(void) { return g_last_error.c_str(); }

size_t jx_workspace_bytes(int32_t n_envs, const jx_env_cfg* cfgs, int32_t n_cfgs,
                          const int32_t* cfg_index) {
  if (n_envs < 0 || !cfgs || n_cfgs < 1 || (n_cfgs > 1 && !cfg_index && n_envs > 0)) return 0;
  int64_t mb = 0;
  for (int i = 0; i < n_envs; ++i) {
    int c = cfg_index ? cfg_index[i] : 0;
    if (c < 0 || c >= n_cfgs) return 0;
    if (cfgs[c].side < 5 || cfgs[c].side > kMaxSide) return 0;
    mb += map_bytes_of(cfgs[c].side);
  }
  return (size_t)make_layout(n_envs, n_cfgs, mb).total;
}

jx_status jx_create(jx_ctx** out, int32_t device, void* hip_stream, void* workspace_dev,
                    size_t ws_bytes) {
  if (!out) return set_error(JX_EINVAL, "out is null");
  *out = nullptr;
  if (!workspace_dev) return set_error(JX_EINVAL, "workspace is null");
  if (((uintptr_t)workspace_dev & 255) != 0) return set_error(JX_EINVAL, "workspace must be 256-byte aligned");
  int n_dev = 0;
  HIPCHK(hipGetDeviceCount(&n_dev));
  if (device < 0 || device >= n_dev) return set_error(JX_EINVAL, "bad device index");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  jx_ctx* c = new jx_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (uint8_t*)workspace_dev;
  c->ws_bytes = ws_bytes;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  // the device is current: resolve this device's copy of the static scratch
  // array once, here, so the entry point that allocates nothing needs no set-up
  c->scratch_err = scratch_device_address(device, &c->scratch);
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return set_error(JX_EDEVICE, "stream creation failed");
  }
  *out = c;
  return JX_OK;
}

void jx_destroy(jx_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  delete c;
}

jx_status jx_reset(jx_ctx* c, int32_t n_envs, const uint64_t* seeds, const jx_env_cfg* cfgs,
                   int32_t n_cfgs, const int32_t* cfg_index, uint8_t* obs_dev) {
  TraceRange range("jx_reset");
  if (!c) return set_error(JX_EINVAL, "null context");
  if (n_envs < 0) return set_error(JX_EINVAL, "n_envs < 0");
  if (!cfgs || n_cfgs < 1) return set_error(JX_EINVAL, "need at least one configuration");
  if (n_cfgs > 1 && !cfg_index && n_envs > 0) return set_error(JX_EINVAL, "cfg_index required when n_cfgs > 1");
  if (n_envs > 0 && !seeds) return set_error(JX_EINVAL, "seeds is null");
  if (obs_dev && ((uintptr_t)obs_dev & 3)) return set_error(JX_EINVAL, "obs must be 4-byte aligned");
  for (int k = 0; k < n_cfgs; ++k) {
    std::string why;
    if (!validate_cfg(cfgs[k], &why)) return set_error(JX_EINVAL, "cfg " + std::to_string(k) + ": " + why);
    if (obs_fmt_of(cfgs[k]) != obs_fmt_of(cfgs[0]))
      return set_error(JX_EINVAL, "every configuration must use the same obs_layout and obs_dtype");
  }
  if (obs_dev && ((uintptr_t)obs_dev & (obs_align(obs_fmt_of(cfgs[0])) - 1)))
    return set_error(JX_EINVAL, "obs must be 16-byte aligned for the floating formats");
  std::vector<uint8_t> img;
  Layout L;
  std::vector<int64_t> oo;
  std::vector<int32_t> idx;
  jx_status st = build_image(n_envs, seeds, cfgs, n_cfgs, cfg_index, &img, &L, &oo, &idx);
  if (st != JX_OK) return st;
  if ((size_t)L.total > c->ws_bytes)
    return set_error(JX_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  HIPCHK(hipSetDevice(c->device));
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  HIPCHK(hipMemcpyAsync(c->ws, img.data(), (size_t)L.total, hipMemcpyHostToDevice, c->stream));
  c->L = L;
  c->n = n_envs;
  c->S = bind_state(c->ws, L, n_envs);
  c->cfgs.assign(cfgs, cfgs + n_cfgs);
  // the caller's map texts need not outlive this call: keep copies
  c->ascii_texts.assign(n_cfgs, std::string());
  for (int k = 0; k < n_cfgs; ++k) {
    if (cfgs[k].ascii_map) {
      c->ascii_texts[k] = cfgs[k].ascii_map;
      c->cfgs[k].ascii_map = c->ascii_texts[k].c_str();
    }
  }
  c->cfg_idx = idx;
  c->obs_off = oo;
  c->dev_cfgs.clear();
  c->max_side = 0;
  c->max_w = 0;
  for (int k = 0; k < n_cfgs; ++k) {
    c->dev_cfgs.push_back(derive_cfg(cfgs[k]));
    c->max_side = std::max(c->max_side, cfgs[k].side);
    c->max_w = std::max(c->max_w, cfgs[k].obs_w);
  }
  set_uniform(&c->S, cfgs, n_cfgs, idx);
  c->S.obs_fmt = obs_fmt_of(cfgs[0]);
  DevIo io{};
  io.obs = obs_dev;
  io.mode = MODE_RESET;
  io.store_mode = 0;
  if (n_envs > 0) {
    LaunchCfg keep = c->launch;
    c->launch = LaunchCfg{0, 1, 1, 0};
    jx_status r = launch_or_fail(c, io, c->stream);
    c->launch = keep;
    if (r != JX_OK) return r;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return JX_OK;
}

int32_t jx_num_envs(const jx_ctx* c) { return c ? c->n : -1; }

int64_t jx_obs_bytes(const jx_ctx* c) {
  if (!c || c->n < 0) return -1;
  return c->obs_off.empty() ? 0 : c->obs_off.back();
}

jx_status jx_obs_offsets(const jx_ctx* c, int64_t* offsets_host) {
  jx_status st = check_ready(c);
  if (st) return st;
  if (!offsets_host) return set_error(JX_EINVAL, "offsets is null");
  std::memcpy(offsets_host, c->obs_off.data(), 8 * c->obs_off.size());
  return JX_OK;
}

jx_status jx_step(jx_ctx* c, const uint8_t* actions, uint8_t* obs, float* reward, uint8_t* done,
                  uint8_t* prev_action) {
  TraceRange range("jx_step");
  jx_status st = check_ready(c);
  if (st) return st;
  if (c->n == 0) return JX_OK;
  if (!actions || !obs || !reward || !done) return set_error(JX_EINVAL, "null buffer");
  if ((uintptr_t)obs & (obs_align(c->S.obs_fmt) - 1))
    return set_error(JX_EINVAL, "obs must be 4-byte aligned (16-byte for the floating formats)");
  DevIo io{};
  io.act = actions;
  io.obs = obs;
  io.rew = reward;
  io.done = done;
  io.prev = prev_action;
  io.mode = MODE_STEP;
  io.store_mode = c->launch.store_mode;
  return launch_or_fail(c, io, c->stream);
}

// Arguments of a T-step rollout.  JX_OK with *nothing = true when there is no
// work (no envs or T = 0).
static jx_status check_rollout(const jx_ctx* c, int32_t T, const uint8_t* actions, const uint8_t* obs,
                               int64_t obs_stride, const float* reward, const uint8_t* done, bool* nothing) {
  *nothing = true;
  jx_status st = check_ready(c);
  if (st) return st;
  if (T < 0) return set_error(JX_EINVAL, "T < 0");
  if (c->n == 0 || T == 0) return JX_OK;
  if (!actions || !obs || !reward || !done) return set_error(JX_EINVAL, "null buffer");
  const int64_t ob = c->obs_off.back();
  const int al = obs_align(c->S.obs_fmt);
  if (obs_stride < 0 || (obs_stride != 0 && obs_stride < ob) || (obs_stride & (al - 1)) ||
      ((uintptr_t)obs & (al - 1)))
    return set_error(JX_EINVAL, "obs_stride must be 0 or >= jx_obs_bytes(); obs and obs_stride 4-byte aligned "
                                "(16-byte for the floating formats)");
  *nothing = false;
  return JX_OK;
}

// The fused form: one launch for all T steps.  Under the persistent mapping
// (byte frames) persistent waves claim envs from the queue counters of launch
// `seq`; the pipelined mapping runs the plain fused kernel with 4 waves per
// workgroup.
static jx_status rollout_fused(jx_ctx* c, const DevState& S, int32_t T, const uint8_t* actions, uint8_t* obs,
                               int64_t obs_stride, float* reward, uint8_t* done, uint8_t* prev_action,
                               uint32_t seq) {
  LaunchCfg lc = c->launch;
  if (lc.form == JX_FORM_PIPELINE) lc = LaunchCfg{0, 4, 1, lc.store_mode};
  int rc = launch_rollout_fused(S, actions, obs, obs_stride, reward, done, prev_action, T, lc, c->max_side,
                                c->n_cu, seq, c->stream);
  if (rc) return set_error(JX_EDEVICE, std::string("fused rollout launch: ") + kernel_error_string(rc));
  return JX_OK;
}

// Step t's I/O of a rollout whose buffers are given by value.
static DevIo step_io(const jx_ctx* c, int t, const uint8_t* actions, uint8_t* obs, int64_t obs_stride,
                     float* reward, uint8_t* done, uint8_t* prev_action) {
  DevIo io{};
  io.act = actions + (int64_t)t * c->n;
  io.obs = obs + (int64_t)t * obs_stride;
  io.rew = reward + (int64_t)t * c->n;
  io.done = done + (int64_t)t * c->n;
  io.prev = prev_action ? prev_action + (int64_t)t * c->n : nullptr;
  io.mode = MODE_STEP;
  io.store_mode = c->launch.store_mode;
  return io;
}

jx_status jx_rollout(jx_ctx* c, int32_t T, const uint8_t* actions, uint8_t* obs, int64_t obs_stride,
                     float* reward, uint8_t* done, uint8_t* prev_action, int32_t flags) {
  TraceRange range("jx_rollout");
  bool nothing = true;
  jx_status st = check_rollout(c, T, actions, obs, obs_stride, reward, done, &nothing);
  if (st || nothing) return st;
  HIPCHK(hipSetDevice(c->device));
  if (flags & JX_ROLLOUT_FUSED) {
    st = rollout_fused(c, c->S, T, actions, obs, obs_stride, reward, done, prev_action, c->seq);
    if (st == JX_OK && c->launch.form == JX_FORM_PERSISTENT) c->seq += 1;
    return st;
  }
  if (!(flags & JX_ROLLOUT_GRAPH)) {
    for (int t = 0; t < T; ++t) {
      st = launch_or_fail(c, step_io(c, t, actions, obs, obs_stride, reward, done, prev_action), c->stream);
      if (st) return st;
    }
    return JX_OK;
  }
  // The captured kernels read their buffers from the workspace descriptor,
  // so one graph per (T, mapping) serves every call.
  RolloutDesc d{actions, obs, reward, done, prev_action, obs_stride, c->n, c->launch.store_mode};
  int rc = launch_set_desc(c->S.rdesc, d, c->stream);
  if (rc) return set_error(JX_EDEVICE, std::string("descriptor update: ") + kernel_error_string(rc));
  const std::array<int32_t, 6> key = {T, c->launch.form, c->launch.waves_per_group, c->launch.waves_per_env,
                                      c->launch.groups_per_cu, c->launch.store_mode};
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    jx_status lst = JX_OK;
    DevIo io{};
    io.mode = MODE_STEP;
    // a kernel (not a memset node) clears the queue counters at the head
    if (c->launch.form == JX_FORM_PERSISTENT && launch_clear_queues(c->S.queues, c->cap_stream) != 0)
      lst = set_error(JX_EDEVICE, "queue clear launch failed");
    for (int t = 0; t < T && lst == JX_OK; ++t)
      lst = launch_or_fail(c, io, c->cap_stream, c->S.rdesc, t, t);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (lst != JX_OK) {
      if (g) hipGraphDestroy(g);
      return lst;
    }
    if (e != hipSuccess) return set_error(JX_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(JX_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (c->graphs.size() >= 8) {
      hipGraphExecDestroy(c->graphs.begin()->second);
      c->graphs.erase(c->graphs.begin());
    }
    it = c->graphs.emplace(key, ge).first;
  }
  HIPCHK(hipGraphLaunch(it->second, c->stream));
  // the replay's last launch cleared counter set T % 4: continue from there
  if (c->launch.form == JX_FORM_PERSISTENT) c->seq = (uint32_t)T;
  return JX_OK;
}

jx_status jx_rollout_noalloc(jx_ctx* c, int32_t T, const uint8_t* actions, uint8_t* obs, int64_t obs_stride,
                             float* reward, uint8_t* done, uint8_t* prev_action, int32_t flags) {
  bool nothing = true;
  jx_status st = check_rollout(c, T, actions, obs, obs_stride, reward, done, &nothing);
  if (st) return st;
  if (flags & ~JX_ROLLOUT_FUSED)
    return set_error(JX_EINVAL, flags & JX_ROLLOUT_GRAPH
                                    ? "JX_ROLLOUT_GRAPH is not accepted: instantiating a graph allocates (use jx_rollout)"
                                    : "unknown rollout flags");
  if (nothing) return JX_OK;
  if (!c->scratch)
    return set_error(JX_EDEVICE, std::string("static scratch of this device unavailable: ") +
                                     kernel_error_string(c->scratch_err));
  HIPCHK(hipSetDevice(c->device));
  // the work-queue counters live in this device's static scratch array; every
  // other field is the context's own
  DevState S = c->S;
  S.queues = c->scratch;
  const bool queues = c->launch.form == JX_FORM_PERSISTENT && c->S.obs_fmt == 0;
  // the last call on this device left its counts behind: clear every counter
  // set with a kernel (capture-safe), then number the launches from 0
  if (queues && launch_clear_queues(c->scratch, c->stream) != 0)
    return set_error(JX_EDEVICE, "queue clear launch failed");
  if (flags & JX_ROLLOUT_FUSED) return rollout_fused(c, S, T, actions, obs, obs_stride, reward, done, prev_action, 0);
  for (int t = 0; t < T; ++t) {
    const DevIo io = step_io(c, t, actions, obs, obs_stride, reward, done, prev_action);
    const int rc = launch_batch(S, io, nullptr, 0, c->launch, c->max_side, c->n_cu, (uint32_t)t, c->stream);
    if (rc != 0) return set_error(JX_EDEVICE, std::string("kernel launch: ") + kernel_error_string(rc));
  }
  return JX_OK;
}

jx_status jx_render(jx_ctx* c, uint8_t* obs, jx_col_debug* dbg) {
  TraceRange range("jx_render");
  jx_status st = check_ready(c);
  if (st) return st;
  if (c->n == 0) return JX_OK;
  if (obs && ((uintptr_t)obs & (obs_align(c->S.obs_fmt) - 1)))
    return set_error(JX_EINVAL, "obs must be 4-byte aligned (16-byte for the floating formats)");
  DevIo io{};
  io.obs = obs;
  io.dbg = dbg;
  io.dbg_stride = c->max_w;
  io.mode = MODE_RENDER;
  io.store_mode = c->launch.store_mode;
  return launch_or_fail(c, io, c->stream);
}

size_t jx_state_bytes(const jx_ctx* c) {
  if (!c || c->n < 0) return 0;
  return (size_t)c->L.rdesc;
}

jx_status jx_state_layout(const jx_ctx* c, jx_field* f, int32_t cap, int32_t* n_fields) {
  jx_status st = check_ready(c);
  if (st) return st;
  const Layout& L = c->L;
  const int n = c->n;
  struct F {
    const char* name;
    int64_t off;
    int elem;
    int64_t count;
  } all[] = {{"header", L.hdr, 1, (int64_t)sizeof(WsHeader)},
             {"x", L.x, 4, n},
             {"y", L.y, 4, n},
             {"theta", L.th, 4, n},
             {"t", L.t, 4, n},
             {"episode", L.ep, 4, n},
             {"goal", L.goal, 4, n},
             {"door", L.door, 4, n},
             {"key", L.key, 4, n},
             {"decor", L.decor, 4, 2 * (int64_t)n},
             {"akey", L.akey, 4, 3 * (int64_t)n},
             {"doors", L.doors, 4, n},
             {"flags", L.flags, 1, n},
             {"events", L.events, 1, n},
             {"n_decor", L.ndecor, 1, n},
             {"invalid", L.invalid, 4, n},
             {"seed", L.seed, 8, n},
             {"cfg_index", L.cfg_idx, 4, n},
             {"map_offset", L.map_off, 4, n},
             {"obs_offset", L.obs_off, 8, (int64_t)n + 1},
             {"order", L.order, 4, n},
             {"cfgs", L.cfgs, (int)sizeof(DevCfg), (int64_t)c->cfgs.size()},
             {"maps", L.maps, 1, L.rdesc - L.maps}};
  const int total = (int)(sizeof(all) / sizeof(all[0]));
  if (n_fields) *n_fields = total;
  if (!f) return JX_OK;
  for (int i = 0; i < total && i < cap; ++i) {
    std::memset(&f[i], 0, sizeof(jx_field));
    std::snprintf(f[i].name, sizeof(f[i].name), "%s", all[i].name);
    f[i].offset = all[i].off;
    f[i].elem = all[i].elem;
    f[i].count = (int32_t)all[i].count;
    f[i].bytes = all[i].elem * all[i].count;
  }
  return JX_OK;
}

jx_status jx_get_state(const jx_ctx* c, void* host, size_t bytes) {
  jx_status st = check_ready(c);
  if (st) return st;
  if (!host || bytes < (size_t)c->L.rdesc) return set_error(JX_EINVAL, "host buffer too small");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(host, c->ws, (size_t)c->L.rdesc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return JX_OK;
}

jx_status jx_set_state(jx_ctx* c, const void* host, size_t bytes) {
  jx_status st = check_ready(c);
  if (st) return st;
  if (!host || bytes < (size_t)c->L.rdesc) return set_error(JX_EINVAL, "state image too small");
  const uint8_t* b = (const uint8_t*)host;
  WsHeader h;
  std::memcpy(&h, b + c->L.hdr, sizeof(h));
  if (h.magic != kStateMagic || h.n_envs != c->n || h.state_bytes != c->L.rdesc ||
      h.n_cfgs != (int32_t)c->cfgs.size())
    return set_error(JX_EINVAL, "state image does not match this context");
  if (std::memcmp(b + c->L.cfgs, c->dev_cfgs.data(), sizeof(DevCfg) * c->dev_cfgs.size()) != 0 ||
      std::memcmp(b + c->L.obs_off, c->obs_off.data(), 8 * c->obs_off.size()) != 0 ||
      std::memcmp(b + c->L.cfg_idx, c->cfg_idx.data(), 4 * (size_t)c->n) != 0)
    return set_error(JX_EINVAL, "state image configuration differs from this context");
  // every index the kernels dereference must be in range
  st = check_state_image(b, c->L, c->n, c->cfgs, c->cfg_idx);
  if (st) return st;
  std::vector<uint8_t> img(b, b + c->L.rdesc);
  WsHeader* hh = (WsHeader*)(img.data() + c->L.hdr);
  hh->queue = 0;
  hh->exited = 0;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(c->ws, img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return JX_OK;
}

jx_status jx_set_launch(jx_ctx* c, const jx_launch* l) {
  if (!c || !l) return set_error(JX_EINVAL, "null argument");
  const int w = l->waves_per_group;
  if (l->form != JX_FORM_PLAIN && l->form != JX_FORM_PERSISTENT && l->form != JX_FORM_PIPELINE)
    return set_error(JX_EINVAL, "bad form");
  if (w != 1 && w != 2 && w != 4 && w != 8) return set_error(JX_EINVAL, "waves_per_group must be 1, 2, 4 or 8");
  if (l->form == JX_FORM_PIPELINE && w == 8) return set_error(JX_EINVAL, "pipelined form: 1, 2 or 4 wave pairs");
  if (l->form != JX_FORM_PLAIN && (l->groups_per_cu < 1 || l->groups_per_cu > 16))
    return set_error(JX_EINVAL, "groups_per_cu must be in 1..16");
  if (l->store_mode != 0 && l->store_mode != 1) return set_error(JX_EINVAL, "store_mode must be 0 or 1");
  const int wpe = l->waves_per_env;
  if (wpe != 1 && wpe != 2 && wpe != 4) return set_error(JX_EINVAL, "waves_per_env must be 1, 2 or 4");
  if (wpe > 1 && l->form != JX_FORM_PLAIN) return set_error(JX_EINVAL, "waves_per_env > 1 needs the plain form");
  if (wpe > w) return set_error(JX_EINVAL, "waves_per_env must not exceed waves_per_group");
  c->launch = LaunchCfg{l->form, w, std::max(1, l->groups_per_cu), l->store_mode, wpe};
  return JX_OK;
}

jx_status jx_get_launch(const jx_ctx* c, jx_launch* l) {
  if (!c || !l) return set_error(JX_EINVAL, "null argument");
  l->form = c->launch.form;
  l->waves_per_group = c->launch.waves_per_group;
  l->groups_per_cu = c->launch.groups_per_cu;
  l->store_mode = c->launch.store_mode;
  l->waves_per_env = c->launch.waves_per_env;
  return JX_OK;
}

jx_status jx_sync(jx_ctx* c) {
  if (!c) return set_error(JX_EINVAL, "null context");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipGetLastError());
  return JX_OK;
}

jx_status jx_make_layout(uint64_t seed, const jx_env_cfg* cfg, uint8_t* grid) {
  if (!cfg || !grid) return set_error(JX_EINVAL, "null argument");
  std::string why;
  if (!validate_cfg(*cfg, &why)) return set_error(JX_EINVAL, why);
  if (cfg->ascii_map) {
    int32_t keys[3];
    if (parse_ascii_map(cfg->ascii_map, cfg->side, grid, keys, &why) < 0) return set_error(JX_EINVAL, why);
    return JX_OK;
  }
  if (!make_maze(seed, cfg->side, cfg->loop_frac, grid)) return set_error(JX_EINVAL, "maze generation failed");
  return JX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
namespace {

std::string tune_key(const jx_ctx* c) {
  hipDeviceProp_t p;
  hipGetDeviceProperties(&p, c->device);
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* d, size_t n) {
    const uint8_t* b = (const uint8_t*)d;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(c->dev_cfgs.data(), sizeof(DevCfg) * c->dev_cfgs.size());
  mix(c->cfg_idx.data(), 4 * c->cfg_idx.size());
  std::ostringstream o;
  o << p.gcnArchName << "/cu" << c->n_cu << "/n" << c->n << "/h" << std::hex << h;
  std::string s = o.str();
  for (char& ch : s)
    if (ch == ' ' || ch == '\n') ch = '_';
  return s;
}

bool cache_lookup(const char* path, const std::string& key, LaunchCfg* out) {
  if (!path) return false;
  std::ifstream f(path);
  std::string k;
  LaunchCfg l{};
  bool found = false;
  while (f >> k >> l.form >> l.waves_per_group >> l.groups_per_cu >> l.store_mode >> l.waves_per_env)
    if (k == key) {
      *out = l;
      found = true;
    }
  return found;
}

}  // namespace

extern "C" jx_status jx_autotune(jx_ctx* c, const uint8_t* actions, int32_t iters,
                                 uint8_t* obs_scratch, const char* cache_path, jx_launch* chosen) {
  jx_status st = check_ready(c);
  if (st) return st;
  if (iters < 1 || !actions || !obs_scratch) return set_error(JX_EINVAL, "need iters >= 1, actions and obs scratch");
  if (c->n == 0) return JX_OK;
  HIPCHK(hipSetDevice(c->device));
  const std::string key = tune_key(c);
  LaunchCfg hit{};
  if (cache_lookup(cache_path, key, &hit)) {
    c->launch = hit;
    if (chosen) jx_get_launch(c, chosen);
    return JX_OK;
  }
  const size_t total = (size_t)c->L.rdesc;  // the state image
  const int64_t ob = c->obs_off.back();
  const int n = c->n;
  uint8_t* snap = nullptr;
  uint8_t* io_buf = nullptr;
  HIPCHK(hipMalloc(&snap, total));
  if (hipMalloc(&io_buf, (size_t)iters * n * 5) != hipSuccess) {
    hipFree(snap);
    return set_error(JX_ENOMEM, "autotune buffers");
  }
  float* rew = (float*)io_buf;
  uint8_t* dn = io_buf + (size_t)iters * n * 4;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMemcpyAsync(snap, c->ws, total, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(snap);
    hipFree(io_buf);
    return set_error(JX_EDEVICE, "autotune set-up failed");
  }

  std::vector<LaunchCfg> cands;
  for (int w : {1, 2, 4, 8})
    for (int s : {0, 1}) cands.push_back(LaunchCfg{0, w, 1, s});
  // several waves per env (small batches of large frames)
  for (int w : {4, 8})
    for (int e : {2, 4}) cands.push_back(LaunchCfg{0, w, 1, 0, e});
  for (int w : {1, 2, 4})
    for (int g : {2, 4, 8})
      for (int s : {0, 1}) cands.push_back(LaunchCfg{1, w, g, s});
  for (int p : {1, 2, 4})
    for (int g : {1, 2, 4})
      for (int s : {0, 1}) cands.push_back(LaunchCfg{2, p, g, s});
  const LaunchCfg keep = c->launch;
  std::vector<uint8_t> ref_obs(ob), ref_state(total), ref_io((size_t)iters * n * 5);
  std::vector<uint8_t> cur_obs(ob), cur_state(total), cur_io((size_t)iters * n * 5);
  float best_ms = 1e30f;
  LaunchCfg best = cands[0];
  jx_status result = JX_OK;
  for (size_t k = 0; k < cands.size() && result == JX_OK; ++k) {
    c->launch = cands[k];
    float ms_min = 1e30f;
    for (int rep = 0; rep < 2 && result == JX_OK; ++rep) {
      if (hipMemcpyAsync(c->ws, snap, total, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
          hipEventRecord(e0, c->stream) != hipSuccess) {
        result = set_error(JX_EDEVICE, "autotune: state restore failed");
        break;
      }
      for (int t = 0; t < iters && result == JX_OK; ++t) {
        DevIo io{};
        io.act = actions + (int64_t)t * n;
        io.obs = obs_scratch;
        io.rew = rew + (int64_t)t * n;
        io.done = dn + (int64_t)t * n;
        io.mode = MODE_STEP;
        io.store_mode = c->launch.store_mode;
        result = launch_or_fail(c, io, c->stream);
      }
      if (result != JX_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        result = set_error(JX_EDEVICE, "autotune run failed");
        break;
      }
      ms_min = std::min(ms_min, ms);
    }
    if (result != JX_OK) break;
    std::vector<uint8_t>& o = (k == 0) ? ref_obs : cur_obs;
    std::vector<uint8_t>& s = (k == 0) ? ref_state : cur_state;
    std::vector<uint8_t>& i2 = (k == 0) ? ref_io : cur_io;
    if (hipMemcpy(o.data(), obs_scratch, ob, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(s.data(), c->ws, total, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(i2.data(), io_buf, i2.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      result = set_error(JX_EDEVICE, "autotune: result copy failed");
      break;
    }
    const bool same = (k == 0) || (o == ref_obs && s == ref_state && i2 == ref_io);
    if (!same) {
      result = set_error(JX_EDEVICE, "autotune: candidate mapping changed the results");
      break;
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = cands[k];
    }
  }
  // the caller's state comes back whatever happened above
  if ((hipMemcpyAsync(c->ws, snap, total, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
       hipStreamSynchronize(c->stream) != hipSuccess) && result == JX_OK)
    result = set_error(JX_EDEVICE, "autotune: state restore failed");
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(snap);
  hipFree(io_buf);
  if (result != JX_OK) {
    c->launch = keep;
    return result;
  }
  c->launch = best;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key << " " << best.form << " " << best.waves_per_group << " " << best.groups_per_cu << " "
      << best.store_mode << " " << best.waves_per_env << "\n";
  }
  if (chosen) jx_get_launch(c, chosen);
  return JX_OK;
}
