// jx_host.cpp -- host-only parts of the runtime (no HIP calls): argument and
// configuration validation, the workspace layout, the state image of a reset
// and the checks on a state image loaded by jx_set_state.  Kept apart from the
// HIP calls so that a sanitizer build can exercise them on the CPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "jx.h"
#include "jx_common.h"
#include "jx_internal.h"
#include "jx_layout.h"

namespace jx {

thread_local std::string g_last_error;

jx_status set_error(jx_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

bool validate_cfg(const jx_env_cfg& c, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (c.side < 5 || c.side > kMaxSide) return bad("side must be in 5..64");
  if (c.n_colors < 1 || c.n_colors > 8) return bad("n_colors must be in 1..8");
  if (!(c.loop_frac >= 0.f && c.loop_frac <= 1.f)) return bad("loop_frac must be in [0, 1]");
  if (c.key_door != 0 && c.key_door != 1) return bad("key_door must be 0 or 1");
  if (c.goal_sprite != 0 && c.goal_sprite != 1) return bad("goal_sprite must be 0 or 1");
  if (c.max_decor < 0 || c.max_decor > kMaxDecor) return bad("max_decor must be in 0..2");
  if (c.obs_h < 2 || c.obs_h > kMaxH || (c.obs_h & 1)) return bad("obs_h must be even, 2..128");
  if (c.obs_w < 4 || c.obs_w > kMaxW || (c.obs_w & 3)) return bad("obs_w must be a multiple of 4, 4..128");
  if (!(c.fov_deg >= 0.f && c.fov_deg < 180.f)) return bad("fov_deg must be in [0, 180)");
  if (c.n_actions != 4 && c.n_actions != 6) return bad("n_actions must be 4 or 6");
  if (c.episode_cap < 1) return bad("episode_cap must be >= 1");
  if (!std::isfinite(c.move) || !std::isfinite(c.turn) || !std::isfinite(c.r_goal) ||
      !std::isfinite(c.r_key) || !(c.pickup_radius >= 0.f) || !std::isfinite(c.pickup_radius))
    return bad("move, turn, rewards and pickup_radius must be finite (radius >= 0)");
  if (std::fabs(c.move) >= 1.f) return bad("|move| must be below one tile");
  if (c.shade_levels < 0 || c.shade_levels > kMaxShadeLevels) return bad("shade_levels must be in 0..16");
  if (c.shade_levels > 0 && !(c.shade_dist > 0.f && std::isfinite(c.shade_dist)))
    return bad("shade_dist must be finite and > 0 when shading is on");
  if (c.obs_layout != JX_OBS_NHWC && c.obs_layout != JX_OBS_NCHW) return bad("obs_layout must be JX_OBS_NHWC or JX_OBS_NCHW");
  if (c.obs_dtype != JX_OBS_U8 && c.obs_dtype != JX_OBS_BF16 && c.obs_dtype != JX_OBS_F32)
    return bad("obs_dtype must be JX_OBS_U8, JX_OBS_BF16 or JX_OBS_F32");
  if (c.ascii_map) {
    if (c.key_door || c.max_decor) return bad("an ascii map brings its own keys and doors: key_door and max_decor must be 0");
    std::vector<uint8_t> g((size_t)c.side * c.side);
    int32_t keys[3];
    std::string w;
    if (parse_ascii_map(c.ascii_map, c.side, g.data(), keys, &w) < 0) return bad(w.c_str());
  }
  return true;
}

DevCfg derive_cfg(const jx_env_cfg& c) {
  DevCfg d{};
  d.side = c.side;
  d.n_colors = c.n_colors;
  d.key_door = c.key_door;
  d.goal_sprite = c.goal_sprite;
  d.max_decor = c.max_decor;
  d.obs_h = c.obs_h;
  d.obs_w = c.obs_w;
  d.n_actions = c.n_actions;
  d.cap = c.episode_cap;
  d.move = c.move;
  d.turn = c.turn;
  d.pr2 = c.pickup_radius * c.pickup_radius;
  d.r_goal = c.r_goal;
  d.r_key = c.r_key;
  d.tanH = (float)std::tan((double)c.fov_deg * M_PI / 360.0);
  d.inv_tanH = (float)(1.0 / (double)d.tanH);
  d.inv_w = (float)(1.0 / (double)c.obs_w);
  const double q = std::tan((double)c.fov_deg * M_PI / 360.0) / (double)c.obs_w;
  d.ray_q_hi = (float)q;
  d.ray_q_lo = (float)(q - (double)d.ray_q_hi);
  d.shade_levels = c.shade_levels;
  d.shade_scale = c.shade_levels > 0 ? (float)((double)c.shade_levels / (double)c.shade_dist) : 0.f;
  d.shade_mul = c.shade_levels > 0 ? (65536u + (uint32_t)c.shade_levels - 1u) / (uint32_t)c.shade_levels : 0u;
  d.ascii = c.ascii_map ? 1 : 0;
  return d;
}

static int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

Layout make_layout(int n, int n_cfgs, int64_t maps_bytes) {
  Layout L{};
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    int64_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  const int64_t nn = std::max(n, 1);
  L.hdr = take(sizeof(WsHeader));
  L.x = take(4 * nn);
  L.y = take(4 * nn);
  L.th = take(4 * nn);
  L.t = take(4 * nn);
  L.ep = take(4 * nn);
  L.goal = take(4 * nn);
  L.door = take(4 * nn);
  L.key = take(4 * nn);
  L.decor = take(8 * nn);
  L.akey = take(12 * nn);
  L.doors = take(4 * nn);
  L.flags = take(nn);
  L.events = take(nn);
  L.ndecor = take(nn);
  L.invalid = take(4 * nn);
  L.seed = take(8 * nn);
  L.cfg_idx = take(4 * nn);
  L.map_off = take(4 * nn);
  L.obs_off = take(8 * (nn + 1));
  L.order = take(4 * nn);
  L.cfgs = take((int64_t)sizeof(DevCfg) * std::max(n_cfgs, 1));
  L.maps = take(std::max<int64_t>(maps_bytes, 16));
  // after the state image: the rollout descriptor (scratch, not state)
  L.rdesc = take(sizeof(RolloutDesc));
  L.queues = take(4 * kQueueWords);
  L.total = o;
  return L;
}

int64_t map_bytes_of(int side) { return align_up((int64_t)side * side, 16); }

int obs_fmt_of(const jx_env_cfg& c) { return c.obs_layout * 3 + c.obs_dtype; }
int64_t frame_bytes(const jx_env_cfg& c) {
  return (int64_t)c.obs_h * c.obs_w * 3 * obs_elem_bytes(obs_fmt_of(c));
}

// Marks a batch whose envs all use one configuration (the common case): the
// kernels then read the configuration from the kernel argument and compute map
// and frame offsets from the env index.
void set_uniform(DevState* s, const jx_env_cfg* cfgs, int n_cfgs, const std::vector<int32_t>& idx) {
  s->any_ascii = 0;
  for (int k = 0; k < n_cfgs; ++k)
    if (cfgs[k].ascii_map) s->any_ascii = 1;
  bool one = n_cfgs >= 1;
  for (size_t i = 1; i < idx.size() && one; ++i) one = idx[i] == idx[0];
  s->uniform = 0;
  if (!one || idx.empty()) return;
  const jx_env_cfg& c = cfgs[idx[0]];
  s->uniform = 1;
  s->ucfg = derive_cfg(c);
  s->map_stride = map_bytes_of(c.side);
  s->obs_stride = frame_bytes(c);
}

DevState bind_state(uint8_t* ws, const Layout& L, int n) {
  DevState s{};
  s.x = (float*)(ws + L.x);
  s.y = (float*)(ws + L.y);
  s.th = (float*)(ws + L.th);
  s.t = (uint32_t*)(ws + L.t);
  s.ep = (uint32_t*)(ws + L.ep);
  s.goal = (int32_t*)(ws + L.goal);
  s.door = (int32_t*)(ws + L.door);
  s.key = (int32_t*)(ws + L.key);
  s.decor = (int32_t*)(ws + L.decor);
  s.akey = (int32_t*)(ws + L.akey);
  s.doors = (uint32_t*)(ws + L.doors);
  s.flags = ws + L.flags;
  s.events = ws + L.events;
  s.ndecor = ws + L.ndecor;
  s.invalid = (uint32_t*)(ws + L.invalid);
  s.seed = (const uint64_t*)(ws + L.seed);
  s.cfg_idx = (const int32_t*)(ws + L.cfg_idx);
  s.map_off = (const uint32_t*)(ws + L.map_off);
  s.obs_off = (const int64_t*)(ws + L.obs_off);
  s.order = (const int32_t*)(ws + L.order);
  s.rdesc = (RolloutDesc*)(ws + L.rdesc);
  s.queues = (uint32_t*)(ws + L.queues);
  s.cfgs = (const DevCfg*)(ws + L.cfgs);
  s.maps = ws + L.maps;
  s.hdr = (WsHeader*)(ws + L.hdr);
  s.n = n;
  return s;
}

// Builds the host image of a freshly reset workspace (state arrays zero; the
// device episode reset fills them).  Maze generation is spread over threads.
jx_status build_image(int n, const uint64_t* seeds, const jx_env_cfg* cfgs, int n_cfgs,
                      const int32_t* cfg_index, std::vector<uint8_t>* img, Layout* Lout,
                      std::vector<int64_t>* obs_off, std::vector<int32_t>* idx_out) {
  std::vector<int32_t> idx(n);
  for (int i = 0; i < n; ++i) {
    int c = cfg_index ? cfg_index[i] : 0;
    if (c < 0 || c >= n_cfgs) return set_error(JX_EINVAL, "cfg_index out of range");
    idx[i] = c;
  }
  std::vector<uint32_t> moff(n);
  int64_t mb = 0;
  for (int i = 0; i < n; ++i) {
    if (mb > 0xFFFFFFFFll) return set_error(JX_ENOMEM, "maps exceed 4 GiB");
    moff[i] = (uint32_t)mb;
    mb += map_bytes_of(cfgs[idx[i]].side);
  }
  Layout L = make_layout(n, n_cfgs, mb);
  img->assign((size_t)L.total, 0);
  uint8_t* b = img->data();
  WsHeader* h = (WsHeader*)(b + L.hdr);
  h->magic = kStateMagic;
  h->n_envs = n;
  h->state_bytes = L.rdesc;
  h->n_cfgs = n_cfgs;
  obs_off->assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const jx_env_cfg& c = cfgs[idx[i]];
    (*obs_off)[i + 1] = (*obs_off)[i] + frame_bytes(c);
  }
  std::memcpy(b + L.seed, seeds, 8 * (size_t)n);
  std::memcpy(b + L.cfg_idx, idx.data(), 4 * (size_t)n);
  std::memcpy(b + L.map_off, moff.data(), 4 * (size_t)n);
  std::memcpy(b + L.obs_off, obs_off->data(), 8 * (size_t)(n + 1));
  for (int i = 0; i < n; ++i) ((int32_t*)(b + L.decor))[2 * i] = ((int32_t*)(b + L.decor))[2 * i + 1] = -1;
  for (int i = 0; i < 3 * n; ++i) ((int32_t*)(b + L.akey))[i] = -1;
  // costliest envs first for the persistent queue (frame bytes, then map side)
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    const jx_env_cfg& A = cfgs[idx[a]];
    const jx_env_cfg& C = cfgs[idx[c]];
    int64_t ca = (int64_t)A.obs_h * A.obs_w * 4 + (int64_t)A.side * A.side;
    int64_t cc = (int64_t)C.obs_h * C.obs_w * 4 + (int64_t)C.side * C.side;
    return ca > cc;
  });
  std::memcpy(b + L.order, order.data(), 4 * (size_t)n);
  for (int c = 0; c < n_cfgs; ++c) ((DevCfg*)(b + L.cfgs))[c] = derive_cfg(cfgs[c]);
  // mazes
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int n_thr = (n >= 256) ? (int)hw : 1;
  std::vector<std::thread> thr;
  std::vector<int> okv(n_thr, 1);
  for (int tI = 0; tI < n_thr; ++tI) {
    thr.emplace_back([&, tI] {
      for (int i = tI; i < n; i += n_thr) {
        const jx_env_cfg& c = cfgs[idx[i]];
        if (c.ascii_map) {
          int32_t keys[3];
          if (parse_ascii_map(c.ascii_map, c.side, b + L.maps + moff[i], keys, nullptr) < 0) okv[tI] = 0;
          std::memcpy(b + L.akey + 12 * (int64_t)i, keys, 12);
        } else if (!make_maze(seeds[i], c.side, c.loop_frac, b + L.maps + moff[i])) {
          okv[tI] = 0;
        }
      }
    });
  }
  for (auto& t : thr) t.join();
  for (int v : okv)
    if (!v) return set_error(JX_EINVAL, "maze generation failed");
  *Lout = L;
  *idx_out = idx;
  return JX_OK;
}


// Checks a state image against the context it is loaded into: every index the
// kernels dereference must be in range and every map border must block.
jx_status check_state_image(const uint8_t* b, const Layout& L, int n, const std::vector<jx_env_cfg>& cfgs,
                            const std::vector<int32_t>& cfg_idx) {
  int64_t expect_moff = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t mo;
    std::memcpy(&mo, b + L.map_off + 4 * i, 4);
    if ((int64_t)mo != expect_moff) return set_error(JX_EINVAL, "state image: map offsets differ from this context");
    expect_moff += map_bytes_of(cfgs[cfg_idx[i]].side);
  }
  for (int i = 0; i < n; ++i) {
    const int N = cfgs[cfg_idx[i]].side;
    const int NN = N * N;
    float x, y, th;
    std::memcpy(&x, b + L.x + 4 * i, 4);
    std::memcpy(&y, b + L.y + 4 * i, 4);
    std::memcpy(&th, b + L.th + 4 * i, 4);
    int32_t ids[5];
    std::memcpy(&ids[0], b + L.goal + 4 * i, 4);
    std::memcpy(&ids[1], b + L.door + 4 * i, 4);
    std::memcpy(&ids[2], b + L.key + 4 * i, 4);
    std::memcpy(&ids[3], b + L.decor + 8 * i, 8);
    const uint8_t nd = b[L.ndecor + i];
    uint32_t moff;
    std::memcpy(&moff, b + L.map_off + 4 * i, 4);
    bool ok = std::isfinite(x) && std::isfinite(y) && std::isfinite(th) && x >= 0.f && y >= 0.f &&
              x < (float)N && y < (float)N && nd <= kMaxDecor && b[L.flags + i] <= 31 &&
              moff + (uint64_t)NN <= (uint64_t)(L.rdesc - L.maps);
    for (int k = 0; k < 5; ++k) ok = ok && ids[k] >= -1 && ids[k] < NN;
    for (int k = 0; k < 3; ++k) {
      int32_t ak;
      std::memcpy(&ak, b + L.akey + 12 * (int64_t)i + 4 * k, 4);
      ok = ok && ak >= -1 && ak < NN;
    }
    if (ok) {
      // every border tile of the map must be a wall (the walks rely on it)
      const uint8_t* m = b + L.maps + moff;
      auto wall = [](uint8_t v) { return !(v & kTileDoor) && (v & 0x0F) != 0; };
      for (int k = 0; k < N && ok; ++k)
        ok = wall(m[k]) && wall(m[(N - 1) * N + k]) && wall(m[k * N]) && wall(m[k * N + N - 1]);
    }
    for (int k = 0; k < nd; ++k) ok = ok && ids[3 + k] >= 0;
    if (!ok) return set_error(JX_EINVAL, "state image: env " + std::to_string(i) + " holds an out-of-range value");
  }
  return JX_OK;
}

}  // namespace jx
