// jx_kernels.hip -- fused step + raycast render for gfx950 (CDNA4).
//
// One 64-lane wave owns one environment for the whole step:
//   1. stage the env's N x N tile map from HBM into the wave's LDS slice;
//   2. apply the action (turn / move / strafe, axis-separated collision), then
//      key, goal, reward, truncation (rules of the key-door and navigation tasks,
//      Table 1 and Table 2 of the paper);
//   3. on done, reset the episode in place: spawn, heading, goal by BFS, door on
//      a shortest path, key in the start region, decor.  BFS runs bit-parallel:
//      lane y holds map row y as a 64-bit mask, one frontier expansion per
//      iteration (shift within the row, lane shuffle across rows);
//   4. cast one ray per screen column (lane c takes columns c, c+64, ...) with
//      DDA over tile boundaries (Sec. 2.1) through the LDS map, and reduce each
//      column to a span record: wall colour, wall half-height in rows, nearest
//      covering sprite's colour and half-height (billboard sprites, Fig. 1);
//   5. expand the span records straight into row-major uint8 RGB: each lane
//      emits 4 consecutive pixels (12 bytes) per iteration, so a wave writes 768
//      contiguous bytes per store instruction.
// Nothing here is a dense contraction, so there is no MFMA; the bound is the
// HBM write of the frames and the vector ALU of the span expansion.
#include <hip/hip_runtime.h>

#include "jx_internal.h"

namespace jx {

namespace {

constexpr uint32_t rgb(uint32_t r, uint32_t g, uint32_t b) { return r | (g << 8) | (b << 16); }

// Colours of this build (the paper draws flat colours without assets).
__constant__ uint32_t kPalette[8] = {rgb(180, 40, 40), rgb(40, 160, 40),  rgb(40, 60, 180),
                                     rgb(190, 170, 40), rgb(150, 40, 170), rgb(40, 160, 170),
                                     rgb(200, 110, 30), rgb(150, 150, 150)};
constexpr uint32_t kCeil = rgb(50, 50, 60);
constexpr uint32_t kFloor = rgb(90, 80, 70);
constexpr uint32_t kDoor = rgb(120, 0, 0);
constexpr uint32_t kKeyRgb = rgb(255, 40, 40);
constexpr uint32_t kGoalRgb = rgb(255, 230, 0);
constexpr uint32_t kDecorRgb = rgb(0, 200, 120);

constexpr float kTwoPiF = 6.28318548202514648f;  // float nearest to 2*pi

// ---- wave primitives ---------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t shfl_idx64(uint64_t v, int src) {
  uint32_t lo = __shfl((int)(uint32_t)v, src, 64);
  uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
  uint32_t lo = __shfl_up((int)(uint32_t)v, d, 64);
  uint32_t hi = __shfl_up((int)(uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_down64(uint64_t v, int d) {
  uint32_t lo = __shfl_down((int)(uint32_t)v, d, 64);
  uint32_t hi = __shfl_down((int)(uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = (uint32_t)__shfl_up((int)v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// ---- SplitMix64 (Steele, Lea & Flood 2014) --------------------------------------
__device__ __forceinline__ uint64_t sm_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm_mix(uint64_t v) { return sm_next(v); }
__device__ __forceinline__ uint32_t sm_draw(uint64_t& s, uint32_t n) {
  return (uint32_t)(((sm_next(s) >> 32) * (uint64_t)n) >> 32);
}

// ---- row-mask set operations (lane y < N holds row y) ---------------------------
// Tile id of the r-th set bit in row-major order of the distributed mask.
__device__ int mask_select(uint64_t m, uint32_t r, int N, int lane) {
  uint32_t c = (uint32_t)__popcll(m);
  uint32_t incl = wave_incl_scan(c, lane);
  uint32_t excl = incl - c;
  uint64_t own = __ballot(r >= excl && r < incl);
  int L = __ffsll((unsigned long long)own) - 1;
  uint64_t mm = shfl_idx64(m, L);
  uint32_t k = r - (uint32_t)__shfl((int)excl, L, 64);
  for (uint32_t i = 0; i < k; ++i) mm &= mm - 1;
  return L * N + (__ffsll((unsigned long long)mm) - 1);
}
__device__ __forceinline__ uint32_t mask_count(uint64_t m, int lane) {
  uint32_t incl = wave_incl_scan((uint32_t)__popcll(m), lane);
  return (uint32_t)__shfl((int)incl, 63, 64);
}
__device__ __forceinline__ int mask_first(uint64_t m, int N) {
  uint64_t own = __ballot(m != 0ull);
  if (own == 0ull) return -1;
  int L = __ffsll((unsigned long long)own) - 1;
  uint64_t mm = shfl_idx64(m, L);
  return L * N + (__ffsll((unsigned long long)mm) - 1);
}
__device__ __forceinline__ uint64_t bit_of(int id, int N, int lane) {
  return (id >= 0 && lane == id / N) ? (1ull << (id % N)) : 0ull;
}

struct Bfs {
  int level;
  uint64_t frontier;
  uint64_t visited;
};
// Level-synchronous BFS over the passable mask; stops after `stop` levels
// (stop < 0: until the frontier empties).  Every wave reaches the exit: the
// visited set grows each iteration and is bounded by the map.
__device__ Bfs bfs_rows(uint64_t pass, int src, int N, int stop, int lane) {
  uint64_t F = bit_of(src, N, lane);
  uint64_t V = F;
  int level = 0;
  while (level != stop) {
    uint64_t up = shfl_up64(F, 1);
    uint64_t dn = shfl_down64(F, 1);
    if (lane == 0) up = 0ull;
    if (lane == 63) dn = 0ull;
    uint64_t nf = ((F << 1) | (F >> 1) | up | dn) & pass & ~V;
    if (!wave_any(nf != 0ull)) break;
    V |= nf;
    F = nf;
    ++level;
  }
  return {level, F, V};
}

struct Episode {
  float x, y, th;
  int goal, door, key, nd, dec0, dec1;
};

// Episode reset for episode `e` of the env with layout in `lmap` (0 floor).
__device__ Episode episode_reset(const DevCfg& cf, const uint8_t* lmap, uint64_t seed, uint32_t e,
                                 int lane) {
  const int N = cf.side;
  uint64_t s = seed ^ sm_mix((uint64_t)e + 1ull);
  uint64_t freem = 0ull;
  if (lane < N) {
    const uint8_t* row = lmap + lane * N;
    for (int xx = 0; xx < N; ++xx)
      if (row[xx] == 0) freem |= 1ull << xx;
  }
  const uint32_t n_free = mask_count(freem, lane);
  Episode ep;
  const int spawn = mask_select(freem, sm_draw(s, n_free), N, lane);
  const uint32_t k24 = (uint32_t)(sm_next(s) >> 40);
  ep.th = (float)k24 * (kTwoPiF * 0x1p-24f);
  ep.x = (float)(spawn % N) + 0.5f;
  ep.y = (float)(spawn / N) + 0.5f;

  Bfs b = bfs_rows(freem, spawn, N, -1, lane);
  const int L = b.level;
  ep.goal = mask_first(b.frontier, N);
  ep.door = -1;
  ep.key = -1;
  if (cf.key_door && L >= 2) {
    const int h = L / 2;
    Bfs a = bfs_rows(freem, spawn, N, h, lane);
    Bfs g = bfs_rows(freem, ep.goal, N, L - h, lane);
    ep.door = mask_first(a.frontier & g.frontier, N);
    const uint64_t pass2 = freem & ~bit_of(ep.door, N, lane);
    Bfs r = bfs_rows(pass2, spawn, N, -1, lane);
    const uint64_t region = r.visited & ~bit_of(spawn, N, lane);
    const uint32_t c = mask_count(region, lane);
    ep.key = (c == 0) ? spawn : mask_select(region, sm_draw(s, c), N, lane);
  }
  ep.nd = 0;
  ep.dec0 = -1;
  ep.dec1 = -1;
  if (cf.max_decor > 0) {
    uint64_t cand = freem & ~bit_of(spawn, N, lane) & ~bit_of(ep.goal, N, lane) &
                    ~bit_of(ep.key, N, lane) & ~bit_of(ep.door, N, lane);
    const uint32_t C = mask_count(cand, lane);
    const int md = cf.max_decor > kMaxDecor ? kMaxDecor : cf.max_decor;
    int nd = (int)sm_draw(s, (uint32_t)(md + 1));
    if (nd > (int)C) nd = (int)C;
    for (int j = 0; j < nd; ++j) {
      const int id = mask_select(cand, sm_draw(s, C - (uint32_t)j), N, lane);
      cand &= ~bit_of(id, N, lane);
      if (j == 0) ep.dec0 = id;
      else ep.dec1 = id;
    }
    ep.nd = nd;
  }
  return ep;
}

__device__ __forceinline__ uint32_t pick(uint32_t w, uint32_t sp, int i, uint32_t bg) {
  return i < (int)(sp >> 24) ? (sp & 0xFFFFFFu) : (i < (int)(w >> 24) ? (w & 0xFFFFFFu) : bg);
}

struct U3 {
  uint32_t a, b, c;
};

__device__ __forceinline__ void store12(uint8_t* p, uint32_t a, uint32_t b, uint32_t c, int nt) {
  U3* q = reinterpret_cast<U3*>(p);
  if (nt) {
    __builtin_nontemporal_store(a, &q->a);
    __builtin_nontemporal_store(b, &q->b);
    __builtin_nontemporal_store(c, &q->c);
  } else {
    *q = U3{a, b, c};
  }
}

struct ColDbg {
  int32_t hit, side;
  float t;
  int32_t cell;
};

// Render the env's current state into its frame (and debug records).
__device__ void render_env(const DevCfg& cf, const DevIo& io, int64_t obs_off, int env, int lane,
                          uint8_t* lmap, uint32_t* lcol, float x, float y, float th, int goal,
                          int door, int key, uint32_t fl, int nd, int dec0, int dec1) {
  const int N = cf.side, H = cf.obs_h, W = cf.obs_w, K = cf.n_colors;
  if (door >= 0 && !(fl & FL_DOOR_OPEN) && lane == 0) lmap[door] = 2;
  wave_sync();
  float sn, cs;
  sincosf(th, &sn, &cs);
  const float tanH = cf.tanH;
  const float px = -sn * tanH, py = cs * tanH;

  // Sprites in fixed slots, in painting-index order: key, goal, decor 0, decor 1.
  // Empty slots are skipped, which keeps the relative order of the active ones.
  const int sid[4] = {(key >= 0 && !(fl & FL_KEY)) ? key : -1, (cf.goal_sprite && goal >= 0) ? goal : -1,
                      nd > 0 ? dec0 : -1, nd > 1 ? dec1 : -1};
  const uint32_t srgb[4] = {kKeyRgb, kGoalRgb, kDecorRgb, kDecorRgb};
  float sY[4], sU[4], sHW[4], sHS[4];
  bool sVis[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int id = sid[j] < 0 ? 0 : sid[j];
    const float dx = ((float)(id % N) + 0.5f) - x;
    const float dy = ((float)(id / N) + 0.5f) - y;
    const float tY = dx * cs + dy * sn;
    const float tX = dy * cs - dx * sn;
    const float den = tanH * tY;
    sY[j] = tY;
    sVis[j] = sid[j] >= 0 && tY > 0.05f;
    sU[j] = (0.5f * (float)W) * (1.0f + tX / den);
    sHW[j] = (0.5f * (float)W) * 0.25f / den;
    sHS[j] = (float)H * 0.25f / tY;
  }

  const int ix0 = (int)floorf(x), iy0 = (int)floorf(y);
  const float halfH = (float)(H >> 1);
  const float INF = __builtin_huge_valf();
  for (int col = lane; col < W; col += 64) {
    const float camX = (float)(2 * col + 1 - W) / (float)W;
    const float rx = fmaf(camX, px, cs);
    const float ry = fmaf(camX, py, sn);
    int ix = ix0, iy = iy0;
    const int stx = rx > 0.f ? 1 : -1, sty = ry > 0.f ? 1 : -1;
    float Xn = (float)(rx > 0.f ? ix + 1 : ix);
    float Yn = (float)(ry > 0.f ? iy + 1 : iy);
    const float ivx = 1.0f / rx, ivy = 1.0f / ry;
    float tx = rx != 0.f ? (Xn - x) * ivx : INF;
    float ty = ry != 0.f ? (Yn - y) * ivy : INF;
    float tst = INF;
    int side = 0, hit = -1, cell = 1;
    for (int it = 0; it < 4 * N + 8; ++it) {
      if (tx < ty) {
        ix += stx;
        tst = tx;
        side = 0;
        Xn += (float)stx;
        tx = (Xn - x) * ivx;
      } else {
        iy += sty;
        tst = ty;
        side = 1;
        Yn += (float)sty;
        ty = (Yn - y) * ivy;
      }
      if ((unsigned)ix >= (unsigned)N || (unsigned)iy >= (unsigned)N) break;
      const int v = lmap[iy * N + ix];
      if (v) {
        hit = iy * N + ix;
        cell = v;
        break;
      }
    }
    uint32_t wc = (cell == 2) ? kDoor : kPalette[(hit < 0 ? 0 : hit) % K];
    if (side) wc = (wc >> 1) & 0x7F7F7Fu;
    const float hh = (float)H / (2.0f * tst);
    const uint32_t wcount = (uint32_t)fminf(fmaxf(ceilf(hh - 0.5f), 0.f), halfH);
    // nearest covering sprite; on equal depth the later slot wins (painted last)
    float bestY = INF, bestHS = 0.f;
    uint32_t bestRgb = 0u;
    bool any = false;
    const float cc = (float)col + 0.5f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (sVis[j] && fabsf(cc - sU[j]) < sHW[j] && sY[j] < tst && sY[j] <= bestY) {
        bestY = sY[j];
        bestHS = sHS[j];
        bestRgb = srgb[j];
        any = true;
      }
    }
    uint32_t srec = 0u;
    if (any) {
      const uint32_t scount = (uint32_t)fminf(fmaxf(ceilf(bestHS - 0.5f), 0.f), halfH);
      srec = bestRgb | (scount << 24);
    }
    lcol[2 * col] = wc | (wcount << 24);
    lcol[2 * col + 1] = srec;
    if (io.dbg) {
      ColDbg* d = reinterpret_cast<ColDbg*>(io.dbg) + (int64_t)env * io.dbg_stride + col;
      *d = ColDbg{hit, side, tst, cell};
    }
  }
  wave_sync();
  if (!io.obs) return;

  uint8_t* base = io.obs + obs_off;
  const int Q = W >> 2, G = H * Q, H2 = H >> 1;
  int row = lane / Q, cq = lane - row * Q;
  const int dr = 64 / Q, dq = 64 - dr * Q;
  const uint4* l4 = reinterpret_cast<const uint4*>(lcol);
  const int nt = io.store_mode;
  for (int g = lane; g < G; g += 64) {
    const uint4 A = l4[2 * cq], B = l4[2 * cq + 1];
    const bool upper = row < H2;
    const int i = upper ? (H2 - 1 - row) : (row - H2);
    const uint32_t bg = upper ? kCeil : kFloor;
    const uint32_t p0 = pick(A.x, A.y, i, bg), p1 = pick(A.z, A.w, i, bg);
    const uint32_t p2 = pick(B.x, B.y, i, bg), p3 = pick(B.z, B.w, i, bg);
    store12(base + 12 * (int64_t)g, p0 | (p1 << 24), (p1 >> 8) | (p2 << 16), (p2 >> 16) | (p3 << 8),
            nt);
    row += dr;
    cq += dq;
    if (cq >= Q) {
      cq -= Q;
      ++row;
    }
  }
}

// The whole per-env pipeline.  All lanes run the uniform parts redundantly;
// lane 0 writes the scalar results with vector stores.
__device__ void process_env(const DevState& S, const DevIo& io, int env, int lane, uint8_t* lmap,
                            uint32_t* lcol) {
  const DevCfg cf = S.cfgs[S.cfg_idx[env]];
  const int N = cf.side, NN = N * N;
  const uint32_t* gm = reinterpret_cast<const uint32_t*>(S.maps + S.map_off[env]);
  uint32_t* lm32 = reinterpret_cast<uint32_t*>(lmap);
  for (int i = lane; i < ((NN + 3) >> 2); i += 64) lm32[i] = gm[i];

  float x = S.x[env], y = S.y[env], th = S.th[env];
  uint32_t t = S.t[env], ep = S.ep[env];
  int goal = S.goal[env], door = S.door[env], key = S.key[env];
  int dec0 = S.decor[2 * env], dec1 = S.decor[2 * env + 1];
  uint32_t fl = S.flags[env];
  int nd = S.ndecor[env];
  const uint64_t seed = S.seed[env];
  wave_sync();

  const int mode = io.mode;
  float reward = 0.f;
  uint32_t ev = 0;
  bool done = false;
  if (mode == MODE_STEP) {
    const int a = io.act[env];
    float sn, cs;
    sincosf(th, &sn, &cs);
    float mvx = 0.f, mvy = 0.f, dth = 0.f;
    if (a >= cf.n_actions) {
      ev |= EV_INVALID;
    } else if (cf.n_actions == 4) {
      if (a == 0) { mvx = cs; mvy = sn; }
      else if (a == 1) { mvx = -cs; mvy = -sn; }
      else if (a == 2) dth = -cf.turn;
      else dth = cf.turn;
    } else {
      if (a == 0) { mvx = cs; mvy = sn; }
      else if (a == 1) { mvx = -cs; mvy = -sn; }
      else if (a == 2) { mvx = sn; mvy = -cs; }
      else if (a == 3) { mvx = -sn; mvy = cs; }
      else if (a == 4) dth = -cf.turn;
      else dth = cf.turn;
    }
    if (dth != 0.f) {
      float t2 = th + dth;
      if (t2 < 0.f) t2 += kTwoPiF;
      else if (t2 >= kTwoPiF) t2 -= kTwoPiF;
      th = t2;
    }
    const float mx = cf.move * mvx, my = cf.move * mvy;
    const bool dclosed = door >= 0 && !(fl & FL_DOOR_OPEN);
    auto blocks = [&](int tx, int ty) -> bool {
      if ((unsigned)tx >= (unsigned)N || (unsigned)ty >= (unsigned)N) return true;
      const int id = ty * N + tx;
      return lmap[id] != 0 || (dclosed && id == door);
    };
    if (mx != 0.f) {
      const float nx = x + mx;
      if (!blocks((int)floorf(nx), (int)floorf(y))) x = nx;
      else ev |= EV_BLOCKED_X;
    }
    if (my != 0.f) {
      const float ny = y + my;
      if (!blocks((int)floorf(x), (int)floorf(ny))) y = ny;
      else ev |= EV_BLOCKED_Y;
    }
    if (key >= 0 && !(fl & FL_KEY)) {
      const float dx = x - ((float)(key % N) + 0.5f);
      const float dy = y - ((float)(key / N) + 0.5f);
      if (dx * dx + dy * dy < cf.pr2) {
        fl |= FL_KEY | FL_DOOR_OPEN;
        reward += cf.r_key;
        ev |= EV_KEY;
      }
    }
    bool term = false;
    if (goal >= 0 && (int)floorf(x) == goal % N && (int)floorf(y) == goal / N) {
      reward += cf.r_goal;
      term = true;
      ev |= EV_GOAL;
    }
    t += 1;
    const bool trunc = t >= (uint32_t)cf.cap;
    if (trunc) ev |= EV_TRUNC;
    done = term || trunc;
  }
  if (mode == MODE_RESET || done) {
    const uint32_t e = (mode == MODE_RESET) ? 0u : ep + 1u;
    const Episode n = episode_reset(cf, lmap, seed, e, lane);
    x = n.x;
    y = n.y;
    th = n.th;
    goal = n.goal;
    door = n.door;
    key = n.key;
    nd = n.nd;
    dec0 = n.dec0;
    dec1 = n.dec1;
    t = 0;
    ep = e;
    fl = 0;
    if (done) ev |= EV_RESET;
  }
  if (io.obs || io.dbg)
    render_env(cf, io, S.obs_off[env], env, lane, lmap, lcol, x, y, th, goal, door, key, fl, nd,
               dec0, dec1);
  if (lane == 0 && mode != MODE_RENDER) {
    S.x[env] = x;
    S.y[env] = y;
    S.th[env] = th;
    S.t[env] = t;
    S.ep[env] = ep;
    S.goal[env] = goal;
    S.door[env] = door;
    S.key[env] = key;
    S.decor[2 * env] = dec0;
    S.decor[2 * env + 1] = dec1;
    S.flags[env] = (uint8_t)fl;
    S.ndecor[env] = (uint8_t)nd;
    S.events[env] = (uint8_t)ev;
    if (ev & EV_INVALID) S.invalid[env] += 1u;
    if (mode == MODE_STEP) {
      io.rew[env] = reward;
      io.done[env] = done ? 1 : 0;
    }
  }
}

// I/O of this launch: given by value, or (graph replays) from the descriptor.
__device__ __forceinline__ DevIo io_of(const DevIo& io, const RolloutDesc* rd, int t) {
  if (!rd) return io;
  DevIo r = io;
  const int64_t n = rd->n;
  r.act = rd->act + (int64_t)t * n;
  r.obs = rd->obs + (int64_t)t * rd->obs_stride;
  r.rew = rd->rew + (int64_t)t * n;
  r.done = rd->done + (int64_t)t * n;
  r.store_mode = rd->store_mode;
  return r;
}

template <int MAXN, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_plain(DevState S, DevIo io0, const RolloutDesc* rd,
                                                    int t) {
  __shared__ __align__(16) uint8_t smap[WPB][MAXN * MAXN];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int env = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WPB + w);
  if (env >= S.n) return;
  const DevIo io = io_of(io0, rd, t);
  process_env(S, io, env, lane, smap[w], scol[w]);
}

// Persistent form: each wave pulls env indices (costliest first) from the
// workspace queue until it runs dry.  The last wave to leave zeroes the queue
// for the next launch, so consecutive launches and graph replays need no reset.
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void k_persist(DevState S, DevIo io0, const RolloutDesc* rd,
                                                      int t, int total_waves) {
  __shared__ __align__(16) uint8_t smap[WPB][kMaxSide * kMaxSide];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  WsHeader* h = S.hdr;
  const DevIo io = io_of(io0, rd, t);
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(&h->queue, 1u);
    item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
    if (item >= (uint32_t)S.n) break;
    const int env = __builtin_amdgcn_readfirstlane(S.order[item]);
    process_env(S, io, env, lane, smap[w], scol[w]);
  }
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(&h->exited, 1u) == (uint32_t)total_waves - 1u) {
      atomicExch(&h->queue, 0u);
      atomicExch(&h->exited, 0u);
    }
  }
}

// Serving form: work items span several clients' batches.
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void k_serve(const DevState* states, const DevIo* ios,
                                                    const ServeItem* items, int n_items,
                                                    uint32_t* counters, int total_waves) {
  __shared__ __align__(16) uint8_t smap[WPB][kMaxSide * kMaxSide];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(&counters[0], 1u);
    item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
    if (item >= (uint32_t)n_items) break;
    const int d = __builtin_amdgcn_readfirstlane(items[item].desc);
    const int env = __builtin_amdgcn_readfirstlane(items[item].env);
    const DevState S = states[d];
    const DevIo io = ios[d];
    process_env(S, io, env, lane, smap[w], scol[w]);
  }
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1u) == (uint32_t)total_waves - 1u) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

__global__ void k_set_desc(RolloutDesc* rd, RolloutDesc v) {
  if (threadIdx.x == 0) *rd = v;
}

template <int MAXN>
int launch_plain_n(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t, int wpb,
                   hipStream_t st) {
  const int grid = (s.n + wpb - 1) / wpb;
  switch (wpb) {
    case 1: hipLaunchKernelGGL((k_plain<MAXN, 1>), dim3(grid), dim3(64), 0, st, s, io, rd, t); break;
    case 2: hipLaunchKernelGGL((k_plain<MAXN, 2>), dim3(grid), dim3(128), 0, st, s, io, rd, t); break;
    case 4: hipLaunchKernelGGL((k_plain<MAXN, 4>), dim3(grid), dim3(256), 0, st, s, io, rd, t); break;
    case 8: hipLaunchKernelGGL((k_plain<MAXN, 8>), dim3(grid), dim3(512), 0, st, s, io, rd, t); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

}  // namespace

int launch_set_desc(RolloutDesc* rd_dev, const RolloutDesc& value, void* stream) {
  hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), rd_dev,
                     value);
  return (int)hipGetLastError();
}

int launch_batch(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t,
                 const LaunchCfg& lc, int max_side, int n_cu, void* stream) {
  if (s.n <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int wpb = lc.waves_per_group;
  if (lc.form == 0) {
    if (max_side <= 16) return launch_plain_n<16>(s, io, rd, t, wpb, st);
    if (max_side <= 32) return launch_plain_n<32>(s, io, rd, t, wpb, st);
    return launch_plain_n<64>(s, io, rd, t, wpb, st);
  }
  int groups = n_cu * lc.groups_per_cu;
  const int need = (s.n + wpb - 1) / wpb;
  if (groups > need) groups = need;
  if (groups < 1) groups = 1;
  const int waves = groups * wpb;
  switch (wpb) {
    case 1: hipLaunchKernelGGL((k_persist<1>), dim3(groups), dim3(64), 0, st, s, io, rd, t, waves); break;
    case 2: hipLaunchKernelGGL((k_persist<2>), dim3(groups), dim3(128), 0, st, s, io, rd, t, waves); break;
    case 4: hipLaunchKernelGGL((k_persist<4>), dim3(groups), dim3(256), 0, st, s, io, rd, t, waves); break;
    case 8: hipLaunchKernelGGL((k_persist<8>), dim3(groups), dim3(512), 0, st, s, io, rd, t, waves); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

int launch_serve(const DevState* states_dev, const DevIo* ios_dev, const ServeItem* items_dev,
                 int n_items, uint32_t* counters_dev, int waves_per_group, int n_groups,
                 void* stream) {
  if (n_items <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int wpb = waves_per_group;
  const int waves = n_groups * wpb;
  switch (wpb) {
    case 1: hipLaunchKernelGGL((k_serve<1>), dim3(n_groups), dim3(64), 0, st, states_dev, ios_dev, items_dev, n_items, counters_dev, waves); break;
    case 2: hipLaunchKernelGGL((k_serve<2>), dim3(n_groups), dim3(128), 0, st, states_dev, ios_dev, items_dev, n_items, counters_dev, waves); break;
    case 4: hipLaunchKernelGGL((k_serve<4>), dim3(n_groups), dim3(256), 0, st, states_dev, ios_dev, items_dev, n_items, counters_dev, waves); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

const char* kernel_error_string(int code) { return hipGetErrorString((hipError_t)code); }

}  // namespace jx
