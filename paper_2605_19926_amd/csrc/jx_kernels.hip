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
//      contiguous bytes per store instruction.  The training-buffer formats
//      (NCHW planes, byte / 255 as bfloat16 or float32) expand the same records
//      into converted elements.
// Nothing here is a dense contraction, so there is no MFMA; the bound is the
// HBM write of the frames and the vector ALU of the span expansion.
#include <hip/hip_runtime.h>

#include <mutex>

#include "jx_internal.h"

namespace jx {

namespace {

constexpr uint32_t rgb(uint32_t r, uint32_t g, uint32_t b) { return r | (g << 8) | (b << 16); }

// Colours of this library (the paper draws flat colours without assets).  The
// table is copied into each workgroup's LDS at kernel start: an indexed lookup
// in LDS costs no global load, and a global load inside a step loop would
// wait for every frame store the wave has in flight.
constexpr int kColorWords = 32;
constexpr int kClrPalette = 0;  // 8 wall colours, indexed by tile id mod K
constexpr int kClrWall9 = 8;    // ASCII maps: walls '1'..'9'
constexpr int kClrDoor = 17;    // ASCII maps: doors by type (8 slots; 5 types)
constexpr uint32_t kColorTable[kColorWords] = {
    rgb(180, 40, 40), rgb(40, 160, 40),  rgb(40, 60, 180),  rgb(190, 170, 40),
    rgb(150, 40, 170), rgb(40, 160, 170), rgb(200, 110, 30), rgb(150, 150, 150),
    rgb(180, 40, 40), rgb(40, 160, 40),  rgb(40, 60, 180),  rgb(190, 170, 40),
    rgb(150, 40, 170), rgb(40, 160, 170), rgb(200, 110, 30), rgb(150, 150, 150),
    rgb(230, 230, 230),
    rgb(120, 0, 0), rgb(0, 30, 130), rgb(140, 120, 0), rgb(70, 110, 230), rgb(230, 200, 60),
    rgb(120, 0, 0), rgb(120, 0, 0), rgb(120, 0, 0)};
// ASCII maps: key billboards by colour (red, blue, yellow)
constexpr uint32_t kAKeyRgb[3] = {rgb(255, 40, 40), rgb(40, 110, 255), rgb(255, 200, 40)};
// Tile bytes (layout sources): low nibble wall class (1 default, 2..10 '1'..'9'),
// bit 7 door (type in bits 4..6, index in 0..3), bits 5/6 spawn/goal candidates
// on floor tiles.
constexpr uint32_t kTileDoor = 0x80u, kTileSpawn = 0x20u, kTileGoal = 0x40u;
constexpr uint32_t kDoorBlueUnlocked = 3u, kDoorYellowUnlocked = 4u;

__device__ __forceinline__ void stage_colors(uint32_t* lclr) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kColorWords; ++i) lclr[i] = kColorTable[i];
  }
  __syncthreads();
}

// Training-buffer formats (fmt = layout * 3 + dtype): the floating types hold
// byte / 255 rounded to nearest-even.  The quotient is an IEEE division in
// float (correctly rounded); bfloat16 rounds that float to nearest-even, which
// equals rounding the exact quotient directly because float carries more than
// twice bfloat16's 8 significant bits plus two.
template <int DT>
__device__ __forceinline__ uint32_t norm_entry(uint32_t b) {
  const uint32_t u = __float_as_uint((float)b / 255.0f);
  if (DT == 2) return u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// Colour table and, for the floating formats, the byte -> element table
// (256 words), both into the workgroup's LDS.
template <int FMT>
__device__ __forceinline__ void stage_tables(uint32_t* lclr, uint32_t* lcvt) {
  if (FMT % 3 != 0)
    for (int i = (int)threadIdx.x; i < 256; i += (int)blockDim.x) lcvt[i] = norm_entry<FMT % 3>((uint32_t)i);
  stage_colors(lclr);
}
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
__device__ __forceinline__ uint32_t uniform_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ float uniform_f(float v) {
  return __uint_as_float((uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(v)));
}
__device__ __forceinline__ double uniform_d(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = uniform_u((uint32_t)b), hi = uniform_u((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

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
// ASC: the batch may hold ASCII maps (else that code is compiled out).
template <bool ASC>
__device__ Episode episode_reset(const DevCfg& cf, const uint8_t* lmap, uint64_t seed, uint32_t e,
                                 int lane) {
  const int N = cf.side;
  uint64_t s = seed ^ sm_mix((uint64_t)e + 1ull);
  // lane y: row y as bit masks of floor tiles, spawn and goal candidates, doors
  uint64_t freem = 0ull, spawnm = 0ull, goalm = 0ull, doorm = 0ull;
  if (lane < N) {
    const uint8_t* row = lmap + lane * N;
    for (int xx = 0; xx < N; ++xx) {
      const uint32_t v = row[xx];
      const uint64_t bit = 1ull << xx;
      if ((v & 0x8Fu) == 0u) {
        freem |= bit;
        if (v & kTileSpawn) spawnm |= bit;
        if (v & kTileGoal) goalm |= bit;
      }
      if (v & kTileDoor) doorm |= bit;
    }
  }
  const uint32_t n_free = mask_count(freem, lane);
  Episode ep;
  if (ASC && cf.ascii) {
    // ASCII maps: spawn among the spawn candidates (every floor tile if none),
    // heading, goal among the goal candidates (else the farthest tile from the
    // spawn with doors passable, smallest id); keys and doors come from the map
    const uint32_t n_s = mask_count(spawnm, lane);
    const int spawn = n_s ? mask_select(spawnm, sm_draw(s, n_s), N, lane)
                          : mask_select(freem, sm_draw(s, n_free), N, lane);
    const uint32_t k24 = (uint32_t)(sm_next(s) >> 40);
    ep.th = (float)k24 * (kTwoPiF * 0x1p-24f);
    ep.x = (float)(spawn % N) + 0.5f;
    ep.y = (float)(spawn / N) + 0.5f;
    const uint32_t n_g = mask_count(goalm, lane);
    ep.goal = n_g ? mask_select(goalm, sm_draw(s, n_g), N, lane)
                  : mask_first(bfs_rows(freem | doorm, spawn, N, -1, lane).frontier, N);
    ep.door = ep.key = -1;
    ep.nd = 0;
    ep.dec0 = ep.dec1 = -1;
    return ep;
  }
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

typedef __attribute__((address_space(1))) uint32_t GlobalU32;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x2 GlobalU32x2;
typedef __attribute__((address_space(1))) u32x4 GlobalU32x4;

// 12 bytes (4 RGB pixels) to global memory; non-temporal on request.
__device__ __forceinline__ void store12(uint8_t* p, uint32_t a, uint32_t b, uint32_t c, int nt) {
  if (nt) {
    GlobalU32* q = (GlobalU32*)p;
    __builtin_nontemporal_store(a, q);
    __builtin_nontemporal_store(b, q + 1);
    __builtin_nontemporal_store(c, q + 2);
  } else {
    GlobalU32* q = (GlobalU32*)p;
    q[0] = a;
    q[1] = b;
    q[2] = c;
  }
}

// Pixel colours of one column group (4 columns), byte-parallel.  A column's
// span record is (wall rgb | cov << 24, sprite rgb | sc << 24), where rows at
// distance i < sc from the horizon show the sprite, sc <= i < cov the wall and
// the rest ceiling (above) or floor (below).  The group keeps:
//   pw, ps  the 4 wall / sprite colours packed as 12 frame bytes (3 dwords);
//   cova/covb, sca/scb  cov and sc of pixels (0,1) / (2,3) in bytes 1 and 3,
//           biased by 0x7F, so that subtracting i from both bytes at once
//           leaves the byte's sign bit set exactly when i < count (0x7F + count
//           - i stays in [0x40, 0xBF] for counts and i up to 64: no carries);
//   any     the largest cov: rows at i >= any are background in this group.
struct ColGroup {
  uint32_t pw[3], ps[3];
  uint32_t cova, covb, sca, scb;
  uint32_t any;
};

// v_perm_b32 selectors: bytes 0-3 of {hi, lo} come from lo, 4-7 from hi;
// 8..11 replicate the sign bit of bytes 1, 3, 5, 7; 12 gives 0x00.
constexpr uint32_t kSelPack0 = 0x04020100u;  // lo.b0 lo.b1 lo.b2 hi.b0
constexpr uint32_t kSelPack1 = 0x05040201u;  // lo.b1 lo.b2 hi.b0 hi.b1
constexpr uint32_t kSelPack2 = 0x06050402u;  // lo.b2 hi.b0 hi.b1 hi.b2
constexpr uint32_t kSelCount = 0x070C030Cu;  // 0, lo.b3, 0, hi.b3
constexpr uint32_t kSelMask0 = 0x09080808u;  // pixel 0 x3, pixel 1
constexpr uint32_t kSelMask1 = 0x0A0A0909u;  // pixel 1 x2, pixel 2 x2
constexpr uint32_t kSelMask2 = 0x0B0B0B0Au;  // pixel 2, pixel 3 x3
constexpr uint32_t kCountBias = 0x7F007F00u;
constexpr uint32_t kRowStep = 0x01000100u;    // i in bytes 1 and 3

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t bitsel(uint32_t m, uint32_t a, uint32_t b) {
  return (m & a) | (~m & b);
}

__device__ __forceinline__ ColGroup col_group(const uint32_t* lcol, int cq) {
  const uint4* l4 = reinterpret_cast<const uint4*>(lcol);
  const uint4 A = l4[2 * cq], B = l4[2 * cq + 1];
  // A = (w0, s0, w1, s1), B = (w2, s2, w3, s3)
  ColGroup g;
  g.pw[0] = perm(A.z, A.x, kSelPack0);
  g.pw[1] = perm(B.x, A.z, kSelPack1);
  g.pw[2] = perm(B.z, B.x, kSelPack2);
  g.ps[0] = perm(A.w, A.y, kSelPack0);
  g.ps[1] = perm(B.y, A.w, kSelPack1);
  g.ps[2] = perm(B.w, B.y, kSelPack2);
  g.cova = perm(A.z, A.x, kSelCount) + kCountBias;
  g.covb = perm(B.z, B.x, kSelCount) + kCountBias;
  g.sca = perm(A.w, A.y, kSelCount) + kCountBias;
  g.scb = perm(B.w, B.y, kSelCount) + kCountBias;
  const uint32_t a = max(A.x >> 24, A.z >> 24), b = max(B.x >> 24, B.z >> 24);
  g.any = max(a, b);
  return g;
}

// Crossings per batch of the DDA walk (one LDS round trip each).
constexpr int kDdaBatch = 4;

constexpr uint32_t kCeil3[3] = {kCeil | (kCeil << 24), (kCeil >> 8) | (kCeil << 16),
                                (kCeil >> 16) | (kCeil << 8)};
constexpr uint32_t kFloor3[3] = {kFloor | (kFloor << 24), (kFloor >> 8) | (kFloor << 16),
                                 (kFloor >> 16) | (kFloor << 8)};

// Writes the mirrored row pair at distance i (row H/2-1-i above, H/2+i below);
// ii = i * kRowStep.  When no lane of the wave has a wall or sprite pixel at
// its distance, the whole wave stores the constant ceiling and floor patterns.
__device__ __forceinline__ void emit_pair(const ColGroup& g, uint32_t i, uint32_t ii, uint8_t* up,
                                          uint8_t* dn, int nt) {
  if (__ballot(i < g.any) == 0ull) {
    store12(up, kCeil3[0], kCeil3[1], kCeil3[2], nt);
    store12(dn, kFloor3[0], kFloor3[1], kFloor3[2], nt);
    return;
  }
  const uint32_t ca = g.cova - ii, cb = g.covb - ii;  // sign bits: i < cov
  const uint32_t sa = g.sca - ii, sb = g.scb - ii;    // sign bits: i < sc
  const uint32_t m0 = perm(cb, ca, kSelMask0), m1 = perm(cb, ca, kSelMask1), m2 = perm(cb, ca, kSelMask2);
  const uint32_t x0 = bitsel(perm(sb, sa, kSelMask0), g.ps[0], g.pw[0]);
  const uint32_t x1 = bitsel(perm(sb, sa, kSelMask1), g.ps[1], g.pw[1]);
  const uint32_t x2 = bitsel(perm(sb, sa, kSelMask2), g.ps[2], g.pw[2]);
  store12(up, bitsel(m0, x0, kCeil3[0]), bitsel(m1, x1, kCeil3[1]), bitsel(m2, x2, kCeil3[2]), nt);
  store12(dn, bitsel(m0, x0, kFloor3[0]), bitsel(m1, x1, kFloor3[1]), bitsel(m2, x2, kFloor3[2]), nt);
}

// ---- training-buffer formats --------------------------------------------------
// Each lane still covers a group of 4 columns and one mirrored row pair per
// iteration; it emits kWords dwords per row: contiguous ([row][col][ch]) in
// NHWC, or kElem dwords into each of the 3 channel planes in NCHW.  Colour
// words hold converted elements; per-pixel masks come from the same biased
// counts as the byte format (v_perm sign-bit replication, selector 8 + pixel).
template <int FMT>
struct ObsFmt {
  static constexpr bool kPlanar = FMT >= 3;
  static constexpr int kDtype = FMT % 3;
  static constexpr int kElem = kDtype == 0 ? 1 : (kDtype == 1 ? 2 : 4);
  static constexpr int kWords = 3 * kElem;  // dwords per lane and row
  static constexpr int kPer = 4 / kElem;    // elements per dword
  // pixel (0..3 in the group) and channel of element j of dword k
  static constexpr int pixel(int k, int j) { return kPlanar ? (k % kElem) * kPer + j : (k * kPer + j) / 3; }
  static constexpr int channel(int k, int j) { return kPlanar ? k / kElem : (k * kPer + j) % 3; }
  static constexpr uint32_t mask_sel(int k) {
    uint32_t v = 0;
    for (int b = 0; b < 4; ++b) v |= (uint32_t)(8 + pixel(k, b / kElem)) << (8 * b);
    return v;
  }
  // byte strides of a frame row, a lane's column group and a channel plane
  __device__ static int64_t row_bytes(int W) { return (int64_t)(kPlanar ? W : 3 * W) * kElem; }
  static constexpr int kGroupBytes = (kPlanar ? 4 : 12) * kElem;
};
static_assert(ObsFmt<0>::mask_sel(0) == kSelMask0 && ObsFmt<0>::mask_sel(1) == kSelMask1 &&
                  ObsFmt<0>::mask_sel(2) == kSelMask2, "byte format masks");

template <int FMT>
struct ColGroupF {
  uint32_t pw[ObsFmt<FMT>::kWords], ps[ObsFmt<FMT>::kWords];
  uint32_t cova, covb, sca, scb;
  uint32_t any;
};

template <int DT>
__device__ __forceinline__ uint32_t elem_of(const uint32_t* lcvt, uint32_t b) {
  return DT == 0 ? b : lcvt[b];
}

// The kWords dwords of 4 pixels with colours c[0..3] (rgb words).
template <int FMT>
__device__ __forceinline__ void pack_words(const uint32_t* lcvt, const uint32_t (&c)[4],
                                           uint32_t (&out)[ObsFmt<FMT>::kWords]) {
  using F = ObsFmt<FMT>;
#pragma unroll
  for (int k = 0; k < F::kWords; ++k) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < F::kPer; ++j)
      v |= elem_of<F::kDtype>(lcvt, (c[F::pixel(k, j)] >> (8 * F::channel(k, j))) & 0xFFu) << (8 * F::kElem * j);
    out[k] = v;
  }
}

// The same words for one colour on all 4 pixels, at compile time (the
// constant evaluator divides with IEEE round-to-nearest-even, as the device
// does): the ceiling and floor then live in scalar registers.
template <int DT>
constexpr uint32_t norm_const(uint32_t b) {
  const uint32_t u = __builtin_bit_cast(uint32_t, (float)b / 255.0f);
  return DT == 0 ? b : (DT == 2 ? u : (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
template <int FMT>
struct BgWords {
  uint32_t w[ObsFmt<FMT>::kWords];
};
template <int FMT>
constexpr BgWords<FMT> bg_words(uint32_t rgb) {
  using F = ObsFmt<FMT>;
  BgWords<FMT> r{};
  for (int k = 0; k < F::kWords; ++k)
    for (int j = 0; j < F::kPer; ++j)
      r.w[k] |= norm_const<F::kDtype>((rgb >> (8 * F::channel(k, j))) & 0xFFu) << (8 * F::kElem * j);
  return r;
}

template <int FMT>
__device__ __forceinline__ ColGroupF<FMT> col_group_f(const uint32_t* lcol, const uint32_t* lcvt, int cq) {
  const uint4* l4 = reinterpret_cast<const uint4*>(lcol);
  const uint4 A = l4[2 * cq], B = l4[2 * cq + 1];
  ColGroupF<FMT> g;
  const uint32_t w[4] = {A.x, A.z, B.x, B.z}, sp[4] = {A.y, A.w, B.y, B.w};
  pack_words<FMT>(lcvt, w, g.pw);
  pack_words<FMT>(lcvt, sp, g.ps);
  g.cova = perm(A.z, A.x, kSelCount) + kCountBias;
  g.covb = perm(B.z, B.x, kSelCount) + kCountBias;
  g.sca = perm(A.w, A.y, kSelCount) + kCountBias;
  g.scb = perm(B.w, B.y, kSelCount) + kCountBias;
  const uint32_t a = max(A.x >> 24, A.z >> 24), b = max(B.x >> 24, B.z >> 24);
  g.any = max(a, b);
  return g;
}

// Stores one row's dwords of a lane: p is the lane's place in plane 0.
template <int FMT>
__device__ __forceinline__ void store_words(uint8_t* p, int64_t plane, const uint32_t (&v)[ObsFmt<FMT>::kWords],
                                            int nt) {
  using F = ObsFmt<FMT>;
  constexpr int runs = F::kPlanar ? 3 : 1, per = F::kPlanar ? F::kElem : F::kWords;
#pragma unroll
  for (int r = 0; r < runs; ++r) {
    GlobalU32* q = (GlobalU32*)(p + r * plane);
    if (nt) {
#pragma unroll
      for (int k = 0; k < per; ++k) __builtin_nontemporal_store(v[r * per + k], q + k);
    } else if (per % 4 == 0) {
#pragma unroll
      for (int k = 0; k < per; k += 4)
        *(GlobalU32x4*)(q + k) = u32x4{v[r * per + k], v[r * per + k + 1], v[r * per + k + 2], v[r * per + k + 3]};
    } else if (per % 2 == 0) {
#pragma unroll
      for (int k = 0; k < per; k += 2)
        *(GlobalU32x2*)(q + k) = u32x2{v[r * per + k], v[r * per + k + 1]};
    } else {
#pragma unroll
      for (int k = 0; k < per; ++k) q[k] = v[r * per + k];
    }
  }
}

// Mirrored row pair at distance i (as emit_pair) in format FMT; cw / fw are
// the ceiling / floor dwords.
template <int FMT>
__device__ __forceinline__ void emit_pair_f(const ColGroupF<FMT>& g, uint32_t i, uint32_t ii, uint8_t* up,
                                            uint8_t* dn, int64_t plane, int nt) {
  using F = ObsFmt<FMT>;
  constexpr BgWords<FMT> cb_ = bg_words<FMT>(kCeil), fb_ = bg_words<FMT>(kFloor);
  const uint32_t(&cw)[F::kWords] = cb_.w;
  const uint32_t(&fw)[F::kWords] = fb_.w;
  if (__ballot(i < g.any) == 0ull) {
    store_words<FMT>(up, plane, cw, nt);
    store_words<FMT>(dn, plane, fw, nt);
    return;
  }
  const uint32_t ca = g.cova - ii, cb = g.covb - ii;
  const uint32_t sa = g.sca - ii, sb = g.scb - ii;
  uint32_t u[F::kWords], d[F::kWords];
#pragma unroll
  for (int k = 0; k < F::kWords; ++k) {
    const uint32_t m = perm(cb, ca, F::mask_sel(k));
    const uint32_t x = bitsel(perm(sb, sa, F::mask_sel(k)), g.ps[k], g.pw[k]);
    u[k] = bitsel(m, x, cw[k]);
    d[k] = bitsel(m, x, fw[k]);
  }
  store_words<FMT>(up, plane, u, nt);
  store_words<FMT>(dn, plane, d, nt);
}

struct ColDbg {
  int32_t hit, side;
  float t;
  int32_t cell;
};

// Casts the env's columns and reduces each to a span record in lcol (and
// writes debug records when asked).
// dsn, dcs: sine and cosine of the heading in double.
template <bool ASC>
__device__ void render_columns(const DevCfg& cf, const DevIo& io, int env, int lane, uint8_t* lmap,
                               const uint32_t* lclr,
                               uint32_t* lcol, float x, float y, double dsn, double dcs, int goal,
                               int door, int key, uint32_t fl, int nd, int dec0, int dec1,
                               uint32_t doors, int ak0, int ak1, int ak2) {
  const int N = cf.side, H = cf.obs_h, W = cf.obs_w, K = cf.n_colors, S_lv = cf.shade_levels;
  // the shut locked door blocks rays like a wall (tile id `shut`, -1 if none)
  const int shut = (door >= 0 && !(fl & FL_DOOR_OPEN)) ? door : -1;
  const float sn = (float)dsn, cs = (float)dcs;
  // column c's ray offset along `right` is (2c + 1 - W) * q, q = tanH / W
  const double rq = (double)cf.ray_q_hi + (double)cf.ray_q_lo;

  // Sprites in fixed slots, in painting-index order: key, goal, decor 0, decor 1
  // (ASCII maps: red, blue, yellow key, goal).  Empty slots are skipped, which
  // keeps the relative order of the active ones.
  const bool asc = ASC && cf.ascii != 0;
  const int gsp = (cf.goal_sprite && goal >= 0) ? goal : -1;
  const int sid[4] = {asc ? ((ak0 >= 0 && !(fl & FL_AKEY0)) ? ak0 : -1) : ((key >= 0 && !(fl & FL_KEY)) ? key : -1),
                      asc ? ((ak1 >= 0 && !(fl & (FL_AKEY0 << 1))) ? ak1 : -1) : gsp,
                      asc ? ((ak2 >= 0 && !(fl & (FL_AKEY0 << 2))) ? ak2 : -1) : (nd > 0 ? dec0 : -1),
                      asc ? gsp : (nd > 1 ? dec1 : -1)};
  const uint32_t srgb[4] = {asc ? kAKeyRgb[0] : kKeyRgb, asc ? kAKeyRgb[1] : kGoalRgb,
                            asc ? kAKeyRgb[2] : kDecorRgb, asc ? kGoalRgb : kDecorRgb};
  float sY[4], sU[4], sHW[4], sHS[4];
  bool sVis[4];
  const float halfW = 0.5f * (float)W;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    sVis[j] = false;
    sY[j] = sU[j] = sHW[j] = sHS[j] = 0.f;
    if (sid[j] < 0) continue;  // uniform across the wave
    const int id = sid[j];
    const float dx = ((float)(id % N) + 0.5f) - x;
    const float dy = ((float)(id / N) + 0.5f) - y;
    const float tY = dx * cs + dy * sn;
    const float tX = dy * cs - dx * sn;
    const float inv = 1.0f / tY;             // one division per sprite
    const float q = inv * cf.inv_tanH;       // 1 / (tanH tY)
    sY[j] = tY;
    sVis[j] = tY > 0.05f;
    sU[j] = halfW * (1.0f + tX * q);
    sHW[j] = halfW * 0.25f * q;
    sHS[j] = (float)H * 0.25f * inv;
  }

  const int ix0 = (int)floorf(x), iy0 = (int)floorf(y);
  const float halfH = (float)(H >> 1);
  const float INF = __builtin_huge_valf();
  for (int col = lane; col < W; col += 64) {
    // The ray components are formed in double and rounded once: dir and the
    // column's offset along `right` can nearly cancel, and a float sum would
    // then lose most of the component's digits.  Each float component is
    // within half an ulp of the exact one.
    const double k = (double)(2 * col + 1 - W) * rq;
    const float rx = (float)fma(k, -dsn, dcs);
    const float ry = (float)fma(k, dcs, dsn);
    const int ix = ix0, iy = iy0;
    const int stx = rx > 0.f ? 1 : -1, sty = ry > 0.f ? 1 : -1;
    const float Xn = (float)(rx > 0.f ? ix + 1 : ix);
    const float Yn = (float)(ry > 0.f ? iy + 1 : iy);
    const float ivx = __builtin_amdgcn_rcpf(rx), ivy = __builtin_amdgcn_rcpf(ry);
    // Ray parameter of the k-th x / y grid line ahead: t0 + k |1/r|, one fused
    // multiply-add from the crossing count (Xn - x is exact, 1/r within an
    // ulp), so every crossing parameter is within a few float ulps of the
    // exact one whatever the walk's length.
    const float t0x = rx != 0.f ? (Xn - x) * ivx : INF;
    const float t0y = ry != 0.f ? (Yn - y) * ivy : INF;
    const float dtx = rx != 0.f ? fabsf(ivx) : 0.f, dty = ry != 0.f ? fabsf(ivy) : 0.f;
    float kx = 0.f, ky = 0.f;
    float tx = t0x, ty = t0y;
    float tst = INF;
    int side = 0, hit = -1, cell = 1;
    uint32_t hv = 1u;  // tile byte of the hit
    // Branch-free walk in batches: the sequence of tiles a ray crosses does
    // not depend on the map, only where it stops does.  Each batch computes
    // the next kDdaBatch crossings (one grid line each: the tile index moves
    // by +-1 on an x crossing, +-N on a y crossing, and that axis's crossing
    // count by one), issues their LDS reads together and keeps the first
    // blocking one, so a lane waits for one LDS round trip per batch instead
    // of one per crossing.  The border of
    // blocking tiles (checked on the host) stops every walk inside the map;
    // crossings past the stop are discarded and read a clamped address.
    const int dy = sty * N, NN = N * N;
    int id = iy * N + ix;
    const uint32_t last = (uint32_t)(NN - 1);
    bool found = false;
    for (int it = 0; it < 4 * N + 8 && !found; it += kDdaBatch) {
      int ids[kDdaBatch];
      float ts[kDdaBatch];
      bool sd[kDdaBatch];
#pragma unroll
      for (int u = 0; u < kDdaBatch; ++u) {
        const bool sx = tx < ty;
        ts[u] = sx ? tx : ty;
        sd[u] = !sx;
        id += sx ? stx : dy;
        kx = sx ? kx + 1.f : kx;
        ky = sx ? ky : ky + 1.f;
        tx = fmaf(kx, dtx, t0x);
        ty = fmaf(ky, dty, t0y);
        ids[u] = id;
      }
      // bit u: crossing u stops the walk (blocking tile, shut door, or off the map)
      uint32_t stop = 0;
      uint32_t vs[kDdaBatch];
#pragma unroll
      for (int u = 0; u < kDdaBatch; ++u) {
        const uint32_t uid = (uint32_t)ids[u];
        vs[u] = lmap[uid < last ? uid : last];
      }
      if (asc) {
        // map doors block while their bit in `doors` is clear
#pragma unroll
        for (int u = 0; u < kDdaBatch; ++u) {
          const uint32_t v = vs[u];
          const bool open = (v & kTileDoor) && ((doors >> (v & 15u)) & 1u);
          stop |= (uint32_t)((((v & 0x8Fu) != 0u) && !open) | ((uint32_t)ids[u] > last)) << u;
        }
      } else {
#pragma unroll
        for (int u = 0; u < kDdaBatch; ++u)
          stop |= (uint32_t)((vs[u] != 0u) | (ids[u] == shut) | ((uint32_t)ids[u] > last)) << u;
      }
      tst = ts[kDdaBatch - 1];  // kept only if nothing in the batch stops the walk
      side = sd[kDdaBatch - 1] ? 1 : 0;
      if (stop) {
        int sid_ = ids[kDdaBatch - 1];
        uint32_t sv = vs[kDdaBatch - 1];
#pragma unroll
        for (int u = kDdaBatch - 2; u >= 0; --u) {  // the earliest stop wins
          const bool b = (stop >> u) & 1u;
          tst = b ? ts[u] : tst;
          side = b ? (sd[u] ? 1 : 0) : side;
          sid_ = b ? ids[u] : sid_;
          sv = b ? vs[u] : sv;
        }
        found = true;
        const bool out = (uint32_t)sid_ > last;
        hit = out ? -1 : sid_;
        hv = out ? 1u : sv;
        cell = (!out && (sid_ == shut || (hv & kTileDoor))) ? 2 : 1;
      }
    }
    uint32_t wc;
    const uint32_t wcls = hv & 15u;
    if (asc && (hv & kTileDoor)) wc = lclr[kClrDoor + ((hv >> 4) & 7u)];
    else if (cell == 2) wc = kDoor;
    else if (asc && wcls >= 2u && wcls <= 10u) wc = lclr[kClrWall9 + wcls - 2u];
    else wc = lclr[kClrPalette + (hit < 0 ? 0 : hit) % K];
    if (side) wc = (wc >> 1) & 0x7F7F7Fu;
    if (S_lv > 0) {
      // distance shading: level l = min(floor(t* S / D), S - 1), each channel
      // scaled by (S - l) / S and rounded down; the division by S (numerators
      // below 4096) is a multiply by ceil(2^16 / S) and a shift
      const int lv = min((int)floorf(tst * cf.shade_scale), S_lv - 1);
      const uint32_t f = (uint32_t)(S_lv - lv), m = cf.shade_mul;
      const uint32_t r = ((wc & 0xFFu) * f * m) >> 16;
      const uint32_t g = (((wc >> 8) & 0xFFu) * f * m) >> 16;
      const uint32_t b = (((wc >> 16) & 0xFFu) * f * m) >> 16;
      wc = r | (g << 8) | (b << 16);
    }
    const float hh = halfH * __builtin_amdgcn_rcpf(tst);
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
    uint32_t srec = 0u, scount = 0u;
    if (any) {
      scount = (uint32_t)fminf(fmaxf(ceilf(bestHS - 0.5f), 0.f), halfH);
      srec = bestRgb | (scount << 24);
    }
    // span record: wall colour with the covered half-height (wall or sprite),
    // sprite colour with the sprite's half-height
    lcol[2 * col] = wc | ((wcount > scount ? wcount : scount) << 24);
    lcol[2 * col + 1] = srec;
    if (io.dbg) {
      ColDbg* d = reinterpret_cast<ColDbg*>(io.dbg) + (int64_t)env * io.dbg_stride + col;
      *d = ColDbg{hit, side, tst, cell};
    }
  }
  wave_sync();
}

// s_waitcnt immediate: vector-memory count 4, the other counters untouched.
// After each row pair a wave waits until at most 4 of its stores (two row
// pairs) are in flight: on the 4096-env rollout the HBM write stream measured
// about 1% faster with this bound than with the step-level bound alone (and
// 2% slower with 8 or 12 in flight at the step level).
constexpr int kWaitTwoPairs = 0x0F74;

// Expands the span records into the frame, one mirrored row pair per lane and
// iteration: lane -> (column group cq, distance i from the horizon).  The
// wave's di * Q lanes cover di row pairs of every column group per iteration
// (Q = W / 4 groups, di = 64 / Q), so each lane's group is fixed.
template <int FMT>
__device__ void fill_frame_f(const uint32_t* lcol, const uint32_t* lcvt, uint8_t* base, int W, int H, int lane,
                             int nt, int part, int parts) {
  using F = ObsFmt<FMT>;
  const int Q = W >> 2, H2 = H >> 1;
  const int64_t rowb = F::row_bytes(W), plane = (int64_t)H * W * F::kElem;
  const int di = 64 / Q;
  const int cq = lane % Q;
  int i = lane / Q + part * di;
  if (lane < di * Q) {
    const ColGroupF<FMT> g = col_group_f<FMT>(lcol, lcvt, cq);
    uint8_t* up = base + (int64_t)(H2 - 1 - i) * rowb + F::kGroupBytes * cq;
    uint8_t* dn = base + (int64_t)(H2 + i) * rowb + F::kGroupBytes * cq;
    const int pdi = parts * di;
    const int64_t step = (int64_t)pdi * rowb;
    uint32_t ii = (uint32_t)i * kRowStep;
    const uint32_t dii = (uint32_t)pdi * kRowStep;
    for (; i < H2; i += pdi) {
      emit_pair_f<FMT>(g, (uint32_t)i, ii, up, dn, plane, nt);
      ii += dii;
      up -= step;
      dn += step;
    }
  }
}

template <int FMT>
__device__ void fill_frame(const uint32_t* lcol, const uint32_t* lcvt, uint8_t* base, int W, int H, int lane,
                           int nt, int part = 0, int parts = 1) {
  if constexpr (FMT != 0) {
    fill_frame_f<FMT>(lcol, lcvt, base, W, H, lane, nt, part, parts);
    return;
  }
  // lane -> (column group cq, first distance i); the wave's di * Q lanes
  // (all 64 when Q divides 64, 63 of them at W = 84) cover di row pairs of
  // every column group per iteration, so each lane's column group is fixed and
  // its records stay in registers.  When `parts` waves share the env, wave
  // `part` takes every parts-th block of di row pairs.
  const int Q = W >> 2, H2 = H >> 1;
  const int rowb = 3 * W;
  const int di = 64 / Q;
  const int cq = lane % Q;
  int i = lane / Q + part * di;
  if (lane < di * Q) {
    const ColGroup g = col_group(lcol, cq);
    uint8_t* up = base + (int64_t)(H2 - 1 - i) * rowb + 12 * cq;
    uint8_t* dn = base + (int64_t)(H2 + i) * rowb + 12 * cq;
    const int pdi = parts * di;
    const int64_t step = (int64_t)pdi * rowb;
    uint32_t ii = (uint32_t)i * kRowStep;
    const uint32_t dii = (uint32_t)pdi * kRowStep;
    for (; i < H2; i += pdi) {
      emit_pair(g, (uint32_t)i, ii, up, dn, nt);
      __builtin_amdgcn_s_waitcnt(kWaitTwoPairs);
      ii += dii;
      up -= step;
      dn += step;
    }
  }
}

// Everything one env-step produces, handed from the computing wave to the
// wave that writes it back (or kept by the same wave in the plain form).
struct EnvOut {
  int64_t obs_off;
  int env, W, H, mode;
  float x, y, th, reward;
  uint32_t t, ep, fl, nd, ev, done, doors;
  uint32_t prev;  // previous action beside the frame (n_actions: none)
  int goal, door, key, dec0, dec1;
  double sn, cs;  // sine and cosine of th, in double
};

// Inputs of one env-step, loaded ahead of use: the configuration and state
// (uniform, scalar loads) and this lane's share of the map's dwords.
template <int MAXN>
struct EnvIn {
  static constexpr int kMapWords = (MAXN * MAXN + 255) / 256;  // dwords per lane
  DevCfg cf;
  int env;
  float x, y, th;
  uint32_t t, ep, fl, doors;
  int goal, door, key, dec0, dec1, nd;
  int ak0, ak1, ak2;  // ASCII maps: key tiles (constant per env)
  uint64_t seed;
  double sn, cs;      // sine and cosine of th, in double
  uint32_t map[kMapWords];
};

template <int MAXN>
__device__ __forceinline__ void load_env(const DevState& S, int env, int lane, EnvIn<MAXN>& in) {
  in.env = env;
  in.cf = S.uniform ? S.ucfg : S.cfgs[S.cfg_idx[env]];
  const int NN = in.cf.side * in.cf.side;
  const uint8_t* mp = S.uniform ? S.maps + (int64_t)env * S.map_stride : S.maps + S.map_off[env];
  const uint32_t* gm = reinterpret_cast<const uint32_t*>(mp);
#pragma unroll
  for (int k = 0; k < EnvIn<MAXN>::kMapWords; ++k) {
    const int i = lane + 64 * k;
    in.map[k] = (i < ((NN + 3) >> 2)) ? gm[i] : 0u;
  }
  in.x = S.x[env];
  in.y = S.y[env];
  in.th = S.th[env];
  in.t = S.t[env];
  in.ep = S.ep[env];
  in.goal = S.goal[env];
  in.door = S.door[env];
  in.key = S.key[env];
  in.dec0 = S.decor[2 * env];
  in.dec1 = S.decor[2 * env + 1];
  in.fl = S.flags[env];
  in.nd = S.ndecor[env];
  in.seed = S.seed[env];
  in.doors = S.doors[env];
  in.ak0 = S.akey[3 * env];
  in.ak1 = S.akey[3 * env + 1];
  in.ak2 = S.akey[3 * env + 2];
  sincos((double)in.th, &in.sn, &in.cs);
}

// Bit mask of the map's locked doors of colour c (door type c), gathered by
// the whole wave from its LDS map.
__device__ uint32_t locked_doors_of(const uint8_t* lmap, int NN, uint32_t c, int lane) {
  uint32_t m = 0u;
  for (int i = lane; i < NN; i += 64) {
    const uint32_t v = lmap[i];
    if ((v & kTileDoor) && ((v >> 4) & 7u) == c) m |= 1u << (v & 15u);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m |= (uint32_t)__shfl_xor((int)m, off, 64);
  return m;
}

// Copies the env's layout words from registers into the wave's LDS map.  The
// LDS map is read-only afterwards (the shut door is tested separately), so a
// wave that keeps one env for several steps stages it once.
template <int MAXN>
__device__ __forceinline__ void stage_map(const EnvIn<MAXN>& in, int lane, uint8_t* lmap) {
  const int NN = in.cf.side * in.cf.side;
  uint32_t* lm32 = reinterpret_cast<uint32_t*>(lmap);
#pragma unroll
  for (int k = 0; k < EnvIn<MAXN>::kMapWords; ++k) {
    const int i = lane + 64 * k;
    if (i < ((NN + 3) >> 2)) lm32[i] = in.map[k];
  }
}

// Step, reset and column cast of one env from its loaded inputs: LDS and
// registers only, no global stores (so a wave doing only this never waits on
// outstanding stores).  All lanes run the uniform parts redundantly.
// STAGE: copy the layout into LDS first (else it is already there).
// action < 0: read this env's action from io.act.
template <int MAXN, bool STAGE, bool ASC>
__device__ void produce_env(const EnvIn<MAXN>& in, const DevState& S, const DevIo& io, int action,
                            int lane, uint8_t* lmap, const uint32_t* lclr, uint32_t* lcol, EnvOut& o) {
  const DevCfg& cf = in.cf;
  const int env = in.env;
  const int N = cf.side;
  if (STAGE) stage_map<MAXN>(in, lane, lmap);
  float x = in.x, y = in.y, th = in.th;
  uint32_t t = in.t, ep = in.ep;
  int goal = in.goal, door = in.door, key = in.key;
  int dec0 = in.dec0, dec1 = in.dec1;
  uint32_t fl = in.fl;
  uint32_t doors = in.doors;
  int nd = in.nd;
  const uint64_t seed = in.seed;
  wave_sync();

  const int mode = io.mode;
  float reward = 0.f;
  uint32_t ev = 0;
  bool done = false;
  // sine and cosine of the heading in double (from the env's inputs; they
  // are recomputed only when the heading changes)
  double dsn = in.sn, dcs = in.cs;
  const float sn = (float)dsn, cs = (float)dcs;
  bool heading_changed = false;
  uint32_t prev = (uint32_t)cf.n_actions;
  if (mode == MODE_STEP) {
    const int a = action >= 0 ? action : io.act[env];
    if (a < cf.n_actions) prev = (uint32_t)a;
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
      heading_changed = true;
    }
    const float mx = cf.move * mvx, my = cf.move * mvy;
    const bool dclosed = door >= 0 && !(fl & FL_DOOR_OPEN);
    auto blocks = [&](int tx, int ty) -> bool {
      if ((unsigned)tx >= (unsigned)N || (unsigned)ty >= (unsigned)N) return true;
      const int id = ty * N + tx;
      const uint32_t v = lmap[id];
      if (ASC && (v & kTileDoor)) return !((doors >> (v & 15u)) & 1u);  // map door: shut unless open
      return (v & 0x0Fu) != 0u || (dclosed && id == door);
    };
    // ASCII maps: walking into a shut unlocked door opens it (the move is refused)
    auto bump = [&](int tx, int ty) {
      if ((unsigned)tx >= (unsigned)N || (unsigned)ty >= (unsigned)N) return;
      const uint32_t v = lmap[ty * N + tx];
      const uint32_t type = (v >> 4) & 7u;
      if ((v & kTileDoor) && (type == kDoorBlueUnlocked || type == kDoorYellowUnlocked) &&
          !((doors >> (v & 15u)) & 1u)) {
        doors |= 1u << (v & 15u);
        ev |= EV_DOOR;
      }
    };
    if (mx != 0.f) {
      const float nx = x + mx;
      const int tx = (int)floorf(nx), ty = (int)floorf(y);
      if (!blocks(tx, ty)) {
        x = nx;
      } else {
        ev |= EV_BLOCKED_X;
        if (ASC) bump(tx, ty);
      }
    }
    if (my != 0.f) {
      const float ny = y + my;
      const int tx = (int)floorf(x), ty = (int)floorf(ny);
      if (!blocks(tx, ty)) {
        y = ny;
      } else {
        ev |= EV_BLOCKED_Y;
        if (ASC) bump(tx, ty);
      }
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
    if (ASC && cf.ascii) {
      // ASCII maps: picking up the key of colour c opens every locked door of colour c
      const int ak[3] = {in.ak0, in.ak1, in.ak2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (ak[c] < 0 || (fl & (FL_AKEY0 << c))) continue;
        const float dx = x - ((float)(ak[c] % N) + 0.5f);
        const float dy = y - ((float)(ak[c] / N) + 0.5f);
        if (dx * dx + dy * dy < cf.pr2) {
          fl |= FL_AKEY0 << c;
          reward += cf.r_key;
          ev |= EV_KEY;
          const uint32_t m = locked_doors_of(lmap, N * N, (uint32_t)c, lane);
          if (m & ~doors) ev |= EV_DOOR;
          doors |= m;
        }
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
    if (done) prev = (uint32_t)cf.n_actions;
  }
  if (mode == MODE_RESET || done) {
    const uint32_t e = (mode == MODE_RESET) ? 0u : ep + 1u;
    const Episode n = episode_reset<ASC>(cf, lmap, seed, e, lane);
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
    doors = 0u;
    if (done) ev |= EV_RESET;
    heading_changed = true;
  }
  if (heading_changed) sincos((double)th, &dsn, &dcs);
  if (io.obs || io.dbg)
    render_columns<ASC>(cf, io, env, lane, lmap, lclr, lcol, x, y, dsn, dcs, goal, door, key, fl, nd, dec0, dec1,
                   doors, in.ak0, in.ak1, in.ak2);
  o.obs_off = 0;  // set by the caller (obs_off_of), outside any step loop
  o.env = env;
  o.W = cf.obs_w;
  o.H = cf.obs_h;
  o.mode = mode;
  o.x = x;
  o.y = y;
  o.th = th;
  o.reward = reward;
  o.t = t;
  o.ep = ep;
  o.fl = fl;
  o.nd = (uint32_t)nd;
  o.ev = ev;
  o.done = done ? 1u : 0u;
  o.goal = goal;
  o.door = door;
  o.key = key;
  o.dec0 = dec0;
  o.dec1 = dec1;
  o.doors = doors;
  o.prev = prev;
  o.sn = dsn;
  o.cs = dcs;
}

// Scalar results of one env-step, stored by lane 0 with vector stores.
__device__ void write_back(const DevState& S, const DevIo& io, const EnvOut& o, int lane) {
  if (lane != 0 || o.mode == MODE_RENDER) return;
  const int env = o.env;
  S.x[env] = o.x;
  S.y[env] = o.y;
  S.th[env] = o.th;
  S.t[env] = o.t;
  S.ep[env] = o.ep;
  S.goal[env] = o.goal;
  S.door[env] = o.door;
  S.key[env] = o.key;
  S.decor[2 * env] = o.dec0;
  S.decor[2 * env + 1] = o.dec1;
  S.flags[env] = (uint8_t)o.fl;
  S.ndecor[env] = (uint8_t)o.nd;
  S.events[env] = (uint8_t)o.ev;
  S.doors[env] = o.doors;
  if (o.ev & EV_INVALID) S.invalid[env] += 1u;
  if (o.mode == MODE_STEP) {
    io.rew[env] = o.reward;
    io.done[env] = (uint8_t)o.done;
    if (io.prev) io.prev[env] = (uint8_t)o.prev;
  }
}

// Byte offset of env's frame in a step's observation buffer.
__device__ __forceinline__ int64_t obs_off_of(const DevState& S, int env) {
  return S.uniform ? (int64_t)env * S.obs_stride : S.obs_off[env];
}

// The whole per-env pipeline in one wave.
// part / parts: this wave is one of `parts` waves sharing the env; each runs
// the same step and cast, fills its share of the frame's row pairs, and only
// part 0 writes the state and the step's outputs.
template <int MAXN, bool ASC, int FMT>
__device__ __forceinline__ void process_env(const DevState& S, const DevIo& io, int env, int lane, uint8_t* lmap,
                            const uint32_t* lclr, const uint32_t* lcvt, uint32_t* lcol, int part = 0,
                            int parts = 1) {
  EnvIn<MAXN> in;
  load_env<MAXN>(S, env, lane, in);
  EnvOut o;
  produce_env<MAXN, true, ASC>(in, S, io, -1, lane, lmap, lclr, lcol, o);
  o.obs_off = obs_off_of(S, env);
  if (io.obs) fill_frame<FMT>(lcol, lcvt, io.obs + o.obs_off, o.W, o.H, lane, io.store_mode, part, parts);
  if (part == 0) write_back(S, io, o, lane);
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
  r.prev = rd->prev ? rd->prev + (int64_t)t * n : nullptr;
  r.store_mode = rd->store_mode;
  return r;
}

// wpe waves per env (1, 2 or 4): consecutive waves share an env.
template <int MAXN, int WPB, bool ASC, int FMT>
__global__ __launch_bounds__(64 * WPB) void k_plain(DevState S, DevIo io0, const RolloutDesc* rd,
                                                    int t, int wpe) {
  __shared__ __align__(16) uint8_t smap[WPB][MAXN * MAXN];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  __shared__ uint32_t sclr[kColorWords];
  __shared__ uint32_t scvt[FMT % 3 ? 256 : 1];
  stage_tables<FMT>(sclr, scvt);
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int gw = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WPB + w);
  const int env = gw / wpe, part = gw - env * wpe;
  if (env >= S.n) return;
  const DevIo io = io_of(io0, rd, t);
  process_env<MAXN, ASC, FMT>(S, io, env, lane, smap[w], sclr, scvt, scol[w], part, wpe);
}

// Work distribution of the persistent forms (word 0 of a queue's line counts
// claims, word 1 the waves that left it).  Items (positions in a work
// order) are split over up to 32 queues by position modulo the queue count; a
// workgroup serves queue blockIdx % nq (so each queue is served from one XCD),
// and the queues (one 128-byte line each) sit in different L2 channels: their
// atomics do not serialize on one address.  Each wave first takes one chunk statically, then claims further
// chunks with one atomic each.  Launch `seq` counts in counter set seq % 4 and
// clears set (seq + 1) % 4 for the next launch on the same stream.
struct QueueView {
  uint32_t* ctr;      // this queue's counter
  int q, nq;          // queue index and count
  int items;          // items in this queue
  int waves, wave;    // waves serving it and this wave's rank among them
  int chunk;
};

template <int WPB>
__device__ __forceinline__ QueueView queue_view(uint32_t* queues, uint32_t seq, int n_items, int w,
                                                int lane, int max_chunk = 1 << 30) {
  QueueView v;
  const int grid = (int)gridDim.x;
  v.nq = grid < kQueues ? grid : kQueues;
  v.q = (int)blockIdx.x % v.nq;
  const int slot = (int)(seq % kQueueSlots);
  v.ctr = queues + (slot * kQueues + v.q) * kQueueStride;
  v.items = n_items > v.q ? (n_items - v.q + v.nq - 1) / v.nq : 0;
  v.waves = ((grid - v.q + v.nq - 1) / v.nq) * WPB;
  v.wave = ((int)blockIdx.x / v.nq) * WPB + w;
  const int c = v.items / (2 * v.waves);
  v.chunk = c < 1 ? 1 : (c > max_chunk ? max_chunk : c);
  if (blockIdx.x == 0 && w == 0 && lane < kQueues) {
    const int nxt = (int)((seq + 1) % kQueueSlots);
    queues[(nxt * kQueues + lane) * kQueueStride] = 0u;       // claims
    queues[(nxt * kQueues + lane) * kQueueStride + 1] = 0u;   // exits
  }
  return v;
}

// Calls f(position) for every item position this wave owns or claims.  Every
// wave leaves once its claim passes the end of its queue.
template <typename F>
__device__ __forceinline__ void queue_drain(const QueueView& v, int lane, F&& f) {
  const int dyn0 = v.waves * v.chunk;  // first position handed out by the counter
  int first = v.wave * v.chunk;        // static first chunk
  while (first < v.items) {
    const int end = min(first + v.chunk, v.items);
    for (int j = first; j < end; ++j) f(v.q + j * v.nq);
    if (dyn0 >= v.items) break;        // the static chunks cover the queue
    // a plain read first: a drained queue costs no atomic
    uint32_t cur = 0;
    if (lane == 0) cur = __hip_atomic_load(v.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (dyn0 + __builtin_amdgcn_readfirstlane((int)cur) >= v.items) break;
    uint32_t got = 0;
    if (lane == 0) got = atomicAdd(v.ctr, (uint32_t)v.chunk);
    first = dyn0 + __builtin_amdgcn_readfirstlane((int)got);
  }
  // The last wave to leave the queue returns its claim and exit counters to
  // zero, so every launch leaves its counter set clean and a launch captured
  // once replays correctly.  A wave counts its exit only after its last claim
  // has returned, so no claim can follow the reset.
  if (lane == 0) {
    const uint32_t left = atomicAdd(v.ctr + 1, 1u);
    if (left == (uint32_t)v.waves - 1u) {
      __hip_atomic_store(v.ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(v.ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int WPB, bool ASC>
__global__ __launch_bounds__(64 * WPB) void k_persist(DevState S, DevIo io0, const RolloutDesc* rd,
                                                      int t, uint32_t seq) {
  __shared__ __align__(16) uint8_t smap[WPB][kMaxSide * kMaxSide];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  __shared__ uint32_t sclr[kColorWords];
  stage_colors(sclr);
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const DevIo io = io_of(io0, rd, t);
  const QueueView v = queue_view<WPB>(S.queues, seq, S.n, w, lane);
  queue_drain(v, lane, [&](int pos) {
    const int env = __builtin_amdgcn_readfirstlane(S.order[pos]);
    process_env<kMaxSide, ASC, 0>(S, io, env, lane, smap[w], sclr, nullptr, scol[w]);
  });
}

// Serving form: work items span several clients' batches.
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void k_serve(const DevState* states, const DevIo* ios,
                                                    const ServeItem* items, int n_items,
                                                    uint32_t* queues, uint32_t seq) {
  __shared__ __align__(16) uint8_t smap[WPB][kMaxSide * kMaxSide];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  __shared__ uint32_t sclr[kColorWords];
  stage_colors(sclr);
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const QueueView v = queue_view<WPB>(queues, seq, n_items, w, lane);
  queue_drain(v, lane, [&](int pos) {
    const int d = __builtin_amdgcn_readfirstlane(items[pos].desc);
    const int env = __builtin_amdgcn_readfirstlane(items[pos].env);
    // fields are read from the descriptors where they are used (scalar loads)
    const DevState& S = states[d];
    const DevIo& io = ios[d];
    process_env<kMaxSide, true, 0>(S, io, env, lane, smap[w], sclr, nullptr, scol[w]);
  });
}

// Pipelined form: a workgroup holds P wave pairs.  In each pair a producer
// wave loads, steps and casts envs (prefetching the next env's inputs while it
// computes the current one) and never stores to global memory; a writer wave
// expands the previous env's span records into its frame and stores frame and
// state.  The two alternate LDS buffers, one workgroup barrier per round, so
// producing env k+1 overlaps writing env k, and the writer's outstanding stores
// never stall a load.  Pairs walk the work order (costliest first) with a
// static stride of all pairs in the grid.
template <int MAXN, int P, bool ASC>
__global__ __launch_bounds__(128 * P) void k_pipe(DevState S, DevIo io0, const RolloutDesc* rd,
                                                  int t) {
  __shared__ __align__(16) uint8_t smap[P][MAXN * MAXN];
  __shared__ __align__(16) uint32_t scol[P][2][2 * kMaxW];
  __shared__ EnvOut sout[P][2];
  __shared__ uint32_t sclr[kColorWords];
  stage_colors(sclr);
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int pair = w >> 1;
  const bool writer = (w & 1) != 0;
  const DevIo io = io_of(io0, rd, t);
  const int pairs = (int)gridDim.x * P;
  const int gp = (int)blockIdx.x * P + pair;
  const int lead = (int)blockIdx.x * P;  // the workgroup's pair with the most items
  const int rounds = S.n > lead ? (S.n - lead + pairs - 1) / pairs : 0;
  EnvIn<MAXN> cur, nxt;
  if (!writer && gp < S.n) load_env<MAXN>(S, __builtin_amdgcn_readfirstlane(S.order[gp]), lane, cur);
  for (int k = 0; k <= rounds; ++k) {
    const int b = k & 1;
    if (!writer) {
      const int item = gp + k * pairs;
      if (k < rounds && item < S.n) {
        const int nitem = item + pairs;
        if (nitem < S.n) load_env<MAXN>(S, __builtin_amdgcn_readfirstlane(S.order[nitem]), lane, nxt);
        EnvOut o;
        produce_env<MAXN, true, ASC>(cur, S, io, -1, lane, smap[pair], sclr, scol[pair][b], o);
        o.obs_off = obs_off_of(S, o.env);
        if (lane == 0) sout[pair][b] = o;
        cur = nxt;
      } else if (lane == 0) {
        sout[pair][b].env = -1;
      }
    } else if (k > 0) {
      const EnvOut o = sout[pair][b ^ 1];
      if (o.env >= 0) {
        fill_frame<0>(scol[pair][b ^ 1], nullptr, io.obs + o.obs_off, o.W, o.H, lane, io.store_mode);
        write_back(S, io, o, lane);
      }
    }
    __syncthreads();
  }
}

// One env's fused rollout: the wave carries the env through all T steps with
// the state in registers and its layout staged once in LDS, loading the env's
// actions 128 steps at a time.  Inside the step loop the wave issues no global
// loads, so its frame stores never stall it, and waves drift out of phase: one
// wave's casting overlaps another's stores.  Per step the results are those of
// a single-step launch; the state is written back once, after the last step.
template <int MAXN, bool ASC, int FMT>
__device__ __forceinline__ void roll_env(const DevState& S, int env, int lane, uint8_t* lmap, const uint32_t* lclr,
                                         const uint32_t* lcvt, uint32_t* lcol, const uint8_t* act, uint8_t* obs,
                                         int64_t obs_stride, float* rew, uint8_t* dn, uint8_t* prv, int T,
                                         int store_mode, const DevIo& io, int part = 0, int parts = 1) {
  const int64_t n = S.n;
  EnvIn<MAXN> in;
  load_env<MAXN>(S, env, lane, in);
  stage_map<MAXN>(in, lane, lmap);
  const int64_t obs_off = obs_off_of(S, env);
  uint32_t n_invalid = 0, last_ev = 0;
  for (int t0 = 0; t0 < T; t0 += 128) {
    // lane l holds the actions of steps t0 + l and t0 + 64 + l
    const int s0 = t0 + lane, s1 = t0 + 64 + lane;
    const uint32_t a0 = s0 < T ? act[(int64_t)s0 * n + env] : 0u;
    const uint32_t a1 = s1 < T ? act[(int64_t)s1 * n + env] : 0u;
    const int tend = T - t0 < 128 ? T - t0 : 128;
    for (int k = 0; k < tend; ++k) {
      // (& 0xFF: the action is a byte, so produce_env's load path for a
      // negative action folds away and the step loop issues no load)
      // Wait for this wave's previous frame stores before the next step: a
      // wave then has at most one frame's stores in flight.  Measured on the
      // 4096-env workload this bound keeps the HBM write stream more
      // efficient than letting stores of many steps pile up (and the casting
      // of the other waves still overlaps them).  vmcnt 0, other counters
      // untouched.
      __builtin_amdgcn_s_waitcnt(0x0F70);
      const int a = __shfl((int)(k < 64 ? a0 : a1), k & 63, 64) & 0xFF;
      // an opaque copy of the lane id keeps the per-column set-up inside the
      // loop instead of hoisted out of it and held live across all steps
      int ln = lane;
      asm volatile("" : "+v"(ln));
      EnvOut o;
      produce_env<MAXN, false, ASC>(in, S, io, a, ln, lmap, lclr, lcol, o);
      const int t = t0 + k;
      fill_frame<FMT>(lcol, lcvt, obs + (int64_t)t * obs_stride + obs_off, o.W, o.H, ln, store_mode, part, parts);
      if (lane == 0 && part == 0) {
        rew[(int64_t)t * n + env] = o.reward;
        dn[(int64_t)t * n + env] = (uint8_t)o.done;
        if (prv) prv[(int64_t)t * n + env] = (uint8_t)o.prev;
      }
      // the carried state is uniform across the wave: keep it in scalar registers
      const uint32_t ev = uniform_u(o.ev);
      n_invalid += (ev & EV_INVALID) ? 1u : 0u;
      last_ev = ev;
      in.x = uniform_f(o.x);
      in.y = uniform_f(o.y);
      in.th = uniform_f(o.th);
      in.t = uniform_u(o.t);
      in.ep = uniform_u(o.ep);
      in.fl = uniform_u(o.fl);
      in.nd = (int)uniform_u(o.nd);
      in.goal = (int)uniform_u((uint32_t)o.goal);
      in.door = (int)uniform_u((uint32_t)o.door);
      in.key = (int)uniform_u((uint32_t)o.key);
      in.dec0 = (int)uniform_u((uint32_t)o.dec0);
      in.dec1 = (int)uniform_u((uint32_t)o.dec1);
      in.doors = uniform_u(o.doors);
      in.sn = uniform_d(o.sn);
      in.cs = uniform_d(o.cs);
    }
  }
  if (lane == 0 && part == 0 && T > 0) {
    S.x[env] = in.x;
    S.y[env] = in.y;
    S.th[env] = in.th;
    S.t[env] = in.t;
    S.ep[env] = in.ep;
    S.goal[env] = in.goal;
    S.door[env] = in.door;
    S.key[env] = in.key;
    S.decor[2 * env] = in.dec0;
    S.decor[2 * env + 1] = in.dec1;
    S.flags[env] = (uint8_t)in.fl;
    S.ndecor[env] = (uint8_t)in.nd;
    S.events[env] = (uint8_t)last_ev;
    S.doors[env] = in.doors;
    if (n_invalid) S.invalid[env] += n_invalid;
  }
}

// Fused rollout: one launch for T steps of every env.  Waves take envs by a
// static stride over the work order (costliest first); wpe consecutive waves
// share an env (each fills its share of the row pairs).
template <int MAXN, int WPB, bool ASC, int FMT>
__global__ __launch_bounds__(64 * WPB) void k_roll(DevState S, const uint8_t* act, uint8_t* obs,
                                                   int64_t obs_stride, float* rew, uint8_t* dn,
                                                   uint8_t* prv, int T, int store_mode, int wpe) {
  __shared__ __align__(16) uint8_t smap[WPB][MAXN * MAXN];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  __shared__ uint32_t sclr[kColorWords];
  __shared__ uint32_t scvt[FMT % 3 ? 256 : 1];
  stage_tables<FMT>(sclr, scvt);
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int gw = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WPB + w);
  const int first = gw / wpe, part = gw - first * wpe;
  const int stride = (int)gridDim.x * WPB / wpe;
  DevIo io{};
  io.obs = obs;
  io.mode = MODE_STEP;
  io.store_mode = store_mode;
  for (int item = first; item < S.n; item += stride) {
    const int env = __builtin_amdgcn_readfirstlane(S.order[item]);
    roll_env<MAXN, ASC, FMT>(S, env, lane, smap[w], sclr, scvt, scol[w], act, obs, obs_stride, rew, dn, prv, T,
                             store_mode, io, part, wpe);
  }
}

// Persistent fused rollout: a grid sized to the chip's resident waves drains
// the work order (costliest first) one env per claim, each env carried
// through all T steps as in k_roll.  An env of a 128 x 128 frame costs 16
// times one of 32 x 32, so with uneven shapes dynamic claims keep every wave
// busy until the queue is empty (longest-first list scheduling) where a
// static stride leaves workgroups waiting on their slowest wave.  The queues
// and counter sets are those of k_persist (one claim per env: chunk 1).
template <int MAXN, int WPB, bool ASC>
__global__ __launch_bounds__(64 * WPB) void k_proll(DevState S, const uint8_t* act, uint8_t* obs,
                                                    int64_t obs_stride, float* rew, uint8_t* dn,
                                                    uint8_t* prv, int T, int store_mode, uint32_t seq) {
  __shared__ __align__(16) uint8_t smap[WPB][MAXN * MAXN];
  __shared__ __align__(16) uint32_t scol[WPB][2 * kMaxW];
  __shared__ uint32_t sclr[kColorWords];
  stage_colors(sclr);
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  DevIo io{};
  io.obs = obs;
  io.mode = MODE_STEP;
  io.store_mode = store_mode;
  const QueueView v = queue_view<WPB>(S.queues, seq, S.n, w, lane, 1);
  queue_drain(v, lane, [&](int pos) {
    const int env = __builtin_amdgcn_readfirstlane(S.order[pos]);
    roll_env<MAXN, ASC, 0>(S, env, lane, smap[w], sclr, nullptr, scol[w], act, obs, obs_stride, rew, dn, prv, T,
                           store_mode, io);
  });
}

__global__ void k_clear_queues(uint32_t* q) {
  for (int i = (int)threadIdx.x; i < kQueueWords; i += (int)blockDim.x) q[i] = 0u;
}

__global__ void k_set_desc(RolloutDesc* rd, RolloutDesc v) {
  if (threadIdx.x == 0) *rd = v;
}

// The training-buffer formats (FMT != 0) are built for 4 waves per workgroup
// only: the host maps every launch of such a batch to that shape.
constexpr int kFmtWaves = 4;

template <int MAXN, bool ASC, int FMT>
int launch_plain_n(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t, int wpb, int wpe,
                   hipStream_t st) {
  if constexpr (FMT != 0) {
    const int grid = (int)(((int64_t)s.n * wpe + kFmtWaves - 1) / kFmtWaves);
    hipLaunchKernelGGL((k_plain<MAXN, kFmtWaves, ASC, FMT>), dim3(grid), dim3(64 * kFmtWaves), 0, st, s, io,
                       rd, t, wpe);
    return (int)hipGetLastError();
  } else {
    const int grid = (int)(((int64_t)s.n * wpe + wpb - 1) / wpb);
    switch (wpb) {
      case 1: hipLaunchKernelGGL((k_plain<MAXN, 1, ASC, 0>), dim3(grid), dim3(64), 0, st, s, io, rd, t, wpe); break;
      case 2: hipLaunchKernelGGL((k_plain<MAXN, 2, ASC, 0>), dim3(grid), dim3(128), 0, st, s, io, rd, t, wpe); break;
      case 4: hipLaunchKernelGGL((k_plain<MAXN, 4, ASC, 0>), dim3(grid), dim3(256), 0, st, s, io, rd, t, wpe); break;
      case 8: hipLaunchKernelGGL((k_plain<MAXN, 8, ASC, 0>), dim3(grid), dim3(512), 0, st, s, io, rd, t, wpe); break;
      default: return -1;
    }
    return (int)hipGetLastError();
  }
}

}  // namespace

// Reset, render-only and debug launches always take the plain kernel.
inline bool mode_needs_plain(const DevIo& io, const RolloutDesc* rd) {
  return !rd && (io.mode != MODE_STEP || io.dbg != nullptr || io.obs == nullptr);
}

template <int MAXN, bool ASC, int FMT>
int launch_pipe_n(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t, int p, int groups,
                  hipStream_t st) {
  switch (p) {
    case 1: hipLaunchKernelGGL((k_pipe<MAXN, 1, ASC>), dim3(groups), dim3(128), 0, st, s, io, rd, t); break;
    case 2: hipLaunchKernelGGL((k_pipe<MAXN, 2, ASC>), dim3(groups), dim3(256), 0, st, s, io, rd, t); break;
    case 4: hipLaunchKernelGGL((k_pipe<MAXN, 4, ASC>), dim3(groups), dim3(512), 0, st, s, io, rd, t); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

template <int MAXN, bool ASC, int FMT>
int launch_roll_n(const DevState& s, const uint8_t* act, uint8_t* obs, int64_t obs_stride, float* rew,
                  uint8_t* dn, uint8_t* pv, int T, int wpb, int groups, int nt, int wpe, hipStream_t st) {
  if constexpr (FMT != 0) {
    hipLaunchKernelGGL((k_roll<MAXN, kFmtWaves, ASC, FMT>), dim3(groups), dim3(64 * kFmtWaves), 0, st, s, act,
                       obs, obs_stride, rew, dn, pv, T, nt, wpe);
    return (int)hipGetLastError();
  } else {
    switch (wpb) {
      case 1: hipLaunchKernelGGL((k_roll<MAXN, 1, ASC, 0>), dim3(groups), dim3(64), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, wpe); break;
      case 2: hipLaunchKernelGGL((k_roll<MAXN, 2, ASC, 0>), dim3(groups), dim3(128), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, wpe); break;
      case 4: hipLaunchKernelGGL((k_roll<MAXN, 4, ASC, 0>), dim3(groups), dim3(256), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, wpe); break;
      case 8: hipLaunchKernelGGL((k_roll<MAXN, 8, ASC, 0>), dim3(groups), dim3(512), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, wpe); break;
      default: return -1;
    }
    return (int)hipGetLastError();
  }
}

template <int MAXN, bool ASC, int FMT>
int launch_proll_n(const DevState& s, const uint8_t* act, uint8_t* obs, int64_t obs_stride, float* rew,
                   uint8_t* dn, uint8_t* pv, int T, int wpb, int groups, int nt, uint32_t seq, hipStream_t st) {
  switch (wpb) {
    case 1: hipLaunchKernelGGL((k_proll<MAXN, 1, ASC>), dim3(groups), dim3(64), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, seq); break;
    case 2: hipLaunchKernelGGL((k_proll<MAXN, 2, ASC>), dim3(groups), dim3(128), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, seq); break;
    case 4: hipLaunchKernelGGL((k_proll<MAXN, 4, ASC>), dim3(groups), dim3(256), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, seq); break;
    case 8: hipLaunchKernelGGL((k_proll<MAXN, 8, ASC>), dim3(groups), dim3(512), 0, st, s, act, obs, obs_stride, rew, dn, pv, T, nt, seq); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

template <bool ASC>
int launch_persist_n(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t, int wpb,
                     int groups, uint32_t seq, hipStream_t st) {
  switch (wpb) {
    case 1: hipLaunchKernelGGL((k_persist<1, ASC>), dim3(groups), dim3(64), 0, st, s, io, rd, t, seq); break;
    case 2: hipLaunchKernelGGL((k_persist<2, ASC>), dim3(groups), dim3(128), 0, st, s, io, rd, t, seq); break;
    case 4: hipLaunchKernelGGL((k_persist<4, ASC>), dim3(groups), dim3(256), 0, st, s, io, rd, t, seq); break;
    case 8: hipLaunchKernelGGL((k_persist<8, ASC>), dim3(groups), dim3(512), 0, st, s, io, rd, t, seq); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

// Picks the kernel variant by the largest map side and by whether the batch
// holds ASCII maps (frame format FMT fixed).
template <template <int, bool, int> class L, int FMT, typename... A>
int by_shape_f(const DevState& s, int max_side, A&&... a) {
  if (s.any_ascii) {
    if (max_side <= 16) return L<16, true, FMT>::run(s, a...);
    if (max_side <= 32) return L<32, true, FMT>::run(s, a...);
    return L<64, true, FMT>::run(s, a...);
  }
  if (max_side <= 16) return L<16, false, FMT>::run(s, a...);
  if (max_side <= 32) return L<32, false, FMT>::run(s, a...);
  return L<64, false, FMT>::run(s, a...);
}
// ... and by the batch's frame format
template <template <int, bool, int> class L, typename... A>
int by_shape(const DevState& s, int max_side, A&&... a) {
  switch (s.obs_fmt) {
    case 0: return by_shape_f<L, 0>(s, max_side, a...);
    case 1: return by_shape_f<L, 1>(s, max_side, a...);
    case 2: return by_shape_f<L, 2>(s, max_side, a...);
    case 3: return by_shape_f<L, 3>(s, max_side, a...);
    case 4: return by_shape_f<L, 4>(s, max_side, a...);
    case 5: return by_shape_f<L, 5>(s, max_side, a...);
    default: return -1;
  }
}
template <int MAXN, bool ASC, int FMT>
struct PlainL {
  static int run(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t, int wpb, int wpe,
                 hipStream_t st) {
    return launch_plain_n<MAXN, ASC, FMT>(s, io, rd, t, wpb, wpe, st);
  }
};
template <int MAXN, bool ASC, int FMT>
struct PipeL {
  static int run(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t, int p, int groups,
                 hipStream_t st) {
    return launch_pipe_n<MAXN, ASC, FMT>(s, io, rd, t, p, groups, st);
  }
};
template <int MAXN, bool ASC, int FMT>
struct RollL {
  static int run(const DevState& s, const uint8_t* act, uint8_t* obs, int64_t obs_stride, float* rew,
                 uint8_t* dn, uint8_t* pv, int T, int wpb, int groups, int nt, int wpe, hipStream_t st) {
    return launch_roll_n<MAXN, ASC, FMT>(s, act, obs, obs_stride, rew, dn, pv, T, wpb, groups, nt, wpe, st);
  }
};

template <int MAXN, bool ASC, int FMT>
struct PRollL {
  static int run(const DevState& s, const uint8_t* act, uint8_t* obs, int64_t obs_stride, float* rew,
                 uint8_t* dn, uint8_t* pv, int T, int wpb, int groups, int nt, uint32_t seq, hipStream_t st) {
    return launch_proll_n<MAXN, ASC, FMT>(s, act, obs, obs_stride, rew, dn, pv, T, wpb, groups, nt, seq, st);
  }
};

int launch_set_desc(RolloutDesc* rd_dev, const RolloutDesc& value, void* stream) {
  hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), rd_dev,
                     value);
  return (int)hipGetLastError();
}

int launch_clear_queues(uint32_t* queues, void* stream) {
  hipLaunchKernelGGL(k_clear_queues, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     queues);
  return (int)hipGetLastError();
}

int launch_batch(const DevState& s, const DevIo& io, const RolloutDesc* rd, int t,
                 const LaunchCfg& lc, int max_side, int n_cu, uint32_t seq, void* stream) {
  if (s.n <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int wpb = lc.waves_per_group;
  // training-buffer formats: plain form only.  Several waves per env only for
  // steps that write frames (resets, renders and debug records take one).
  if (lc.form == 0 || s.obs_fmt != 0) {
    const bool frames = io.mode == MODE_STEP && (rd != nullptr || (io.obs != nullptr && io.dbg == nullptr));
    const int wpe = frames ? lc.waves_per_env : 1;
    return by_shape<PlainL>(s, max_side, io, rd, t, wpb, wpe, st);
  }
  if (lc.form == 2) {
    // waves_per_group counts wave pairs (1, 2 or 4) in the pipelined form
    const int p = wpb > 4 ? 4 : wpb;
    int groups = n_cu * lc.groups_per_cu;
    const int need = (s.n + p - 1) / p;
    if (groups > need) groups = need;
    if (groups < 1) groups = 1;
    if (mode_needs_plain(io, rd)) return by_shape<PlainL>(s, 64, io, rd, t, 1, 1, st);
    return by_shape_f<PipeL, 0>(s, max_side, io, rd, t, p, groups, st);
  }
  int groups = n_cu * lc.groups_per_cu;
  const int need = (s.n + wpb - 1) / wpb;
  if (groups > need) groups = need;
  if (groups < 1) groups = 1;
  return s.any_ascii ? launch_persist_n<true>(s, io, rd, t, wpb, groups, seq, st)
                     : launch_persist_n<false>(s, io, rd, t, wpb, groups, seq, st);
}

int launch_serve(const DevState* states_dev, const DevIo* ios_dev, const ServeItem* items_dev,
                 int n_items, uint32_t* queues_dev, uint32_t seq, int waves_per_group,
                 int n_groups, void* stream) {
  if (n_items <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  switch (waves_per_group) {
    case 1: hipLaunchKernelGGL((k_serve<1>), dim3(n_groups), dim3(64), 0, st, states_dev, ios_dev, items_dev, n_items, queues_dev, seq); break;
    case 2: hipLaunchKernelGGL((k_serve<2>), dim3(n_groups), dim3(128), 0, st, states_dev, ios_dev, items_dev, n_items, queues_dev, seq); break;
    case 4: hipLaunchKernelGGL((k_serve<4>), dim3(n_groups), dim3(256), 0, st, states_dev, ios_dev, items_dev, n_items, queues_dev, seq); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

int launch_rollout_fused(const DevState& s, const uint8_t* act, uint8_t* obs, int64_t obs_stride,
                         float* rew, uint8_t* dn, uint8_t* prev, int T, const LaunchCfg& lc, int max_side,
                         int n_cu, uint32_t seq, void* stream) {
  if (s.n <= 0 || T <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (lc.form == 1 && s.obs_fmt == 0) {
    // persistent: the chip's share of resident workgroups, never more than needed
    const int wpb = lc.waves_per_group;
    int groups = n_cu * lc.groups_per_cu;
    const int need = (s.n + wpb - 1) / wpb;
    if (groups > need) groups = need;
    if (groups < 1) groups = 1;
    return by_shape_f<PRollL, 0>(s, max_side, act, obs, obs_stride, rew, dn, prev, T, wpb, groups, lc.store_mode,
                                 seq, st);
  }
  const int wpb = s.obs_fmt != 0 ? kFmtWaves : lc.waves_per_group;
  const int wpe = lc.waves_per_env;
  // wpe waves per env while they fit on the chip (16 waves per CU), else a stride
  int groups = (int)(((int64_t)s.n * wpe + wpb - 1) / wpb);
  const int cap = n_cu * (16 / wpb > 0 ? 16 / wpb : 1);
  if (groups > cap) groups = cap;
  return by_shape<RollL>(s, max_side, act, obs, obs_stride, rew, dn, prev, T, wpb, groups, lc.store_mode, wpe, st);
}

const char* kernel_error_string(int code) { return hipGetErrorString((hipError_t)code); }

// Work-queue counters of the rollout entry point that allocates nothing: a
// file-scope device array, one copy per device, alive until the process ends.
// In host code `scratch` names a host-side stand-in, not a device address: the
// kernels receive the address looked up below, once per device.
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int scratch_device_address(int device, uint32_t** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[device] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[device];
  return 0;
}

}  // namespace jx
