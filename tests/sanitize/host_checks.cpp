// Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer
// (built with g++ by tests/test_host_sanitize.py; no GPU): the maze generator,
// the ASCII map parser on valid and mangled maps, configuration validation on
// hostile values, the reset image of mixed batches, and the state-image checks
// on images with corrupted fields.  Exits 0 when every check held; any memory
// or undefined-behaviour error aborts the run.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "jx.h"
#include "jx_common.h"
#include "jx_internal.h"
#include "jx_layout.h"

using namespace jx;

static uint64_t g_rng = 0x9E3779B97F4A7C15ull;
static uint64_t rnd() {  // xorshift64*: test inputs only
  g_rng ^= g_rng >> 12;
  g_rng ^= g_rng << 25;
  g_rng ^= g_rng >> 27;
  return g_rng * 2685821657736338717ull;
}
static int fails = 0;
#define CHECK(c, ...)                         \
  do {                                        \
    if (!(c)) {                               \
      std::fprintf(stderr, "FAIL: " __VA_ARGS__); \
      std::fprintf(stderr, "\n");             \
      ++fails;                                \
    }                                         \
  } while (0)

static jx_env_cfg base_cfg(int side, int obs) {
  jx_env_cfg c{};
  c.side = side;
  c.n_colors = 8;
  c.loop_frac = 0.1f;
  c.goal_sprite = 1;
  c.obs_h = obs;
  c.obs_w = obs;
  c.fov_deg = 60.f;
  c.n_actions = 6;
  c.episode_cap = 64;
  c.move = 0.1f;
  c.turn = 0.19634954f;
  c.pickup_radius = 0.3f;
  c.r_goal = 1.f;
  c.r_key = 0.5f;
  return c;
}

static const char* kMap =
    "##########\n"
    "#S..r#..G#\n"
    "#....R...#\n"
    "#..1.#.b.#\n"
    "###B##\"###\n"
    "#..y.#...#\n"
    "#.2..Y..G#\n"
    "#....\\...#\n"
    "#S...#.3.#\n"
    "##########";

int main() {
  // mazes: every side, several loop fractions; borders block
  std::vector<uint8_t> g(64 * 64);
  for (int N = 5; N <= 64; ++N)
    for (float f : {0.f, 0.1f, 0.5f, 1.f})
      for (int k = 0; k < 3; ++k) {
        CHECK(make_maze(rnd(), N, f, g.data()), "maze N=%d", N);
        for (int i = 0; i < N; ++i)
          CHECK(g[i] && g[(N - 1) * N + i] && g[i * N] && g[i * N + N - 1], "maze border N=%d", N);
      }
  CHECK(!make_maze(1, 4, 0.f, g.data()), "side 4 accepted");
  CHECK(!make_maze(1, 65, 0.f, g.data()), "side 65 accepted");

  // ASCII maps: the valid map at several sides, then mangled copies
  int32_t keys[3];
  std::string why;
  for (int N = 10; N <= 64; N += 9) CHECK(parse_ascii_map(kMap, N, g.data(), keys, &why) >= 0, "map N=%d", N);
  const char alphabet[] = "#.S G rby RBY\"\\123456789\n\nxz~\t";
  for (int it = 0; it < 20000; ++it) {
    std::string m(kMap);
    const int edits = 1 + (int)(rnd() % 6);
    for (int e = 0; e < edits; ++e) {
      const uint64_t r = rnd();
      const size_t pos = m.empty() ? 0 : (size_t)(r % (m.size() + 1));
      const char ch = alphabet[(r >> 20) % (sizeof(alphabet) - 1)];
      switch ((r >> 40) % 3) {
        case 0: if (pos < m.size()) m[pos] = ch; break;
        case 1: m.insert(m.begin() + (long)pos, ch); break;
        default: if (pos < m.size()) m.erase(pos, 1 + (size_t)((r >> 50) % 12)); break;
      }
    }
    const int N = 5 + (int)(rnd() % 60);
    const int rc = parse_ascii_map(m.c_str(), N, g.data(), keys, &why);
    if (rc >= 0) {
      for (int i = 0; i < N; ++i)
        CHECK(g[i] && g[(N - 1) * N + i] && g[i * N] && g[i * N + N - 1], "accepted map without border");
      for (int c = 0; c < 3; ++c) CHECK(keys[c] >= -1 && keys[c] < N * N, "key out of range");
    }
  }
  CHECK(parse_ascii_map("", 10, g.data(), keys, &why) < 0, "empty map accepted");

  // configuration validation: hostile field values never crash it
  const float fv[] = {0.f, -1.f, 1e30f, std::numeric_limits<float>::quiet_NaN(),
                      std::numeric_limits<float>::infinity(), 0.5f, 60.f, 179.99f};
  const int iv[] = {0, -1, 1, 2, 4, 6, 8, 64, 65, 128, 129, 1 << 30};
  for (int it = 0; it < 200000; ++it) {
    jx_env_cfg c = base_cfg(16, 64);
    const int f = (int)(rnd() % 14);
    const int32_t i = iv[rnd() % (sizeof(iv) / sizeof(iv[0]))];
    const float x = fv[rnd() % (sizeof(fv) / sizeof(fv[0]))];
    switch (f) {
      case 0: c.side = i; break;
      case 1: c.n_colors = i; break;
      case 2: c.loop_frac = x; break;
      case 3: c.obs_h = i; break;
      case 4: c.obs_w = i; break;
      case 5: c.fov_deg = x; break;
      case 6: c.n_actions = i; break;
      case 7: c.episode_cap = i; break;
      case 8: c.move = x; break;
      case 9: c.pickup_radius = x; break;
      case 10: c.shade_levels = i; c.shade_dist = x; break;
      case 11: c.max_decor = i; break;
      case 12: c.obs_layout = i; c.obs_dtype = i; break;
      default: c.ascii_map = kMap; c.side = i; break;
    }
    std::string w;
    if (validate_cfg(c, &w)) {
      CHECK(c.side >= 5 && c.side <= 64 && c.obs_h >= 2 && c.obs_h <= 128 && c.obs_w >= 4 && c.obs_w <= 128,
            "validated an out-of-range configuration");
      (void)derive_cfg(c);
    }
  }

  // reset images of mixed batches; the state checks accept them and refuse
  // corrupted copies without reading out of bounds
  for (int it = 0; it < 60; ++it) {
    const int n_cfgs = 1 + (int)(rnd() % 4);
    std::vector<jx_env_cfg> cfgs;
    for (int k = 0; k < n_cfgs; ++k) {
      jx_env_cfg c = base_cfg(5 + (int)(rnd() % 60), 4 * (1 + (int)(rnd() % 32)));
      c.key_door = (int)(rnd() & 1);
      if (k == 3) {
        c = base_cfg(10 + (int)(rnd() % 50), 64);
        c.ascii_map = kMap;
      }
      cfgs.push_back(c);
    }
    const int n = (int)(rnd() % 300);
    std::vector<uint64_t> seeds(n);
    std::vector<int32_t> idx(n);
    for (int i = 0; i < n; ++i) {
      seeds[i] = rnd();
      idx[i] = (int32_t)(rnd() % n_cfgs);
    }
    std::vector<uint8_t> img;
    Layout L;
    std::vector<int64_t> oo;
    std::vector<int32_t> idx_out;
    const jx_status st = build_image(n, seeds.data(), cfgs.data(), n_cfgs, idx.data(), &img, &L, &oo, &idx_out);
    CHECK(st == JX_OK, "build_image: %s", g_last_error.c_str());
    if (st != JX_OK) continue;
    CHECK((int64_t)img.size() == L.total, "image size");
    CHECK(check_state_image(img.data(), L, n, cfgs, idx_out) == JX_OK, "fresh image refused: %s",
          g_last_error.c_str());
    for (int k = 0; k < 200 && n > 0; ++k) {
      std::vector<uint8_t> bad(img);
      const int64_t off = (int64_t)(rnd() % (uint64_t)L.rdesc);
      bad[(size_t)off] = (uint8_t)rnd();
      (void)check_state_image(bad.data(), L, n, cfgs, idx_out);
    }
  }
  // an out-of-range index is refused
  {
    std::vector<jx_env_cfg> cfgs{base_cfg(16, 64)};
    std::vector<uint64_t> seeds{1, 2, 3};
    std::vector<uint8_t> img;
    Layout L;
    std::vector<int64_t> oo;
    std::vector<int32_t> idx;
    build_image(3, seeds.data(), cfgs.data(), 1, nullptr, &img, &L, &oo, &idx);
    int32_t far = 16 * 16;
    std::memcpy(img.data() + L.goal + 4, &far, 4);
    CHECK(check_state_image(img.data(), L, 3, cfgs, idx) == JX_EINVAL, "goal out of range accepted");
    const float nan = std::numeric_limits<float>::quiet_NaN();
    std::memcpy(img.data() + L.goal + 4, &idx[0], 4);
    std::memcpy(img.data() + L.x + 8, &nan, 4);
    CHECK(check_state_image(img.data(), L, 3, cfgs, idx) == JX_EINVAL, "NaN position accepted");
  }
  std::printf("host checks: %d failures\n", fails);
  return fails ? 1 : 0;
}
