/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built with
 * gcc by tests/test_host_sanitize.py): mazes of every side, ASCII maps with
 * mangled text, resets, steps with every action and out-of-range actions, and
 * renders (both tie branches, tie masks) at frame sizes from 2x4 to 128x128,
 * plus a short rollout.  Exits 0 when every call returned normally. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "jx_oracle.h"

static uint64_t g_rng = 0x2545F4914F6CDD1Dull;
static uint64_t rnd(void) { /* xorshift64*: test inputs only */
  g_rng ^= g_rng >> 12;
  g_rng ^= g_rng << 25;
  g_rng ^= g_rng >> 27;
  return g_rng * 2685821657736338717ull;
}
static double unif(void) { return (double)(rnd() >> 11) * (1.0 / 9007199254740992.0); }

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

static orc_cfg cfg_of(int N, int H, int W, int kd, const char* map) {
  orc_cfg c;
  memset(&c, 0, sizeof(c));
  c.side = N;
  c.n_colors = 8;
  c.loop_frac = (double)0.1f;
  c.key_door = kd;
  c.goal_sprite = 1;
  c.max_decor = kd ? 2 : 0;
  c.obs_h = H;
  c.obs_w = W;
  c.fov_deg = 60.0;
  c.n_actions = 6;
  c.episode_cap = 40;
  c.move = (double)0.1f;
  c.turn = (double)0.19634954f;
  c.pickup_radius = (double)0.3f;
  c.r_goal = 1.0;
  c.r_key = 0.5;
  c.shade_levels = (int)(rnd() % 3) * 4;
  c.shade_dist = 10.0;
  c.ascii_map = map;
  return c;
}

int main(void) {
  static uint8_t grid[64 * 64];
  static uint8_t obs[128 * 128 * 3], tie[128 * 128];
  static int32_t hit[128], side[128], cf[128], ah[128], as[128];
  static double ts[128], at[128];
  int32_t keys[3];
  int bad = 0;
  for (int N = 5; N <= 64; ++N)
    for (int k = 0; k < 3; ++k)
      if (orc_maze(rnd(), N, unif(), grid) < 0) ++bad;
  if (orc_maze(1, 4, 0.0, grid) >= 0 || orc_maze(1, 65, 0.0, grid) >= 0) ++bad;
  /* mangled ASCII maps */
  const char alphabet[] = "#.S G rby RBY\"\\123456789\n\nxz~";
  char buf[512];
  for (int it = 0; it < 20000; ++it) {
    size_t len = strlen(kMap);
    memcpy(buf, kMap, len + 1);
    const int edits = 1 + (int)(rnd() % 6);
    for (int e = 0; e < edits; ++e) {
      const uint64_t r = rnd();
      const size_t pos = (size_t)(r % (len + 1));
      const char ch = alphabet[(r >> 20) % (sizeof(alphabet) - 1)];
      if ((r >> 40) % 3 == 0 && pos < len) {
        buf[pos] = ch;
      } else if ((r >> 40) % 3 == 1 && len + 2 < sizeof(buf)) {
        memmove(buf + pos + 1, buf + pos, len - pos + 1);
        buf[pos] = ch;
        ++len;
      } else if (pos < len) {
        memmove(buf + pos, buf + pos + 1, len - pos);
        --len;
      }
    }
    (void)orc_ascii(buf, 5 + (int)(rnd() % 60), grid, keys);
  }
  /* episodes: reset, steps with every action (and invalid ones), renders */
  for (int it = 0; it < 400; ++it) {
    const int ascii = (it % 5) == 0;
    const int N = ascii ? 10 + (int)(rnd() % 55) : 5 + (int)(rnd() % 60);
    const int H = 2 * (1 + (int)(rnd() % 64)), W = 4 * (1 + (int)(rnd() % 32));
    orc_cfg c = cfg_of(N, H, W, ascii ? 0 : (int)(rnd() & 1), ascii ? kMap : NULL);
    const uint64_t seed = rnd();
    if (ascii) {
      if (orc_ascii(kMap, N, grid, keys) < 0) { ++bad; continue; }
    } else if (orc_maze(seed, N, c.loop_frac, grid) < 0) {
      ++bad;
      continue;
    }
    orc_state s, s2;
    if (orc_reset(grid, &c, seed, (int)(rnd() % 5), &s) != 0) { ++bad; continue; }
    for (int t = 0; t < 30; ++t) {
      double r;
      int32_t d, ev, sf;
      const int a = (int)(rnd() % 8); /* 6 and 7 are out of range */
      if (orc_step(grid, &c, seed, &s, a, &s2, &r, &d, &ev, &sf) != 0) ++bad;
      s = s2;
      const int br = (int)(rnd() & 1);
      if (orc_render_ex(grid, &c, &s, br, obs, hit, side, ts, cf, ah, as, at, tie) != 0) ++bad;
    }
    /* a pose on the exact tile corner and one at the map's edge */
    s.x = floor(s.x);
    s.y = floor(s.y);
    (void)orc_render(grid, &c, &s, obs, hit, side, ts, cf, ah, as, at);
  }
  /* a short rollout */
  {
    orc_cfg c = cfg_of(16, 64, 64, 1, NULL);
    uint64_t seeds[8];
    static uint8_t acts[8 * 50];
    static uint8_t last[8 * 64 * 64 * 3]; /* last frame of every env */
    int64_t counts[4];
    for (int i = 0; i < 8; ++i) seeds[i] = rnd();
    for (int i = 0; i < 8 * 50; ++i) acts[i] = (uint8_t)(rnd() % 6);
    if (orc_rollout(&c, 8, seeds, 50, acts, last, counts) != 8 * 50) ++bad;
  }
  printf("oracle checks: %d failures\n", bad);
  return bad ? 1 : 0;
}
