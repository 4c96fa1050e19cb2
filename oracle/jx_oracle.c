/*
 * jx_oracle.c -- the FP64 CPU oracle (test infrastructure only; see jx_oracle.h).
 *
 * Plain and slow on purpose: every rule is written out as its definition, with
 * no blocking, fusion or reordering.  Where the paper (JAXenstein) fixes a rule
 * the comment names the section; where it is silent the comment states the
 * reading taken.  Build: gcc -O2 -fPIC -shared (no fast-math).
 */
#include "jx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Random numbers.  SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state  */
/* advances by the golden gamma and each output is the state passed through  */
/* the variant-13 finaliser.  A uniform draw over [0, n) takes the top 32     */
/* output bits h and returns floor(h * n / 2^32) (Lemire's multiply-shift).   */
/* ------------------------------------------------------------------------ */
static const uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

uint64_t orc_rng_next(uint64_t* s) {
  *s += kGamma;
  uint64_t z = *s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t orc_mix64(uint64_t v) {
  uint64_t s = v;
  return orc_rng_next(&s);
}

uint32_t orc_rng_range(uint64_t* s, uint32_t n) {
  uint64_t h = orc_rng_next(s) >> 32;
  return (uint32_t)((h * (uint64_t)n) >> 32);
}

/* Removes and returns element r of list[0..*len). */
static int32_t list_take(int32_t* list, int32_t* len, int32_t r) {
  int32_t v = list[r];
  for (int32_t i = r; i + 1 < *len; ++i) list[i] = list[i + 1];
  *len -= 1;
  return v;
}

/* ------------------------------------------------------------------------ */
/* Layout.  The paper's worlds are tile maps (Sec. 2.2, Sec. 3.2, Table 2).   */
/* Reading for the synthetic mazes: recursive-backtracker depth-first search  */
/* on a lattice of m = (N-1)/2 cells per side, cell (i, j) at tile            */
/* (2i+1, 2j+1); every other tile starts as wall.  Start cell = draw(m*m).    */
/* At each step the unvisited lattice neighbours of the stack top are listed  */
/* in the order north (j-1), east (i+1), south (j+1), west (i-1); none: pop;  */
/* else take neighbour draw(count), open the tile between and the neighbour,  */
/* push it.  Loops: the separator tiles still standing (x, y in [1, 2m-1],    */
/* exactly one of them even), listed row-major, C of them; k = floor(         */
/* loop_frac*C + 0.5) of them are opened, each one the draw(remaining)-th of  */
/* the remaining list in row-major order.                                     */
/* ------------------------------------------------------------------------ */
int32_t orc_maze(uint64_t seed, int32_t N, double loop_frac, uint8_t* grid) {
  if (N < 5 || N > ORC_MAX_SIDE || !grid || loop_frac < 0.0 || loop_frac > 1.0) return -1;
  const int32_t m = (N - 1) / 2;
  memset(grid, 1, (size_t)N * N);
  uint64_t s = seed;

  uint8_t* visited = (uint8_t*)calloc((size_t)m * m, 1);
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * m);
  int32_t sp = 0;
  int32_t start = (int32_t)orc_rng_range(&s, (uint32_t)(m * m));
  int32_t si = start % m, sj = start / m;
  visited[sj * m + si] = 1;
  grid[(2 * sj + 1) * N + (2 * si + 1)] = 0;
  stack[sp++] = start;
  while (sp > 0) {
    int32_t top = stack[sp - 1];
    int32_t i = top % m, j = top / m;
    int32_t ni[4], nj[4], cnt = 0;
    if (j - 1 >= 0 && !visited[(j - 1) * m + i]) { ni[cnt] = i; nj[cnt] = j - 1; ++cnt; }
    if (i + 1 < m && !visited[j * m + i + 1]) { ni[cnt] = i + 1; nj[cnt] = j; ++cnt; }
    if (j + 1 < m && !visited[(j + 1) * m + i]) { ni[cnt] = i; nj[cnt] = j + 1; ++cnt; }
    if (i - 1 >= 0 && !visited[j * m + i - 1]) { ni[cnt] = i - 1; nj[cnt] = j; ++cnt; }
    if (cnt == 0) { --sp; continue; }
    int32_t k = (int32_t)orc_rng_range(&s, (uint32_t)cnt);
    int32_t a = ni[k], b = nj[k];
    /* separator tile between lattice cells (i,j) and (a,b) */
    grid[(j + b + 1) * N + (i + a + 1)] = 0;
    grid[(2 * b + 1) * N + (2 * a + 1)] = 0;
    visited[b * m + a] = 1;
    stack[sp++] = b * m + a;
  }
  free(visited);
  free(stack);

  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
  int32_t C = 0;
  for (int32_t y = 1; y <= 2 * m - 1; ++y)
    for (int32_t x = 1; x <= 2 * m - 1; ++x) {
      int32_t ex = (x % 2 == 0), ey = (y % 2 == 0);
      if (ex != ey && grid[y * N + x] == 1) cand[C++] = y * N + x;
    }
  int32_t k = (int32_t)floor(loop_frac * (double)C + 0.5);
  int32_t len = C;
  for (int32_t t = 0; t < k; ++t) {
    int32_t r = (int32_t)orc_rng_range(&s, (uint32_t)len);
    int32_t id = list_take(cand, &len, r);
    grid[id] = 0;
  }
  free(cand);
  return k;
}

/* Breadth-first distances over 4-connected tiles with pass[id] != 0. */
static void bfs(const uint8_t* pass, int32_t N, int32_t src, int32_t* dist) {
  for (int32_t i = 0; i < N * N; ++i) dist[i] = -1;
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
  int32_t head = 0, tail = 0;
  dist[src] = 0;
  q[tail++] = src;
  while (head < tail) {
    int32_t v = q[head++];
    int32_t x = v % N, y = v / N;
    const int32_t dx[4] = {0, 1, 0, -1}, dy[4] = {-1, 0, 1, 0};
    for (int32_t d = 0; d < 4; ++d) {
      int32_t a = x + dx[d], b = y + dy[d];
      if (a < 0 || b < 0 || a >= N || b >= N) continue;
      int32_t u = b * N + a;
      if (!pass[u] || dist[u] >= 0) continue;
      dist[u] = dist[v] + 1;
      q[tail++] = u;
    }
  }
  free(q);
}

/* ------------------------------------------------------------------------ */
/* ASCII map front-end (Table 2 symbols).  Reading: the text's rows          */
/* (separated by '\n'; a '\r' is ignored) sit at the top-left of the N x N  */
/* grid and every tile the text does not cover is a default wall.  '#'       */
/* default wall; '1'..'9' coloured walls; '.' and ' ' floor; 'S' a spawn     */
/* candidate and 'G' a goal candidate (both floor); 'r', 'b', 'y' a red,     */
/* blue, yellow key lying on a floor tile (at most one per colour); '"' and  */
/* '\' blue and yellow unlocked doors; 'R', 'B', 'Y' red, blue and yellow    */
/* locked doors.  Doors are indexed in row-major order, at most 16.          */
/* Returns the number of doors, or -1 bad arguments, -2 unknown symbol, -3   */
/* text larger than N x N, -4 more than 16 doors, -5 a key colour twice,     */
/* -6 no floor tile.                                                         */
/* ------------------------------------------------------------------------ */
int32_t orc_ascii(const char* text, int32_t N, uint8_t* grid, int32_t* keys3) {
  if (!text || !grid || !keys3 || N < 5 || N > ORC_MAX_SIDE) return -1;
  for (int32_t i = 0; i < N * N; ++i) grid[i] = 1;
  keys3[0] = keys3[1] = keys3[2] = -1;
  int32_t x = 0, y = 0, doors = 0, floors = 0;
  for (const char* p = text; *p; ++p) {
    const char ch = *p;
    if (ch == '\n') {
      ++y;
      x = 0;
      continue;
    }
    if (ch == '\r') continue;
    if (x >= N || y >= N) return -3;
    const int32_t id = y * N + x;
    uint8_t v;
    if (ch == '#') {
      v = 1;
    } else if (ch >= '1' && ch <= '9') {
      v = (uint8_t)(2 + (ch - '1'));
    } else if (ch == '.' || ch == ' ') {
      v = 0;
    } else if (ch == 'S') {
      v = ORC_TILE_SPAWN;
    } else if (ch == 'G') {
      v = ORC_TILE_GOAL;
    } else if (ch == 'r' || ch == 'b' || ch == 'y') {
      const int32_t c = ch == 'r' ? 0 : (ch == 'b' ? 1 : 2);
      if (keys3[c] >= 0) return -5;
      keys3[c] = id;
      v = 0;
    } else if (ch == '"' || ch == '\\' || ch == 'R' || ch == 'B' || ch == 'Y') {
      if (doors >= ORC_MAX_DOORS) return -4;
      int32_t type;
      if (ch == 'R') type = ORC_DOOR_RED_LOCKED;
      else if (ch == 'B') type = ORC_DOOR_BLUE_LOCKED;
      else if (ch == 'Y') type = ORC_DOOR_YELLOW_LOCKED;
      else if (ch == '"') type = ORC_DOOR_BLUE_UNLOCKED;
      else type = ORC_DOOR_YELLOW_UNLOCKED;
      v = (uint8_t)(ORC_TILE_DOOR | (type << 4) | doors);
      ++doors;
    } else {
      return -2;
    }
    if ((v & 0x8F) == 0) ++floors;
    grid[id] = v;
    ++x;
  }
  if (floors == 0) return -6;
  return doors;
}

/* floor tile: neither a wall class nor a door (spawn/goal marks allowed) */
static int is_floor(uint8_t v) { return (v & 0x8F) == 0; }

/* ------------------------------------------------------------------------ */
/* Episode reset.  The paper's tasks (Table 1, Table 2) have spawn and goal  */
/* candidates and keys/locked doors; for the synthetic mazes the readings    */
/* are, with the episode stream s = seed XOR mix64(episode + 1), drawn in    */
/* this order:                                                               */
/*  1. spawn = free[draw(n_free)] (free tiles row-major), agent at its centre */
/*  2. heading: k = next() >> 40, theta = float(k) * float(2pi_f * 2^-24) in  */
/*     float32 (one rounding of exact operands)                               */
/*  3. goal = the free tile farthest from the spawn by BFS, smallest id wins  */
/*  4. key-door (L = goal distance >= 2): door = smallest id v with           */
/*     d(spawn, v) = floor(L/2) and d(v, goal) = L - floor(L/2); start region */
/*     R = tiles reachable from the spawn with the door shut; key = the       */
/*     draw(|R|-1)-th tile of R minus the spawn (row-major), or the spawn     */
/*     itself when R holds nothing else                                       */
/*  5. decor (max_decor > 0): nd = min(draw(max_decor+1), C) tiles, each the  */
/*     draw(remaining)-th of the remaining free tiles other than spawn, goal, */
/*     key and door, in row-major order                                       */
/* ------------------------------------------------------------------------ */
/* Episode reset on an ASCII map.  Reading, with the same episode stream and  */
/* draw order as the generated mazes: 1. spawn = the draw(|S|)-th spawn       */
/* candidate (row-major), or free[draw(n_free)] when the map has none;        */
/* 2. heading as for the mazes; 3. goal = the draw(|G|)-th goal candidate, or */
/* the tile farthest from the spawn by BFS (doors passable, smallest id on    */
/* ties) when the map has none.  Keys lie where the map puts them, all doors  */
/* start shut.                                                                */
static int32_t ascii_reset(const uint8_t* grid, const orc_cfg* cfg, uint64_t* s,
                           const int32_t* freel, int32_t n_free, orc_state* out) {
  const int32_t N = cfg->side;
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
  int32_t nc = 0;
  for (int32_t id = 0; id < N * N; ++id)
    if (is_floor(grid[id]) && (grid[id] & ORC_TILE_SPAWN)) cand[nc++] = id;
  const int32_t spawn = nc > 0 ? cand[orc_rng_range(s, (uint32_t)nc)]
                               : freel[orc_rng_range(s, (uint32_t)n_free)];
  const uint32_t k24 = (uint32_t)(orc_rng_next(s) >> 40);
  const float two_pi_f = (float)(2.0 * M_PI);
  const float step_f = two_pi_f * 0x1p-24f;
  const float th_f = (float)k24 * step_f;
  nc = 0;
  for (int32_t id = 0; id < N * N; ++id)
    if (is_floor(grid[id]) && (grid[id] & ORC_TILE_GOAL)) cand[nc++] = id;
  int32_t goal;
  if (nc > 0) {
    goal = cand[orc_rng_range(s, (uint32_t)nc)];
  } else {
    uint8_t* pass = (uint8_t*)calloc((size_t)N * N, 1);
    int32_t* ds = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
    for (int32_t id = 0; id < N * N; ++id) pass[id] = is_floor(grid[id]) || (grid[id] & ORC_TILE_DOOR);
    bfs(pass, N, spawn, ds);
    int32_t L = 0;
    goal = spawn;
    for (int32_t id = 0; id < N * N; ++id)
      if (ds[id] > L) { L = ds[id]; goal = id; }
    free(pass);
    free(ds);
  }
  free(cand);
  uint8_t* tmp = (uint8_t*)malloc((size_t)N * N);
  int32_t keys3[3];
  const int32_t nd = orc_ascii(cfg->ascii_map, N, tmp, keys3);
  free(tmp);
  if (nd < 0) return -1;
  out->x = (double)(spawn % N) + 0.5;
  out->y = (double)(spawn / N) + 0.5;
  out->theta = (double)th_f;
  out->t = 0;
  out->goal = goal;
  out->door = -1;
  out->key = -1;
  out->n_decor = 0;
  out->decor[0] = out->decor[1] = -1;
  out->akey[0] = keys3[0];
  out->akey[1] = keys3[1];
  out->akey[2] = keys3[2];
  out->akey_taken = 0;
  out->doors_open = 0;
  return 0;
}

int32_t orc_reset(const uint8_t* grid, const orc_cfg* cfg, uint64_t seed, int32_t episode,
                  orc_state* out) {
  if (!grid || !cfg || !out) return -1;
  const int32_t N = cfg->side;
  if (N < 5 || N > ORC_MAX_SIDE) return -1;
  uint64_t s = seed ^ orc_mix64((uint64_t)(uint32_t)episode + 1ULL);

  int32_t* freel = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
  int32_t n_free = 0;
  for (int32_t id = 0; id < N * N; ++id)
    if (is_floor(grid[id])) freel[n_free++] = id;
  if (n_free == 0) { free(freel); return -1; }

  memset(out, 0, sizeof(*out));
  out->akey[0] = out->akey[1] = out->akey[2] = -1;
  if (cfg->ascii_map) {
    int32_t rc = ascii_reset(grid, cfg, &s, freel, n_free, out);
    free(freel);
    if (rc) return rc;
    out->episode = episode;
    return 0;
  }
  int32_t spawn = freel[orc_rng_range(&s, (uint32_t)n_free)];
  uint32_t k24 = (uint32_t)(orc_rng_next(&s) >> 40);
  const float two_pi_f = (float)(2.0 * M_PI);
  const float step_f = two_pi_f * 0x1p-24f;
  float th_f = (float)k24 * step_f;

  uint8_t* pass = (uint8_t*)malloc((size_t)N * N);
  int32_t* ds = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
  for (int32_t id = 0; id < N * N; ++id) pass[id] = is_floor(grid[id]);
  bfs(pass, N, spawn, ds);
  int32_t L = 0, goal = spawn;
  for (int32_t id = 0; id < N * N; ++id)
    if (ds[id] > L) { L = ds[id]; goal = id; }

  int32_t door = -1, key = -1;
  if (cfg->key_door && L >= 2) {
    int32_t h = L / 2;
    int32_t* dg = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
    bfs(pass, N, goal, dg);
    for (int32_t id = 0; id < N * N; ++id)
      if (ds[id] == h && dg[id] == L - h) { door = id; break; }
    free(dg);
    if (door < 0) { free(pass); free(ds); free(freel); return -1; }
    pass[door] = 0;
    int32_t* dr = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
    bfs(pass, N, spawn, dr);
    pass[door] = 1;
    int32_t c = 0;
    for (int32_t id = 0; id < N * N; ++id)
      if (dr[id] >= 0 && id != spawn) ++c;
    if (c == 0) {
      key = spawn;
    } else {
      int32_t r = (int32_t)orc_rng_range(&s, (uint32_t)c);
      for (int32_t id = 0; id < N * N; ++id)
        if (dr[id] >= 0 && id != spawn) {
          if (r == 0) { key = id; break; }
          --r;
        }
    }
    free(dr);
  }

  int32_t nd = 0;
  if (cfg->max_decor > 0) {
    int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * N);
    int32_t C = 0;
    for (int32_t i = 0; i < n_free; ++i) {
      int32_t id = freel[i];
      if (id == spawn || id == goal || id == key || id == door) continue;
      cand[C++] = id;
    }
    int32_t md = cfg->max_decor > ORC_MAX_DECOR ? ORC_MAX_DECOR : cfg->max_decor;
    nd = (int32_t)orc_rng_range(&s, (uint32_t)(md + 1));
    if (nd > C) nd = C;
    int32_t len = C;
    for (int32_t j = 0; j < nd; ++j) {
      int32_t r = (int32_t)orc_rng_range(&s, (uint32_t)len);
      out->decor[j] = list_take(cand, &len, r);
    }
    free(cand);
  }
  for (int32_t j = nd; j < ORC_MAX_DECOR; ++j) out->decor[j] = -1;

  out->x = (double)(spawn % N) + 0.5;
  out->y = (double)(spawn / N) + 0.5;
  out->theta = (double)th_f;
  out->t = 0;
  out->episode = episode;
  out->goal = goal;
  out->door = door;
  out->key = key;
  out->key_taken = 0;
  out->door_open = 0;
  out->n_decor = nd;
  free(pass);
  free(ds);
  free(freel);
  return 0;
}

/* Tile (tx, ty) blocks movement or rays: outside the grid, a wall, a door of */
/* the map that is not open (`doors`: bit = door index), or the generated    */
/* maze's locked door while it is shut (Table 2: doors; Table 1: key-door).   */
static int blocks(const uint8_t* grid, int32_t N, int32_t door, int32_t door_open, int32_t doors,
                  int32_t tx, int32_t ty) {
  if (tx < 0 || ty < 0 || tx >= N || ty >= N) return 1;
  const int32_t id = ty * N + tx;
  const uint8_t v = grid[id];
  if (v & ORC_TILE_DOOR) return !((doors >> (v & 15)) & 1);
  if (v & 0x0F) return 1;
  if (id == door && !door_open) return 1;
  return 0;
}

/* Bit mask of the map's locked doors of colour c (0 red, 1 blue, 2 yellow). */
static int32_t locked_doors_of(const uint8_t* grid, int32_t N, int32_t c) {
  int32_t m = 0;
  for (int32_t id = 0; id < N * N; ++id) {
    const uint8_t v = grid[id];
    if ((v & ORC_TILE_DOOR) && ((v >> 4) & 7) == c) m |= 1 << (v & 15);
  }
  return m;
}

static int near_int(double v, double w) { return fabs(v - floor(v + 0.5)) <= w; }

/* ------------------------------------------------------------------------ */
/* Transition.  Reading (the paper gives no dynamics): actions with 4:       */
/* forward, back, turn left, turn right; with 6: forward, back, strafe left, */
/* strafe right, turn left, turn right.  Turns add -/+ turn to theta, wrapped */
/* once by 2pi into [0, 2pi).  Moves add +-move*dir or +-move*right, dir =    */
/* (cos th, sin th), right = (-sin th, cos th).  Collision is zero-radius and */
/* axis-separated, x first, then y with the updated x.  Key pickup when the   */
/* squared distance to the key tile's centre is below pickup_radius^2 (opens  */
/* the door, reward r_key); goal when the agent's tile is the goal (reward    */
/* r_goal, terminal); truncation when t+1 reaches the cap; done resets the    */
/* episode in place and the returned state is the next episode's first.       */
/* ------------------------------------------------------------------------ */
int32_t orc_step_w(const uint8_t* grid, const orc_cfg* cfg, uint64_t seed, const orc_state* in,
                   int32_t action, orc_state* out, double* reward, int32_t* done, int32_t* events,
                   int32_t* sflags, double window) {
  if (!grid || !cfg || !in || !out) return -1;
  const int32_t N = cfg->side;
  const double W5 = window;
  int32_t ev = 0, sf = 0;
  double r = 0.0;
  double th = in->theta;
  double c = cos(th), s = sin(th);
  double mvx = 0.0, mvy = 0.0, dth = 0.0;
  int valid = (action >= 0 && action < cfg->n_actions);
  if (!valid) {
    ev |= ORC_EV_INVALID;
  } else if (cfg->n_actions == 4) {
    if (action == 0) { mvx = c; mvy = s; }
    else if (action == 1) { mvx = -c; mvy = -s; }
    else if (action == 2) dth = -cfg->turn;
    else dth = cfg->turn;
  } else {
    if (action == 0) { mvx = c; mvy = s; }
    else if (action == 1) { mvx = -c; mvy = -s; }
    else if (action == 2) { mvx = s; mvy = -c; }      /* -right */
    else if (action == 3) { mvx = -s; mvy = c; }      /* +right */
    else if (action == 4) dth = -cfg->turn;
    else dth = cfg->turn;
  }
  double th2 = th;
  if (dth != 0.0) {
    th2 = th + dth;
    if (th2 < 0.0) th2 += 2.0 * M_PI;
    else if (th2 >= 2.0 * M_PI) th2 -= 2.0 * M_PI;
  }
  double mx = cfg->move * mvx, my = cfg->move * mvy;

  const int32_t door = in->door;
  const int32_t dopen = in->door_open;
  int32_t doors = in->doors_open;
  double x = in->x, y = in->y;
  /* Table 2 unlocked doors open when the agent walks into them; that move is
   * refused (reading) */
#define BUMP(tx_, ty_)                                                             \
  do {                                                                             \
    const int32_t bx = (tx_), by = (ty_);                                          \
    if (bx >= 0 && by >= 0 && bx < N && by < N) {                                  \
      const uint8_t bv = grid[by * N + bx];                                        \
      const int32_t bt = (bv >> 4) & 7;                                            \
      if ((bv & ORC_TILE_DOOR) && (bt == ORC_DOOR_BLUE_UNLOCKED || bt == ORC_DOOR_YELLOW_UNLOCKED) && \
          !((doors >> (bv & 15)) & 1)) {                                           \
        doors |= 1 << (bv & 15);                                                   \
        ev |= ORC_EV_DOOR;                                                         \
      }                                                                            \
    }                                                                              \
  } while (0)
  if (mx != 0.0) {
    double nx = x + mx;
    int32_t fy = (int32_t)floor(y);
    if (near_int(nx, W5)) {
      int32_t k = (int32_t)floor(nx + 0.5);
      if (blocks(grid, N, door, dopen, doors, k - 1, fy) != blocks(grid, N, door, dopen, doors, k, fy)) sf |= ORC_SF_MOVE;
    }
    if (!blocks(grid, N, door, dopen, doors, (int32_t)floor(nx), fy)) {
      x = nx;
    } else {
      ev |= ORC_EV_BLOCKED_X;
      BUMP((int32_t)floor(nx), fy);
    }
  }
  if (my != 0.0) {
    double ny = y + my;
    int32_t fx = (int32_t)floor(x);
    if (near_int(ny, W5)) {
      int32_t k = (int32_t)floor(ny + 0.5);
      if (blocks(grid, N, door, dopen, doors, fx, k - 1) != blocks(grid, N, door, dopen, doors, fx, k)) sf |= ORC_SF_MOVE;
    }
    if (near_int(x, W5)) {
      int32_t k = (int32_t)floor(x + 0.5), fny = (int32_t)floor(ny);
      if (blocks(grid, N, door, dopen, doors, k - 1, fny) != blocks(grid, N, door, dopen, doors, k, fny)) sf |= ORC_SF_MOVE;
    }
    if (!blocks(grid, N, door, dopen, doors, fx, (int32_t)floor(ny))) {
      y = ny;
    } else {
      ev |= ORC_EV_BLOCKED_Y;
      BUMP(fx, (int32_t)floor(ny));
    }
  }
#undef BUMP

  int32_t key_taken = in->key_taken, door_open = in->door_open;
  if (in->key >= 0 && !key_taken) {
    double kx = (double)(in->key % N) + 0.5, ky = (double)(in->key / N) + 0.5;
    double d2 = (x - kx) * (x - kx) + (y - ky) * (y - ky);
    double r2 = cfg->pickup_radius * cfg->pickup_radius;
    if (fabs(d2 - r2) <= W5) sf |= ORC_SF_KEY;
    if (d2 < r2) {
      key_taken = 1;
      door_open = 1;
      r += cfg->r_key;
      ev |= ORC_EV_KEY;
    }
  }
  /* Table 2 keys: picking up the key of colour c opens every locked door of
   * colour c (reward r_key each) */
  int32_t ataken = in->akey_taken;
  for (int32_t c = 0; c < 3; ++c) {
    if (in->akey[c] < 0 || ((ataken >> c) & 1)) continue;
    double kx = (double)(in->akey[c] % N) + 0.5, ky = (double)(in->akey[c] / N) + 0.5;
    double d2 = (x - kx) * (x - kx) + (y - ky) * (y - ky);
    double r2 = cfg->pickup_radius * cfg->pickup_radius;
    if (fabs(d2 - r2) <= W5) sf |= ORC_SF_KEY;
    if (d2 < r2) {
      ataken |= 1 << c;
      r += cfg->r_key;
      ev |= ORC_EV_KEY;
      const int32_t m = locked_doors_of(grid, N, c);
      if (m & ~doors) ev |= ORC_EV_DOOR;
      doors |= m;
    }
  }
  int32_t term = 0;
  if (in->goal >= 0) {
    int32_t gx = in->goal % N, gy = in->goal / N;
    int xin = (x >= gx - W5 && x < gx + 1 + W5), yin = (y >= gy - W5 && y < gy + 1 + W5);
    int xedge = (fabs(x - gx) <= W5 || fabs(x - (gx + 1)) <= W5);
    int yedge = (fabs(y - gy) <= W5 || fabs(y - (gy + 1)) <= W5);
    if ((xedge && yin) || (yedge && xin)) sf |= ORC_SF_GOAL;
    if ((int32_t)floor(x) == gx && (int32_t)floor(y) == gy) {
      r += cfg->r_goal;
      term = 1;
      ev |= ORC_EV_GOAL;
    }
  }
  int32_t t2 = in->t + 1;
  int32_t trunc = (t2 >= cfg->episode_cap);
  if (trunc) ev |= ORC_EV_TRUNC;
  int32_t d = term || trunc;
  if (d) {
    orc_reset(grid, cfg, seed, in->episode + 1, out);
    ev |= ORC_EV_RESET;
  } else {
    *out = *in;
    out->x = x;
    out->y = y;
    out->theta = th2;
    out->t = t2;
    out->key_taken = key_taken;
    out->door_open = door_open;
    out->akey_taken = ataken;
    out->doors_open = doors;
  }
  if (reward) *reward = r;
  if (done) *done = d;
  if (events) *events = ev;
  if (sflags) *sflags = sf;
  return 0;
}

int32_t orc_step(const uint8_t* grid, const orc_cfg* cfg, uint64_t seed, const orc_state* in,
                 int32_t action, orc_state* out, double* reward, int32_t* done, int32_t* events,
                 int32_t* sflags) {
  return orc_step_w(grid, cfg, seed, in, action, out, reward, done, events, sflags, 1e-5);
}

/* ------------------------------------------------------------------------ */
/* One ray (Sec. 2.1: first intersection along the column's ray, found by    */
/* marching tile boundary to tile boundary).  The plain definition: from the */
/* start tile, the ray crosses the k-th vertical grid line at parameter      */
/* t_x(k) = (X0 + k*sx - x)/rx and the k-th horizontal one at t_y(k); each   */
/* crossing enters the next tile; the earlier crossing happens first (ties   */
/* cross y first) and the walk stops at the first blocking tile.  Both       */
/* parameters are recomputed from their crossing counts every time (no       */
/* accumulation).  `flip_at` takes the other branch at that comparison.      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t hit, side;
  double t;
  int32_t n_ties, first_tie;
} cast_out;

static void cast_walk(const uint8_t* grid, int32_t N, int32_t door, int32_t door_open, int32_t doors,
                      double x, double y, double rx, double ry, int32_t flip_at, cast_out* o) {
  int32_t ix = (int32_t)floor(x), iy = (int32_t)floor(y);
  int32_t sx = rx > 0 ? 1 : -1, sy = ry > 0 ? 1 : -1;
  double X0 = rx > 0 ? ix + 1 : ix, Y0 = ry > 0 ? iy + 1 : iy;
  int32_t kx = 0, ky = 0;
  o->n_ties = 0;
  o->first_tie = -1;
  o->hit = -1;
  o->side = 0;
  o->t = INFINITY;
  for (int32_t cmp = 0; cmp < 4 * N + 8; ++cmp) {
    double tx = (rx != 0.0) ? (X0 + kx * sx - x) / rx : INFINITY;
    double ty = (ry != 0.0) ? (Y0 + ky * sy - y) / ry : INFINITY;
    int step_x = (tx < ty);
    if (isfinite(tx) && isfinite(ty)) {
      double big = tx > ty ? tx : ty;
      if (fabs(tx - ty) <= 1e-5 * big) {
        if (blocks(grid, N, door, door_open, doors, ix + sx, iy) ||
            blocks(grid, N, door, door_open, doors, ix, iy + sy) ||
            blocks(grid, N, door, door_open, doors, ix + sx, iy + sy)) {
          if (o->n_ties == 0) o->first_tie = cmp;
          o->n_ties += 1;
        }
      }
    }
    if (cmp == flip_at) step_x = !step_x;
    double tc;
    int32_t sd;
    if (step_x) { ix += sx; kx += 1; tc = tx; sd = 0; }
    else { iy += sy; ky += 1; tc = ty; sd = 1; }
    if (blocks(grid, N, door, door_open, doors, ix, iy)) {
      o->hit = (ix >= 0 && iy >= 0 && ix < N && iy < N) ? iy * N + ix : -1;
      o->side = sd;
      o->t = tc;
      return;
    }
  }
}

int32_t orc_cast(const uint8_t* grid, int32_t N, int32_t door, int32_t door_open, double x,
                 double y, double rx, double ry, int32_t* side, double* tstar, int32_t* flags) {
  cast_out o;
  cast_walk(grid, N, door, door_open, 0, x, y, rx, ry, -1, &o);
  if (side) *side = o.side;
  if (tstar) *tstar = o.t;
  if (flags) *flags = (o.n_ties > 0 ? ORC_CF_DDA : 0) | (o.n_ties > 1 ? ORC_CF_MULTI : 0);
  return o.hit;
}

/* Palette (the paper forgoes visual assets: the values are a convention, which the HIP path repeats independently). */
static const uint8_t kPal[8][3] = {{180, 40, 40},  {40, 160, 40}, {40, 60, 180},  {190, 170, 40},
                                   {150, 40, 170}, {40, 160, 170}, {200, 110, 30}, {150, 150, 150}};
static const uint8_t kCeil[3] = {50, 50, 60};
static const uint8_t kFloor[3] = {90, 80, 70};
static const uint8_t kDoor[3] = {120, 0, 0};
static const uint8_t kKeyCol[3] = {255, 40, 40};
static const uint8_t kGoalCol[3] = {255, 230, 0};
static const uint8_t kDecorCol[3] = {0, 200, 120};
/* ASCII maps: walls '1'..'9', doors by type, keys by colour */
static const uint8_t kWall9[9][3] = {{180, 40, 40},  {40, 160, 40},  {40, 60, 180},
                                     {190, 170, 40}, {150, 40, 170}, {40, 160, 170},
                                     {200, 110, 30}, {150, 150, 150}, {230, 230, 230}};
static const uint8_t kDoorCol[5][3] = {{120, 0, 0},   {0, 30, 130},  {140, 120, 0},
                                       {70, 110, 230}, {230, 200, 60}};
static const uint8_t kAKeyCol[3][3] = {{255, 40, 40}, {40, 110, 255}, {255, 200, 40}};

/* ------------------------------------------------------------------------ */
/* Frame.  Camera reading: horizontal FOV with tanH = tan(fov/2); column c   */
/* samples camX = (2c+1-W)/W and ray = dir + camX*tanH*right; since |dir| = 1 */
/* and right is perpendicular, the ray parameter at the hit is the           */
/* perpendicular (fisheye-corrected) distance t*.  Row r (pixel centre       */
/* r+0.5) is wall when |r+0.5-H/2| < H/(2 t*), else ceiling above the        */
/* horizon and floor below.  Wall colour: palette[id mod K], the door colour */
/* for the shut door; each channel halved (>> 1) on y-face hits.  Sprites    */
/* (Fig. 1: fixed billboards): key (not yet taken), goal (goal_sprite),      */
/* decor, in that index order; each a 0.5 x 0.5 solid square centred on its */
/* tile's centre at horizon height.  For d = centre - pos: depth tY = d.dir, */
/* lateral tX = d.right; drawn only when tY > 0.05; screen centre            */
/* u = (W/2)(1 + tX/(tanH tY)), half-width (W/2)*0.25/(tanH tY), half-height */
/* H*0.25/tY; column c covered when |c+0.5-u| < half-width and tY < t*_c;   */
/* row r when |r+0.5-H/2| < half-height.  Painted far to near (descending    */
/* tY; equal tY in ascending index, so the later index wins).                */
/* ------------------------------------------------------------------------ */
/* Marks the rows at distance k from the horizon (row H/2-1-k above, H/2+k
 * below) of column col in the tie mask. */
static void tie_pair(uint8_t* tie, int32_t H, int32_t W, int32_t col, int32_t k) {
  if (!tie || k < 0 || k >= H / 2) return;
  tie[(size_t)(H / 2 - 1 - k) * W + col] = 1;
  tie[(size_t)(H / 2 + k) * W + col] = 1;
}

/* Marks every row r of column col with |r + 0.5 - H/2| < extent (the rows a
 * wall span or a billboard of that half-height covers). */
static void tie_band(uint8_t* tie, int32_t H, int32_t W, int32_t col, double extent) {
  if (!tie) return;
  for (int32_t r = 0; r < H; ++r)
    if (fabs(r + 0.5 - H / 2.0) < extent) tie[(size_t)r * W + col] = 1;
}

int32_t orc_render_ex(const uint8_t* grid, const orc_cfg* cfg, const orc_state* st, int32_t branch,
                      uint8_t* obs, int32_t* hit, int32_t* side, double* tstar, int32_t* cflags,
                      int32_t* alt_hit, int32_t* alt_side, double* alt_t, uint8_t* tie) {
  if (!grid || !cfg || !st || !obs || (branch != 0 && branch != 1)) return -1;
  const int32_t N = cfg->side, H = cfg->obs_h, W = cfg->obs_w;
  const int32_t K = cfg->n_colors;
  if (W <= 0 || H <= 0 || K < 1 || K > 8) return -1;
  const double tanH = tan(cfg->fov_deg * M_PI / 360.0);
  const double c = cos(st->theta), s = sin(st->theta);
  const double dirx = c, diry = s, rgtx = -s, rgty = c;
  const int32_t door = st->door, dopen = st->door_open;
  const double half = H / 2.0;
  if (tie) memset(tie, 0, (size_t)H * W);

  double* tcol = (double*)malloc(sizeof(double) * (size_t)W);
  int32_t* fl = (int32_t*)calloc((size_t)W, sizeof(int32_t));

  for (int32_t col = 0; col < W; ++col) {
    double camX = (2.0 * col + 1.0 - W) / (double)W;
    double rx = dirx + camX * tanH * rgtx;
    double ry = diry + camX * tanH * rgty;
    cast_out o, a;
    cast_walk(grid, N, door, dopen, st->doors_open, st->x, st->y, rx, ry, -1, &o);
    if (o.n_ties > 0) fl[col] |= ORC_CF_DDA;
    if (o.n_ties > 1) fl[col] |= ORC_CF_MULTI;
    a.hit = -1;
    a.side = 0;
    a.t = 0.0;
    if (o.n_ties > 0)
      cast_walk(grid, N, door, dopen, st->doors_open, st->x, st->y, rx, ry, o.first_tie, &a);
    if (alt_hit) alt_hit[col] = a.hit;
    if (alt_side) alt_side[col] = a.side;
    if (alt_t) alt_t[col] = a.t;
    /* the walk this frame shows: branch 1 takes the other side of the first
     * flagged tie (the second valid result of the column, Sec. 2.1 DDA) */
    const cast_out* u = (branch == 1 && o.n_ties > 0) ? &a : &o;
    tcol[col] = u->t;
    if (hit) hit[col] = u->hit;
    if (side) side[col] = u->side;
    if (tstar) tstar[col] = u->t;

    uint8_t wc[3];
    const uint8_t hv = u->hit >= 0 ? grid[u->hit] : 1;
    const uint8_t* base;
    if (u->hit == door && !dopen) base = kDoor;
    else if (hv & ORC_TILE_DOOR) base = kDoorCol[(hv >> 4) & 7];
    else if ((hv & 0x0F) >= 2) base = kWall9[(hv & 0x0F) - 2];
    else base = kPal[(u->hit < 0 ? 0 : u->hit) % K];
    for (int32_t ch = 0; ch < 3; ++ch) wc[ch] = u->side ? (uint8_t)(base[ch] >> 1) : base[ch];
    double hh = H / (2.0 * u->t);
    if (cfg->shade_levels > 0) {
      /* Distance shading (the ray-casting section lets the wall colour depend
       * on the hit distance; this is the library's reading): S levels over
       * [0, D), level l = floor(t* S / D) capped at S - 1, and each channel of
       * the wall colour keeps the fraction (S - l) / S, rounded down. */
      const int32_t S = cfg->shade_levels;
      const double q = u->t * (double)S / cfg->shade_dist;
      int32_t lv = (int32_t)floor(q);
      if (lv > S - 1) lv = S - 1;
      for (int32_t ch = 0; ch < 3; ++ch) wc[ch] = (uint8_t)((wc[ch] * (S - lv)) / S);
      /* F4: the level boundaries are the integers 1..S-1 of q; the level
       * decides the colour of every wall row */
      for (int32_t k = 1; k < S; ++k)
        if (fabs(q - k) <= 1e-5 * q) {
          fl[col] |= ORC_CF_SHADE;
          tie_band(tie, H, W, col, hh);
        }
    }
    /* F2: a pixel centre within the window of the span's edge decides that
     * row pair */
    for (int32_t k = 0; k < H / 2; ++k)
      if (fabs(hh - (k + 0.5)) <= 1e-5 * hh) {
        fl[col] |= ORC_CF_SPAN;
        tie_pair(tie, H, W, col, k);
      }
    for (int32_t r = 0; r < H; ++r) {
      const uint8_t* px;
      if (fabs(r + 0.5 - half) < hh) px = wc;
      else if (r + 0.5 < half) px = kCeil;
      else px = kFloor;
      uint8_t* o3 = obs + ((size_t)r * W + col) * 3;
      o3[0] = px[0];
      o3[1] = px[1];
      o3[2] = px[2];
    }
  }

  /* sprites */
  int32_t sid[8];
  const uint8_t* scol[8];
  int32_t ns = 0;
  if (cfg->ascii_map) {
    /* keys not yet taken in colour order, then the goal */
    for (int32_t c = 0; c < 3; ++c)
      if (st->akey[c] >= 0 && !((st->akey_taken >> c) & 1)) { sid[ns] = st->akey[c]; scol[ns] = kAKeyCol[c]; ++ns; }
  }
  if (st->key >= 0 && !st->key_taken) { sid[ns] = st->key; scol[ns] = kKeyCol; ++ns; }
  if (cfg->goal_sprite && st->goal >= 0) { sid[ns] = st->goal; scol[ns] = kGoalCol; ++ns; }
  for (int32_t j = 0; j < st->n_decor && j < ORC_MAX_DECOR; ++j) {
    sid[ns] = st->decor[j];
    scol[ns] = kDecorCol;
    ++ns;
  }
  double tY[8], tX[8], u[8], hw[8], hs[8], dn[8];
  int32_t vis[8];
  for (int32_t j = 0; j < ns; ++j) {
    double cx = (sid[j] % N) + 0.5, cy = (sid[j] / N) + 0.5;
    double dx = cx - st->x, dy = cy - st->y;
    tY[j] = dx * dirx + dy * diry;
    tX[j] = dx * rgtx + dy * rgty;
    dn[j] = sqrt(dx * dx + dy * dy);
    vis[j] = tY[j] > 0.05;
    if (tY[j] > 0.0) {
      u[j] = (W / 2.0) * (1.0 + tX[j] / (tanH * tY[j]));
      hw[j] = (W / 2.0) * 0.25 / (tanH * tY[j]);
      hs[j] = H * 0.25 / tY[j];
    } else {
      u[j] = hw[j] = hs[j] = 0.0;
    }
  }
  /* painting order: descending tY, equal tY ascending index */
  int32_t order[8];
  for (int32_t j = 0; j < ns; ++j) order[j] = j;
  for (int32_t a = 0; a < ns; ++a)
    for (int32_t b = a + 1; b < ns; ++b) {
      int32_t p = order[a], q = order[b];
      if (tY[q] > tY[p] || (tY[q] == tY[p] && q < p)) { order[a] = q; order[b] = p; }
    }
  for (int32_t oi = 0; oi < ns; ++oi) {
    int32_t j = order[oi];
    if (!vis[j]) continue;
    for (int32_t col = 0; col < W; ++col) {
      if (!(fabs(col + 0.5 - u[j]) < hw[j] && tY[j] < tcol[col])) continue;
      for (int32_t r = 0; r < H; ++r) {
        if (!(fabs(r + 0.5 - half) < hs[j])) continue;
        uint8_t* o3 = obs + ((size_t)r * W + col) * 3;
        o3[0] = scol[j][0];
        o3[1] = scol[j][1];
        o3[2] = scol[j][2];
      }
    }
  }
  /* F3: sprite comparisons inside their windows.  A tied horizontal edge,
   * z-test or near clip decides whether the billboard shows on the column at
   * all (its rows are tied); a tied vertical edge decides one row pair; a tied
   * depth between two billboards decides which of them shows on their rows. */
  for (int32_t j = 0; j < ns; ++j) {
    if (tY[j] <= 0.0) continue;
    double wn = 1e-5 * (1.0 + dn[j]);
    double wu = 1e-5 * (1.0 + fabs(u[j]) + hw[j]) * (1.0 + dn[j] / tY[j]);
    int near_clip = fabs(tY[j] - 0.05) <= wn;
    if (!vis[j] && !near_clip) continue;
    for (int32_t col = 0; col < W; ++col) {
      double e = fabs(col + 0.5 - u[j]) - hw[j];
      if (e >= wu) continue; /* clearly outside horizontally */
      double wz = 1e-5 * (1.0 + dn[j] + tcol[col]);
      double zt = tY[j] - tcol[col];
      int flag = near_clip || fabs(e) < wu || fabs(zt) <= wz;
      if (flag) tie_band(tie, H, W, col, hs[j] * (1.0 + 1e-5));
      int covered = vis[j] && e < 0.0 && zt < 0.0;
      if (covered) {
        for (int32_t k = 0; k < H / 2; ++k)
          if (fabs(hs[j] - (k + 0.5)) <= 1e-5 * hs[j]) {
            flag = 1;
            tie_pair(tie, H, W, col, k);
          }
        for (int32_t q = 0; q < ns; ++q) {
          if (q == j || tY[q] <= 0.05) continue;
          if (fabs(col + 0.5 - u[q]) - hw[q] >= 1e-5 * (1.0 + fabs(u[q]) + hw[q]) * (1.0 + dn[q] / tY[q]))
            continue;
          if (fabs(tY[q] - tY[j]) <= 1e-5 * (1.0 + dn[j] + dn[q])) {
            flag = 1;
            tie_band(tie, H, W, col, hs[j] * (1.0 + 1e-5));
          }
        }
      }
      if (flag) fl[col] |= ORC_CF_SPRITE;
    }
  }
  if (cflags)
    for (int32_t col = 0; col < W; ++col) cflags[col] = fl[col];
  free(tcol);
  free(fl);
  return 0;
}

int32_t orc_render(const uint8_t* grid, const orc_cfg* cfg, const orc_state* st, uint8_t* obs,
                   int32_t* hit, int32_t* side, double* tstar, int32_t* cflags, int32_t* alt_hit,
                   int32_t* alt_side, double* alt_t) {
  return orc_render_ex(grid, cfg, st, 0, obs, hit, side, tstar, cflags, alt_hit, alt_side, alt_t, NULL);
}

int64_t orc_rollout(const orc_cfg* cfg, int32_t n_envs, const uint64_t* seeds, int32_t n_steps,
                    const uint8_t* actions, uint8_t* last_obs, int64_t* counts) {
  if (!cfg || n_envs < 0 || !seeds || n_steps < 0 || !actions) return -1;
  const int32_t N = cfg->side;
  const size_t fb = (size_t)cfg->obs_h * cfg->obs_w * 3;
  uint8_t* grid = (uint8_t*)malloc((size_t)N * N);
  uint8_t* obs = (uint8_t*)malloc(fb);
  int32_t* fl = (int32_t*)malloc(sizeof(int32_t) * (size_t)cfg->obs_w);
  int64_t done_steps = 0;
  if (counts) counts[0] = counts[1] = counts[2] = counts[3] = 0;
  for (int32_t i = 0; i < n_envs; ++i) {
    int32_t keys3[3];
    if (cfg->ascii_map ? orc_ascii(cfg->ascii_map, N, grid, keys3) < 0
                       : orc_maze(seeds[i], N, cfg->loop_frac, grid) < 0)
      break;
    orc_state st, nx;
    orc_reset(grid, cfg, seeds[i], 0, &st);
    for (int32_t t = 0; t < n_steps; ++t) {
      double r;
      int32_t d, ev, sf;
      orc_step(grid, cfg, seeds[i], &st, actions[(size_t)t * n_envs + i], &nx, &r, &d, &ev, &sf);
      st = nx;
      orc_render(grid, cfg, &st, obs, NULL, NULL, NULL, counts ? fl : NULL, NULL, NULL, NULL);
      if (counts) {
        /* columns rendered, columns flagged, F1 columns, steps flagged */
        counts[0] += cfg->obs_w;
        for (int32_t c = 0; c < cfg->obs_w; ++c) {
          counts[1] += fl[c] != 0;
          counts[2] += (fl[c] & ORC_CF_DDA) != 0;
        }
        counts[3] += sf != 0;
      }
      ++done_steps;
    }
    if (last_obs) memcpy(last_obs + (size_t)i * fb, obs, fb);
  }
  free(grid);
  free(obs);
  free(fl);
  return done_steps;
}

/* ---- training-buffer formats --------------------------------------------
 * Reading: the learner of the paper's training runs feeds 64x64 frames and the
 * previous action to a recurrent policy and stores 128-step rollouts (Sec. 3.1,
 * training hyperparameter table).  The paper does not say how frames are
 * normalised; this oracle takes the usual division of the byte by 255.  The
 * quotient is formed in double and rounded once to the target type: the
 * double of b/255 is itself a rounding, but b and 255 are exact in both
 * targets and double carries more than twice their precision plus two bits,
 * so that second rounding equals the direct one (the tests check every byte
 * against exact fractions). */
float orc_norm_f32(int32_t b) { return (float)((double)b / 255.0); }

/* Round-to-nearest-even of a double in [0, 1] to bfloat16 (8 significant
 * bits), done on the exponent and significand directly. */
uint16_t orc_norm_bf16(int32_t b) {
  const double q = (double)b / 255.0;
  if (q == 0.0) return 0;
  int e;
  const double m = frexp(q, &e);        /* q = m 2^e, m in [0.5, 1) */
  const double s = ldexp(m, 8);         /* in [128, 256), exact */
  const double f = floor(s), r = s - f;
  uint32_t k = (uint32_t)f;
  if (r > 0.5 || (r == 0.5 && (k & 1u))) ++k;
  const float v = (float)ldexp((double)k, e - 8);   /* exact in float */
  uint32_t bits;
  memcpy(&bits, &v, 4);
  return (uint16_t)(bits >> 16);
}

int64_t orc_format_frame(const uint8_t* hwc, int32_t H, int32_t W, int32_t layout,
                         int32_t dtype, void* out) {
  if (!hwc || !out || H <= 0 || W <= 0) return -1;
  if (layout != ORC_OBS_NHWC && layout != ORC_OBS_NCHW) return -1;
  if (dtype != ORC_OBS_U8 && dtype != ORC_OBS_BF16 && dtype != ORC_OBS_F32) return -1;
  const int64_t n = (int64_t)H * W * 3;
  for (int32_t r = 0; r < H; ++r)
    for (int32_t c = 0; c < W; ++c)
      for (int32_t ch = 0; ch < 3; ++ch) {
        const uint8_t b = hwc[((int64_t)r * W + c) * 3 + ch];
        const int64_t i = layout == ORC_OBS_NHWC ? ((int64_t)r * W + c) * 3 + ch
                                                 : ((int64_t)ch * H + r) * W + c;
        if (dtype == ORC_OBS_U8) ((uint8_t*)out)[i] = b;
        else if (dtype == ORC_OBS_BF16) ((uint16_t*)out)[i] = orc_norm_bf16(b);
        else ((float*)out)[i] = orc_norm_f32(b);
      }
  return n * (dtype == ORC_OBS_U8 ? 1 : dtype == ORC_OBS_BF16 ? 2 : 4);
}

/* Reading: the policy sees the action that led to the current frame; a frame
 * that opens an episode has none, coded as n_actions (one past the last
 * action, so a one-hot of width n_actions + 1 marks it).  An out-of-range
 * action moved nothing and is coded the same way. */
int32_t orc_prev_action(const orc_cfg* cfg, int32_t action, int32_t done) {
  if (!cfg) return -1;
  if (done || action < 0 || action >= cfg->n_actions) return cfg->n_actions;
  return action;
}
