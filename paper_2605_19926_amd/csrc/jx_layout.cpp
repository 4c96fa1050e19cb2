// jx_layout.cpp -- host generator of the per-env tile maps (runs at reset, off the
// timed path).  The paper's worlds are tile maps (Sec. 2.2, Sec. 3.2, Table 2);
// the synthetic mazes here are recursive-backtracker depth-first-search mazes on
// the lattice of odd tiles, with a fraction of the remaining separator walls
// opened to make loops.
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "jx_layout.h"

namespace jx {

namespace {

struct SplitMix {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform in [0, n): top 32 bits times n, high word
  uint32_t draw(uint32_t n) { return (uint32_t)(((next() >> 32) * (uint64_t)n) >> 32); }
};

// Order-statistics over a fixed list: find and remove the r-th remaining item.
class Remaining {
 public:
  explicit Remaining(int n) : n_(n), tree_(n + 1, 0) {
    for (int i = 1; i <= n; ++i) {
      tree_[i] += 1;
      int j = i + (i & -i);
      if (j <= n) tree_[j] += tree_[i];
    }
    top_ = 1;
    while (top_ * 2 <= n_) top_ *= 2;
  }
  // index of the r-th (0-based) remaining item; removes it
  int take(int r) {
    int pos = 0, rem = r;
    for (int step = top_; step > 0; step >>= 1) {
      int nx = pos + step;
      if (nx <= n_ && tree_[nx] <= rem) {
        pos = nx;
        rem -= tree_[nx];
      }
    }
    for (int i = pos + 1; i <= n_; i += i & -i) tree_[i] -= 1;
    return pos;  // 0-based index
  }

 private:
  int n_, top_;
  std::vector<int> tree_;
};

}  // namespace

bool make_maze(uint64_t seed, int N, float loop_frac, uint8_t* grid) {
  if (N < 5 || N > 64 || !(loop_frac >= 0.f && loop_frac <= 1.f)) return false;
  const int m = (N - 1) / 2;
  std::memset(grid, 1, (size_t)N * N);
  SplitMix rng{seed};
  std::vector<uint8_t> seen((size_t)m * m, 0);
  std::vector<int> stack;
  stack.reserve((size_t)m * m);
  const int start = (int)rng.draw((uint32_t)(m * m));
  seen[start] = 1;
  grid[(2 * (start / m) + 1) * N + 2 * (start % m) + 1] = 0;
  stack.push_back(start);
  while (!stack.empty()) {
    const int cell = stack.back();
    const int ci = cell % m, cj = cell / m;
    int opts[4], n_opts = 0;
    // north, east, south, west
    if (cj > 0 && !seen[cell - m]) opts[n_opts++] = cell - m;
    if (ci + 1 < m && !seen[cell + 1]) opts[n_opts++] = cell + 1;
    if (cj + 1 < m && !seen[cell + m]) opts[n_opts++] = cell + m;
    if (ci > 0 && !seen[cell - 1]) opts[n_opts++] = cell - 1;
    if (n_opts == 0) {
      stack.pop_back();
      continue;
    }
    const int nb = opts[rng.draw((uint32_t)n_opts)];
    const int ni = nb % m, nj = nb / m;
    grid[(ci + ni + 1) + (cj + nj + 1) * N] = 0;      // wall tile between the two cells
    grid[(2 * nj + 1) * N + 2 * ni + 1] = 0;          // the neighbour cell
    seen[nb] = 1;
    stack.push_back(nb);
  }
  // loop walls: standing separators, row-major
  std::vector<int> sep;
  for (int yy = 1; yy <= 2 * m - 1; ++yy)
    for (int xx = 1; xx <= 2 * m - 1; ++xx)
      if (((xx & 1) == 0) != ((yy & 1) == 0) && grid[yy * N + xx]) sep.push_back(yy * N + xx);
  const int C = (int)sep.size();
  const int k = (int)std::floor((double)loop_frac * (double)C + 0.5);
  if (k > 0) {
    Remaining rem(C);
    for (int j = 0; j < k; ++j) grid[sep[rem.take((int)rng.draw((uint32_t)(C - j)))]] = 0;
  }
  return true;
}

}  // namespace jx

namespace jx {

int parse_ascii_map(const char* text, int N, uint8_t* grid, int32_t keys[3], std::string* why) {
  auto fail = [&](const char* m) {
    if (why) *why = m;
    return -1;
  };
  if (!text || !grid || N < 5 || N > 64) return fail("bad arguments");
  for (int i = 0; i < N * N; ++i) grid[i] = 1;
  keys[0] = keys[1] = keys[2] = -1;
  int col = 0, row = 0, n_doors = 0, n_floor = 0;
  for (const char* p = text; *p != '\0'; ++p) {
    const char ch = *p;
    if (ch == '\r') continue;
    if (ch == '\n') {
      ++row;
      col = 0;
      continue;
    }
    if (row >= N || col >= N) return fail("ascii map larger than side x side");
    uint8_t tile = 0;
    switch (ch) {
      case '#': tile = 1; break;
      case '.':
      case ' ': tile = 0; break;
      case 'S': tile = kTileSpawn; break;
      case 'G': tile = kTileGoal; break;
      case 'r':
      case 'b':
      case 'y': {
        const int k = (ch == 'r') ? 0 : (ch == 'b') ? 1 : 2;
        if (keys[k] >= 0) return fail("ascii map has two keys of one colour");
        keys[k] = row * N + col;
        break;
      }
      case 'R':
      case 'B':
      case 'Y':
      case '"':
      case '\\': {
        if (n_doors == kMaxDoors) return fail("ascii map has more than 16 doors");
        const int type = (ch == 'R') ? kDoorRedLocked : (ch == 'B') ? kDoorBlueLocked
                         : (ch == 'Y') ? kDoorYellowLocked : (ch == '"') ? kDoorBlueUnlocked
                                                                          : kDoorYellowUnlocked;
        tile = (uint8_t)(kTileDoor | (type << 4) | n_doors);
        ++n_doors;
        break;
      }
      default:
        if (ch < '1' || ch > '9') return fail("ascii map has an unknown symbol");
        tile = (uint8_t)(ch - '1' + 2);
    }
    if ((tile & 0x8F) == 0) ++n_floor;
    grid[row * N + col] = tile;
    ++col;
  }
  if (n_floor == 0) return fail("ascii map has no floor tile");
  for (int k = 0; k < N; ++k) {
    const uint8_t e[4] = {grid[k], grid[(N - 1) * N + k], grid[k * N], grid[k * N + N - 1]};
    for (uint8_t v : e)
      if ((v & kTileDoor) || (v & 0x0F) == 0) return fail("ascii map border tiles must be walls");
  }
  return n_doors;
}

}  // namespace jx
