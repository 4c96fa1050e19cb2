// jx_layout.h -- host maze generator.
#pragma once
#include <stdint.h>

namespace jx {
// Writes the N x N grid (0 floor, 1 wall) for `seed`; false on bad arguments.
bool make_maze(uint64_t seed, int N, float loop_frac, uint8_t* grid);
}  // namespace jx
