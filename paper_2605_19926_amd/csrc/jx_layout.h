// jx_layout.h -- host layout sources: the seeded maze generator and the ASCII
// map front-end.
#pragma once
#include <stdint.h>

#include <string>

namespace jx {
// Writes the N x N grid (0 floor, 1 wall) for `seed`; false on bad arguments.
bool make_maze(uint64_t seed, int N, float loop_frac, uint8_t* grid);

// Tile bytes shared by every layout source.  0 floor; low nibble 1 = default
// wall (colour palette[id mod K]), 2..10 = coloured wall '1'..'9'; bit 7 = door,
// with its type in bits 4..6 and its index (0..15, row-major) in bits 0..3.  On
// floor tiles bit 5 marks a spawn candidate and bit 6 a goal candidate.
constexpr uint8_t kTileDoor = 0x80, kTileSpawn = 0x20, kTileGoal = 0x40;
enum DoorType : int { kDoorRedLocked = 0, kDoorBlueLocked, kDoorYellowLocked, kDoorBlueUnlocked,
                      kDoorYellowUnlocked };
constexpr int kMaxDoors = 16;

// Parses an ASCII map (the paper's Table 2 symbols, rows separated by '\n')
// into the N x N grid: the text sits at the top-left, every tile it does not
// cover is a default wall.  keys[c] receives the tile of the red, blue, yellow
// key (-1 absent).  Returns the number of doors, or -1 with `why` set when the
// text is malformed, larger than N x N, has more than 16 doors, a key colour
// twice, no floor tile, or a border tile that is not a wall.
int parse_ascii_map(const char* text, int N, uint8_t* grid, int32_t keys[3], std::string* why);
}  // namespace jx
