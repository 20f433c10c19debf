// Host-side plan of a lattice: per-node pull codes, the canonical fluid-solid link list,
// and the tile classification the step kernel dispatches on.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"

namespace lbm {

// D2Q9 (Kaushal, Succi & Ansumali, Sec. II, Table I).
constexpr int kQ = 9;
constexpr int kCx[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[kQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// How the population of direction i reaching a fluid node is obtained (the "pull
// source" of the node for that direction).  Three bits per direction i = 1..8 at bit
// 3*(i-1) of the node word; bit 31 marks a solid node.
enum PullCode : uint32_t {
  kStream = 0,  // S_i(x - c_i), in the domain, fluid
  kBody = 1,    // x - c_i is a body node: half-way bounce-back S_opp(x)   (force-bearing)
  kWall = 2,    // no-slip wall, or the outlet ghost of a solid node: S_opp(x)
  kInlet = 3,   // moving-wall bounce-back at x = -1/2
  kOutlet = 4,  // ghost column nx holds column nx-1: S_i(nx-1, y - c_iy)
  kWrap = 5,    // periodic wrap, then plain streaming
};
constexpr uint32_t kSolidBit = 1u << 31;

constexpr uint32_t pull_code(uint32_t word, int i) { return (word >> (3 * (i - 1))) & 7u; }

// Tile shape of the step kernel: one 256-thread block covers kTileW x kTileH nodes.
constexpr int kTileW = 256;
constexpr int kTileH = 4;

struct Plan {
  int nx = 0, ny = 0, bc_x = 0, bc_y = 0;
  bool has_box = false;
  int box[4] = {-1, -1, -1, -1};
  std::vector<uint32_t> node;     // [ny*nx] pull codes + solid bit
  std::vector<int32_t> links;     // [L][2] (y*nx + x, i), canonical order
  int ntx = 0, nty = 0;           // tiles per row / column
  std::vector<int32_t> tile_slot; // -1: interior tile; >= 0: general tile, partial slot
  int nslots = 0;                 // general tiles
  int64_t n_fluid = 0, n_box = 0;
  // tail control-volume momentum sweep: blocks of kTileW nodes along each box row
  int box_bx = 0, box_rows = 0;
};

// Validate and classify.  Returns LBM_OK or an error code with a message in err.
int build_plan(const lbm_grid& g, const uint8_t* mask, Plan& p, std::string& err);

}  // namespace lbm
