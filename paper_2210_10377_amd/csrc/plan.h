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

// Tiles of the step kernel: one 256-thread block of four 64-lane waves, each wave a strip
// of 64 nodes of one row.  Wide tiles (1 row) put the four strips side by side (256 x 1),
// narrow tiles (4 rows) one above the other (64 x 4), for grids with short rows.
constexpr int kTileW = 256;  // threads of a block, nodes of a wide tile
constexpr int kStripW = 64;
constexpr int kStrips = kTileW / kStripW;

// Origin (x0, y0) of the strip of wave `wave` of tile `tile`, for tiles of `rows` rows
// (1 or 4) and ntx tiles along x.
constexpr void strip_origin(int tile, int wave, int ntx, int rows, int& x0, int& y0) {
  const int ty = tile / ntx, tx = tile - ty * ntx;
  x0 = rows == 1 ? tx * kTileW + wave * kStripW : tx * kStripW;
  y0 = rows == 1 ? ty : ty * rows + wave;
}
// Tile rows for a grid nx wide under the request `tile` (LBM_TILE_*): narrow when asked,
// or automatically when 256-node tiles would leave at least one idle wave per row of a
// grid of at most 1024 columns.
constexpr int tile_rows_for(int nx, int tile) {
  return tile == LBM_TILE_NARROW
             ? 4
             : (tile == LBM_TILE_WIDE
                    ? 1
                    : ((nx <= 1024 && (nx + kTileW - 1) / kTileW * kTileW - nx >= kStripW) ? 4 : 1));
}

// Pull-code word of a node that no body and no outlet bounce-back touches: the rules of
// the domain's edges alone, from the node's coordinates (the precedence of the plan:
// periodic wrap, then wall, inlet, outlet; plain streaming elsewhere).  At y = 0 the
// directions with c_y = +1 bounce back from the wall (periodic y: wrap), at y = ny - 1
// those with c_y = -1; at x = 0 those with c_x = +1 take the inlet rule (periodic x:
// wrap), at x = nx - 1 those with c_x = -1 the outlet rule (periodic x: wrap).
constexpr uint32_t edge_word(int nx, int ny, int bc_x, int bc_y, int x, int y) {
  uint32_t w = 0;
  for (int i = 1; i < kQ; ++i) {
    const int sx = x - kCx[i], sy = y - kCy[i];
    const bool out_x = sx < 0 || sx >= nx, out_y = sy < 0 || sy >= ny;
    uint32_t c = kStream;
    if (out_y && bc_y == LBM_BCY_WALL)
      c = kWall;
    else if (out_x && bc_x == LBM_BCX_INLET_OUTLET)
      c = sx < 0 ? kInlet : kOutlet;
    else if (out_x || out_y)
      c = kWrap;
    w |= c << (3 * (i - 1));
  }
  return w;
}

// edge_word by bit operations on whole words, for the kernels: a pattern holds 1 in the
// low bit of the 3-bit field of each direction of a set; a code times a pattern writes
// the code into those fields.  Equal to edge_word for every node (tested).
constexpr uint32_t dir_pattern(int cx, int cy) {  // directions with c_x = cx (or c_y = cy)
  uint32_t p = 0;
  for (int i = 1; i < kQ; ++i)
    if ((cx != 0 && kCx[i] == cx) || (cy != 0 && kCy[i] == cy)) p |= 1u << (3 * (i - 1));
  return p;
}
constexpr uint32_t edge_word_bits(int nx, int ny, int bc_x, int bc_y, int x, int y) {
  constexpr uint32_t kUp = dir_pattern(0, 1), kDown = dir_pattern(0, -1);
  constexpr uint32_t kRight = dir_pattern(1, 0), kLeft = dir_pattern(-1, 0);
  // Directions whose source lies beyond a bounded or periodic edge.
  const uint32_t py = (y == 0 ? kUp : 0u) | (y == ny - 1 ? kDown : 0u);
  const uint32_t pr = x == 0 ? kRight : 0u, pl = x == nx - 1 ? kLeft : 0u;
  const uint32_t px = pr | pl;
  if (bc_y == LBM_BCY_WALL) {
    const uint32_t xr = pr & ~py, xl = pl & ~py;
    return uint32_t(kWall) * py + (bc_x == LBM_BCX_PERIODIC
                                       ? uint32_t(kWrap) * (xr | xl)
                                       : uint32_t(kInlet) * xr + uint32_t(kOutlet) * xl);
  }
  return (bc_x == LBM_BCX_PERIODIC ? uint32_t(kWrap) * px
                                   : uint32_t(kInlet) * pr + uint32_t(kOutlet) * pl) +
         uint32_t(kWrap) * (py & ~px);
}

// A strip is "plain" when it stays outside the rectangle [gx0, gx1] x [gy0, gy1] that
// holds every node whose pull codes are not edge_word (bodies, their links, outlet
// bounce-backs): its nodes need no per-node metadata.  A plain strip is "interior" when
// it also stays off the first and last rows and holds neither x = 0 nor x = nx - 1 nor
// any x >= nx (plain streaming in every direction).  Host plan and kernels share these
// rules.
constexpr bool strip_is_plain(int nx, int ny, int gx0, int gx1, int gy0, int gy1, int x0,
                              int y0) {
  (void)nx;
  (void)ny;
  return !(y0 <= gy1 && y0 >= gy0 && x0 <= gx1 && x0 + kStripW - 1 >= gx0);
}
constexpr bool strip_is_interior(int nx, int ny, int x0, int y0) {
  return x0 > 0 && x0 + kStripW < nx && y0 > 0 && y0 + 1 < ny;
}

// Class of a strip for the forward step with forces, given the control volume
// [bx0, bx1) x [by0, by1) (bx0 > bx1: none):
//   kStripGeneral: per-node pull codes (not plain), or it touches the ring of nodes
//     within one node of the box surface (flux terms of DRTT) and is not interior;
//   kStripBoxInterior: plain and inside [bx0+1, bx1-2] x [by0+1, by1-2], where every
//     node is in the control volume with all its neighbours: only the box momentum J
//     is accumulated;
//   kStripBoxRing: plain and interior, touching the ring: plain streaming, with the
//     control-volume terms of each node from its coordinates;
//   kStripPlain: everything else (no force terms).
enum StripClass { kStripPlain = 0, kStripBoxInterior = 1, kStripGeneral = 2, kStripBoxRing = 3 };
constexpr int strip_class(int nx, int ny, int gx0, int gx1, int gy0, int gy1, int bx0, int bx1,
                          int by0, int by1, int x0, int y0) {
  if (!strip_is_plain(nx, ny, gx0, gx1, gy0, gy1, x0, y0)) return kStripGeneral;
  const int x1 = x0 + kStripW - 1, y1 = y0;
  if (bx0 > bx1 || y0 > by1 || y1 < by0 - 1 || x0 > bx1 || x1 < bx0 - 1) return kStripPlain;
  if (x0 >= bx0 + 1 && x1 <= bx1 - 2 && y0 >= by0 + 1 && y1 <= by1 - 2) return kStripBoxInterior;
  return strip_is_interior(nx, ny, x0, y0) ? kStripBoxRing : kStripGeneral;
}

struct Plan {
  int nx = 0, ny = 0, bc_x = 0, bc_y = 0;
  bool has_box = false;
  int box[4] = {-1, -1, -1, -1};
  std::vector<uint32_t> node;     // [ny*nx] pull codes + solid bit
  std::vector<int32_t> links;     // [L][2] (y*nx + x, i), canonical order
  int tile_rows = 1;              // 1: wide tiles (256 x 1), 4: narrow tiles (64 x 4)
  int ntx = 0, nty = 0, ntiles = 0;  // tiles per row / column / total
  // Inclusive node rectangle holding every node whose pull codes need the general path
  // (a solid node, codes other than edge_word); empty when gx0 > gx1.  The control
  // volume is classified separately (strip_class).
  int gx0 = 0, gx1 = -1, gy0 = 0, gy1 = -1;
  // Per strip (tile-major, kStrips per tile): the index >= 0 of its force-partial slot
  // when it holds a link node or a control-volume-band node (of its box-momentum slot
  // for a box-interior strip), else -1.  row_slot holds the same per strip in row-major
  // order ([ny][ceil(nx / 64)]), the order the slots are numbered in.
  std::vector<int32_t> strip_slot;
  std::vector<int32_t> row_slot;
  int nslots = 0;                 // general strips with force terms (kPart partials each)
  int njslots = 0;                // box-interior strips (2 partials each: J)
  int ngeneral = 0;               // strips that take the general path
  int64_t n_fluid = 0, n_box = 0;
  // tail control-volume momentum sweep: blocks of kTileW nodes along each box row
  int box_bx = 0, box_rows = 0;
};

// Validate and classify.  Returns LBM_OK or an error code with a message in err.
int build_plan(const lbm_grid& g, const uint8_t* mask, Plan& p, std::string& err);

// The per-strip slot table of tiles of `rows` rows (1: 256 x 1, 4: 64 x 4) over p's
// strips, with the tile counts along x and y: the same slots as p.strip_slot in another
// tile order.
void tile_slots(const Plan& p, int rows, int& ntx, int& nty, std::vector<int32_t>& out);

// Node words a mask change rewrites (index, old word, new word), in index order.
struct PlanDelta {
  std::vector<int64_t> idx;
  std::vector<uint32_t> old_w, new_w;
};

// The plan of a changed mask (and grid g, e.g. a moved control volume) built from the
// plan p of the old mask without re-classifying every node: only the changed nodes
// (`changed`: node indices where solid and fluid swap) and their lattice neighbours are
// re-classified; np receives the same plan build_plan would give, taking p's node words
// (p.node is left empty).  On an error nothing changes.  undo_replan gives p its plan
// back (for a change the caller then refuses).
int replan(const lbm_grid& g, const uint8_t* mask, const std::vector<int32_t>& changed,
           Plan& p, Plan& np, PlanDelta& d, std::string& err);
void apply_delta(Plan& p, const PlanDelta& d, bool forward);
void undo_replan(Plan& p, Plan& np, const PlanDelta& d);

// Adjoint codes: for a fluid node s and direction k (three bits at 3*(k-1)), which
// pulls read S_k(s) apart from the bounce-back of s itself: the node s + c_k streams it
// (kAdjStream), through a periodic wrap (kAdjWrap), or the outlet node
// (nx-1, s_y + c_ky) copies it from the ghost column (kAdjOutlet).  Built by inverting
// the pull codes, so the transposed pull reads exactly what the pull wrote.
constexpr uint32_t kAdjStream = 1u, kAdjWrap = 2u, kAdjOutlet = 4u;
void build_adjoint_codes(const Plan& p, std::vector<uint32_t>& adj);

}  // namespace lbm
