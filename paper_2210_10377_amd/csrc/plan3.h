// Host-side plan of the three-dimensional (D3Q27) path: per-node pull words, per-strip
// classes and force slots, from the mask and the boundary codes (C ABI in lbm3d.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lbm3d.h"

namespace lbm3 {

constexpr int kQ = 27;
// Directions: rest; faces +x -x +y -y +z -z; edges (xy, xz, yz planes, each ++ -- +- -+);
// corners +++ --- ++- --+ +-+ -+- -++ +--.  Direction 2k is opposite to 2k - 1.
constexpr int kCx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                         0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kCy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0,
                         1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kCz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1,
                         1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

constexpr int kTileW = 256;   // nodes of a tile (one block) along x
constexpr int kStripW = 64;   // nodes of a strip (one wave)
constexpr int kStrips = kTileW / kStripW;

// Node word: bit 31 the node is solid; bit i (1..26) the pull of direction i is a
// bounce-back from a solid source (a body node, or the outlet ghost of a solid node).
// Walls, the inlet and periodic wraps follow from the coordinates.
constexpr uint32_t kSolid = 1u << 31;

// Strip table entry: class in bits 30-31, slot index in bits 0-29; kStripEmpty for a
// strip wholly past nx.
enum : uint32_t {
  kPlain = 0u,    // interior, no boundary, outside the control-volume band: streaming path
  kBoxJ = 1u,     // inside V away from its surface: streaming path + J (3-double slot)
  kForce = 2u,    // general path with force terms (15-double slot)
  kEdge = 3u,     // general path without force terms
};
constexpr uint32_t kStripEmpty = 0xffffffffu;
constexpr uint32_t strip_class(uint32_t e) { return e >> 30; }
constexpr uint32_t strip_slot(uint32_t e) { return e & 0x3fffffffu; }

constexpr int kPart = 15;  // FA(3) FB(3) J(3) Phi(3) SI(3)
constexpr int kRow = 18;   // ring row: the 15 record values and J(t+1)(3)

struct Plan3 {
  int nx = 0, ny = 0, nz = 0, bc_x = 0, bc_y = 0, bc_z = 0;
  bool has_box = false;
  int box[6] = {-1, -1, -1, -1, -1, -1};
  bool whole[3] = {false, false, false};  // box spans the whole (periodic) axis
  std::vector<uint32_t> word;   // [nz][ny][nx]
  std::vector<uint32_t> strip;  // [ntiles * kStrips]
  std::vector<uint32_t> fstrips;  // [nslots] strip index of each force slot
  int ntx = 0;                  // tiles per row
  int64_t ntiles = 0;
  int nslots = 0, njslots = 0, ngeneral = 0;
  int64_t n_fluid = 0, n_links = 0, n_box = 0;
  int box_bx = 0, box_rows = 0;  // control-volume sweep: blocks per box row, box rows
};

int build_plan3(const lbm3d_grid& g, const uint8_t* mask, Plan3& p, std::string& err);

// Node words a mask change rewrites (index, old word, new word), in index order.
struct Plan3Delta {
  std::vector<int64_t> idx;
  std::vector<uint32_t> old_w, new_w;
};

// The plan of a changed mask (and grid g, e.g. a moved control volume) from the plan p
// of the old mask: the changed nodes (`changed`: node indices where solid and fluid
// swap), the nodes that pull from them and the strips around them are re-classified, the
// strips around the old and new control volume when it moved, and the slots renumbered;
// np receives the plan build_plan3 would give, taking p's words (p.word is left empty).
// On an error nothing changes; undo_replan3 gives p its plan back.
int replan3(const lbm3d_grid& g, const uint8_t* mask, const std::vector<int32_t>& changed,
            Plan3& p, Plan3& np, Plan3Delta& d, std::string& err);
void apply_delta3(Plan3& p, const Plan3Delta& d, bool forward);
void undo_replan3(Plan3& p, Plan3& np, const Plan3Delta& d);
// Body links (node, direction) in (z, y, x, direction) order.
void plan3_links(const Plan3& p, std::vector<int64_t>& out);

}  // namespace lbm3
