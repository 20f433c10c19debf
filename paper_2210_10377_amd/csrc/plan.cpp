// Host-side classification of every node and direction (the pull rules), the canonical
// link list, and the interior/general tile split of the step kernel.
#include "plan.h"

#include <algorithm>
#include <cstdio>
#include <cstring>

namespace lbm {

namespace {

bool in_box(const Plan& p, int x, int y) {
  return p.has_box && x >= p.box[0] && x < p.box[1] && y >= p.box[2] && y < p.box[3];
}

// Code of the pull rule for fluid node (x, y), direction i (first match wins:
// periodic wrap > wall > inlet > outlet > body > stream).
uint32_t classify(const Plan& p, const uint8_t* mask, int x, int y, int i) {
  int sx = x - kCx[i], sy = y - kCy[i];
  bool wrapped = false;
  if (p.bc_x == LBM_BCX_PERIODIC && (sx < 0 || sx >= p.nx)) {
    sx = (sx + p.nx) % p.nx;
    wrapped = true;
  }
  if (p.bc_y == LBM_BCY_PERIODIC && (sy < 0 || sy >= p.ny)) {
    sy = (sy + p.ny) % p.ny;
    wrapped = true;
  }
  if (p.bc_y == LBM_BCY_WALL && (sy < 0 || sy >= p.ny)) return kWall;
  if (p.bc_x == LBM_BCX_INLET_OUTLET && sx < 0) return kInlet;
  if (p.bc_x == LBM_BCX_INLET_OUTLET && sx >= p.nx)
    return mask[size_t(sy) * p.nx + (p.nx - 1)] ? kWall : kOutlet;
  if (mask[size_t(sy) * p.nx + sx]) return kBody;
  return wrapped ? kWrap : kStream;
}

// Solid nodes of a mask: their number and bounding box (x0 > x1 when there is none).
struct Solids {
  int64_t count = 0;
  int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
};

// Checks of a grid and mask that need no plan: codes, sizes, mask bytes, and the
// control volume (one node inside the domain, every solid node strictly inside it).
// Fills the solid nodes' count and bounding box.
int validate(const lbm_grid& g, const uint8_t* mask, Solids& sol, std::string& err) {
  char buf[256];
  if (g.nx < 3 || g.ny < 3) {
    err = "nx and ny must be >= 3";
    return LBM_EINVAL;
  }
  if (g.bc_x != LBM_BCX_INLET_OUTLET && g.bc_x != LBM_BCX_PERIODIC) {
    err = "unknown bc_x";
    return LBM_EINVAL;
  }
  if (g.bc_y != LBM_BCY_WALL && g.bc_y != LBM_BCY_PERIODIC) {
    err = "unknown bc_y";
    return LBM_EINVAL;
  }
  if (g.tile != LBM_TILE_AUTO && g.tile != LBM_TILE_WIDE && g.tile != LBM_TILE_NARROW) {
    err = "unknown tile shape";
    return LBM_EINVAL;
  }
  if (g.precision != LBM_FP64 && g.precision != LBM_FP32 && g.precision != LBM_FP16DEV &&
      g.precision != LBM_FP32DEV && g.precision != LBM_FP32SR) {
    err = "unknown precision";
    return LBM_EINVAL;
  }
  if (g.collision != LBM_COLL_BGK && g.collision != LBM_COLL_REGULARIZED &&
      g.collision != LBM_COLL_KBC) {
    err = "unknown collision";
    return LBM_EINVAL;
  }
  if (g.max_record < 1) {
    err = "max_record must be >= 1";
    return LBM_EINVAL;
  }
  // One population plane must stay below 2^31 elements (32-bit in-plane offsets).
  const int64_t pitch = (int64_t(g.nx) + 63) / 64 * 64 + 256;  // row padding margin
  if (pitch * int64_t(g.ny) + 4096 >= (int64_t(1) << 31)) {
    err = "grid too large";
    return LBM_ENOMEM;
  }
  // Mask bytes, and the bounding box of the solid nodes (the control volume holds every
  // solid node strictly inside it exactly when it holds their bounding box).
  int sx0 = g.nx, sx1 = -1, sy0 = g.ny, sy1 = -1, fx = 0, fy = 0;
  int64_t count = 0;
  for (int y = 0; y < g.ny; ++y) {
    const uint8_t* row = mask + size_t(y) * g.nx;
    for (int x = 0; x < g.nx; ++x) {
      if (x + 8 <= g.nx) {  // skip eight fluid nodes at a time
        uint64_t v;
        std::memcpy(&v, row + x, 8);
        if (v == 0) {
          x += 7;
          continue;
        }
      }
      if (row[x] == 0) continue;
      ++count;
      if (row[x] > 1) {
        std::snprintf(buf, sizeof buf, "mask byte %zu is %d (must be 0 or 1)",
                      size_t(y) * g.nx + x, int(row[x]));
        err = buf;
        return LBM_EINVAL;
      }
      if (sx1 < 0) {
        fx = x;
        fy = y;
      }
      sx0 = std::min(sx0, x);
      sx1 = std::max(sx1, x);
      sy0 = std::min(sy0, y);
      sy1 = std::max(sy1, y);
    }
  }
  sol.count = count;
  sol.x0 = sx0;
  sol.x1 = sx1;
  sol.y0 = sy0;
  sol.y1 = sy1;
  if (g.box[0] >= 0) {
    const int x0 = g.box[0], x1 = g.box[1], y0 = g.box[2], y1 = g.box[3];
    if (x0 < 1 || y0 < 1 || x1 > g.nx - 1 || y1 > g.ny - 1 || x1 - x0 < 3 || y1 - y0 < 3) {
      err = "control-volume box must lie one node inside the domain and span >= 3 nodes";
      return LBM_EINVAL;
    }
    if (sx1 >= 0 && !(sx0 >= x0 + 1 && sx1 < x1 - 1 && sy0 >= y0 + 1 && sy1 < y1 - 1)) {
      // Name one offending node.
      for (int y = sy0; y <= sy1; ++y)
        for (int x = sx0; x <= sx1; ++x)
          if (mask[size_t(y) * g.nx + x] &&
              !(x >= x0 + 1 && x < x1 - 1 && y >= y0 + 1 && y < y1 - 1)) {
            fx = x;
            fy = y;
            y = sy1 + 1;
            break;
          }
      std::snprintf(buf, sizeof buf,
                    "solid node (%d,%d) is not strictly inside the control-volume box", fx, fy);
      err = buf;
      return LBM_EINVAL;
    }
  }
  return LBM_OK;
}

void set_geometry(Plan& p, const lbm_grid& g) {
  p.nx = g.nx;
  p.ny = g.ny;
  p.bc_x = g.bc_x;
  p.bc_y = g.bc_y;
  p.has_box = g.box[0] >= 0;
  for (int k = 0; k < 4; ++k) p.box[k] = g.box[k];
  p.tile_rows = tile_rows_for(g.nx, g.tile);
}

uint32_t node_word(const Plan& p, const uint8_t* mask, int x, int y) {
  if (mask[size_t(y) * p.nx + x]) return kSolidBit;
  uint32_t w = 0;
  for (int i = 1; i < kQ; ++i) w |= classify(p, mask, x, y, i) << (3 * (i - 1));
  return w;
}

// Everything the plan derives from its node words and geometry: node counts, the
// general rectangle, the canonical link list, strip classes and slots, the box sweep.
void derive(Plan& p, const Solids& sol) {
  const int nx = p.nx, ny = p.ny;
  p.n_fluid = int64_t(nx) * ny - sol.count;
  p.n_box = 0;
  if (p.has_box)
    for (int y = p.box[2]; y < p.box[3]; ++y)
      for (int x = p.box[0]; x < p.box[1]; ++x)
        p.n_box += (p.node[size_t(y) * nx + x] & kSolidBit) ? 0 : 1;

  // Rectangle of every node whose codes need the general path.  `band`: the nodes with
  // a control-volume term (the box and the ring around it).
  auto band = [&](int x, int y) {
    return p.has_box && x >= p.box[0] - 1 && x <= p.box[1] && y >= p.box[2] - 1 &&
           y <= p.box[3];
  };
  p.gx0 = 0;
  p.gx1 = -1;
  p.gy0 = 0;
  p.gy1 = -1;
  // Every such node is a solid node or the neighbour of one (a pull from a solid node,
  // or the outlet rule reading a solid node of the last column), so only the solid
  // nodes' bounding box grown by one node (the whole axis when that crosses a periodic
  // edge) is scanned.
  int xa = sol.x0 - 1, xb = sol.x1 + 1, ya = sol.y0 - 1, yb = sol.y1 + 1;
  if (p.bc_x == LBM_BCX_PERIODIC && (xa < 0 || xb > nx - 1)) {
    xa = 0;
    xb = nx - 1;
  }
  if (p.bc_y == LBM_BCY_PERIODIC && (ya < 0 || yb > ny - 1)) {
    ya = 0;
    yb = ny - 1;
  }
  xa = std::max(xa, 0);
  xb = std::min(xb, nx - 1);
  ya = std::max(ya, 0);
  yb = std::min(yb, ny - 1);
  if (sol.count == 0) yb = ya - 1;
  for (int y = ya; y <= yb; ++y) {
    const uint32_t* row = p.node.data() + size_t(y) * nx;
    // Away from x = 0 and x = nx - 1 the edge word of a row is one value.
    const uint32_t emid = edge_word(nx, ny, p.bc_x, p.bc_y, nx / 2, y);
    int lo = -1, hi = -1;
    for (int x = xa; x <= xb; ++x)
      if (row[x] != ((x == 0 || x == nx - 1) ? edge_word(nx, ny, p.bc_x, p.bc_y, x, y) : emid)) {
        if (lo < 0) lo = x;
        hi = x;
      }
    if (lo < 0) continue;
    if (p.gx0 > p.gx1) {
      p.gx0 = lo;
      p.gx1 = hi;
      p.gy0 = p.gy1 = y;
    } else {
      p.gx0 = std::min(p.gx0, lo);
      p.gx1 = std::max(p.gx1, hi);
      p.gy1 = y;
    }
  }

  // Canonical link list: (x, i) with x + c_i a solid mask node, i.e. the pull of the
  // opposite direction bounces back from the body.  Off the first and last rows such
  // nodes lie in the general rectangle.
  p.links.clear();
  auto scan_links = [&](int y, int xa, int xb) {
    for (int x = xa; x <= xb; ++x) {
      const size_t k = size_t(y) * nx + x;
      if (p.node[k] & kSolidBit) continue;
      for (int i = 1; i < kQ; ++i)
        if (pull_code(p.node[k], kOpp[i]) == kBody) {
          p.links.push_back(int32_t(k));
          p.links.push_back(i);
        }
    }
  };
  for (int y = 0; y < ny; ++y) {
    if (y == 0 || y == ny - 1)
      scan_links(y, 0, nx - 1);
    else if (p.gx0 <= p.gx1 && y >= p.gy0 && y <= p.gy1)
      scan_links(y, p.gx0, p.gx1);
  }

  // Strips (strip_class) in row-major order, y then x: general strips holding a link
  // node or a node with a control-volume term own a force-partial slot (kPart sums);
  // box-interior strips own a slot of the box-momentum partials.  The slots are numbered
  // in this order whatever the tile shape, so every shape reduces the same partials in
  // the same order (bitwise the same forces).
  const int nsx = (nx + kStripW - 1) / kStripW;
  p.row_slot.assign(size_t(ny) * nsx, -1);
  p.nslots = p.njslots = p.ngeneral = 0;
  for (int y0 = 0; y0 < ny; ++y0)
    for (int sx = 0; sx < nsx; ++sx) {
      const int x0 = sx * kStripW;
      const int cls = p.has_box
                          ? strip_class(nx, ny, p.gx0, p.gx1, p.gy0, p.gy1, p.box[0], p.box[1],
                                        p.box[2], p.box[3], x0, y0)
                          : strip_class(nx, ny, p.gx0, p.gx1, p.gy0, p.gy1, 1, 0, 1, 0, x0, y0);
      int32_t& slot = p.row_slot[size_t(y0) * nsx + sx];
      if (cls == kStripPlain) continue;
      if (cls == kStripBoxInterior) {
        slot = p.njslots++;
        continue;
      }
      if (cls == kStripGeneral) ++p.ngeneral;
      bool forces = false;
      for (int x = x0; x < std::min(x0 + kStripW, nx); ++x) {
        const uint32_t wd = p.node[size_t(y0) * nx + x];
        bool link = false;
        if (!(wd & kSolidBit))
          for (int i = 1; i < kQ; ++i) link = link || pull_code(wd, i) == kBody;
        forces = forces || link || band(x, y0);
      }
      if (forces) slot = p.nslots++;
    }
  tile_slots(p, p.tile_rows, p.ntx, p.nty, p.strip_slot);
  p.ntiles = p.ntx * p.nty;
  p.box_bx = p.box_rows = 0;
  if (p.has_box) {
    p.box_bx = (p.box[1] - p.box[0] + kTileW - 1) / kTileW;
    p.box_rows = p.box[3] - p.box[2];
  }
}

}  // namespace

int build_plan(const lbm_grid& g, const uint8_t* mask, Plan& p, std::string& err) {
  Solids sol;
  const int rc = validate(g, mask, sol, err);
  if (rc != LBM_OK) return rc;
  p = Plan();
  set_geometry(p, g);
  p.node.assign(size_t(g.nx) * size_t(g.ny), 0u);
  for (int y = 0; y < g.ny; ++y)
    for (int x = 0; x < g.nx; ++x) p.node[size_t(y) * g.nx + x] = node_word(p, mask, x, y);
  derive(p, sol);
  return LBM_OK;
}

int replan(const lbm_grid& g, const uint8_t* mask, const std::vector<int32_t>& changed,
           Plan& p, Plan& np, PlanDelta& d, std::string& err) {
  Solids sol;
  const int rc = validate(g, mask, sol, err);
  if (rc != LBM_OK) return rc;
  // Node words that can change: those of the changed nodes and of their lattice
  // neighbours (a pull reads its source node, and the outlet rule the last column of
  // the neighbouring rows).
  Plan geo;
  set_geometry(geo, g);
  std::vector<int64_t> idx;
  idx.reserve(changed.size() * kQ);
  for (int32_t c : changed) {
    const int x = c % g.nx, y = c / g.nx;
    for (int i = 0; i < kQ; ++i) {
      int ax = x + kCx[i], ay = y + kCy[i];
      if (g.bc_x == LBM_BCX_PERIODIC) ax = (ax + g.nx) % g.nx;
      if (g.bc_y == LBM_BCY_PERIODIC) ay = (ay + g.ny) % g.ny;
      if (ax < 0 || ax >= g.nx || ay < 0 || ay >= g.ny) continue;
      idx.push_back(int64_t(ay) * g.nx + ax);
    }
  }
  std::sort(idx.begin(), idx.end());
  idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
  d = PlanDelta();
  for (int64_t k : idx) {
    const uint32_t w = node_word(geo, mask, int(k % g.nx), int(k / g.nx));
    if (w == p.node[size_t(k)]) continue;
    d.idx.push_back(k);
    d.old_w.push_back(p.node[size_t(k)]);
    d.new_w.push_back(w);
  }
  // The new plan takes p's words (no copy) with the delta applied.
  apply_delta(p, d, true);
  np = Plan();
  set_geometry(np, g);
  np.node.swap(p.node);
  derive(np, sol);
  return LBM_OK;
}

void tile_slots(const Plan& p, int rows, int& ntx, int& nty, std::vector<int32_t>& out) {
  const int tile_w = kTileW / rows;
  ntx = (p.nx + tile_w - 1) / tile_w;
  nty = (p.ny + rows - 1) / rows;
  const int nsx = (p.nx + kStripW - 1) / kStripW;
  out.assign(size_t(ntx) * nty * kStrips, -1);
  for (int tile = 0; tile < ntx * nty; ++tile)
    for (int w = 0; w < kStrips; ++w) {
      int x0 = 0, y0 = 0;
      strip_origin(tile, w, ntx, rows, x0, y0);
      if (y0 < p.ny && x0 < p.nx)
        out[size_t(tile) * kStrips + w] = p.row_slot[size_t(y0) * nsx + x0 / kStripW];
    }
}

void apply_delta(Plan& p, const PlanDelta& d, bool forward) {
  for (size_t j = 0; j < d.idx.size(); ++j)
    p.node[size_t(d.idx[j])] = forward ? d.new_w[j] : d.old_w[j];
}

void undo_replan(Plan& p, Plan& np, const PlanDelta& d) {
  p.node.swap(np.node);
  apply_delta(p, d, false);
}

void build_adjoint_codes(const Plan& p, std::vector<uint32_t>& adj) {
  adj.assign(p.node.size(), 0u);
  for (int y = 0; y < p.ny; ++y)
    for (int x = 0; x < p.nx; ++x) {
      const uint32_t w = p.node[size_t(y) * p.nx + x];
      if (w & kSolidBit) continue;
      for (int i = 1; i < kQ; ++i) {
        const uint32_t c = pull_code(w, i);
        int sx = x - kCx[i], sy = y - kCy[i];
        sx = (sx + p.nx) % p.nx;
        sy = (sy + p.ny) % p.ny;
        uint32_t bit = 0;
        if (c == kStream) {
          bit = kAdjStream;
        } else if (c == kWrap) {
          bit = kAdjWrap;
        } else if (c == kOutlet) {
          bit = kAdjOutlet;
          sx = p.nx - 1;
        } else {
          continue;  // bounce-back: read back from the node itself
        }
        adj[size_t(sy) * p.nx + sx] |= bit << (3 * (i - 1));
      }
    }
}

}  // namespace lbm
