// Host-side classification of every node and direction (the pull rules), the canonical
// link list, and the interior/general tile split of the step kernel.
#include "plan.h"

#include <algorithm>
#include <cstdio>

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

}  // namespace

int build_plan(const lbm_grid& g, const uint8_t* mask, Plan& p, std::string& err) {
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
  if (g.precision != LBM_FP64 && g.precision != LBM_FP32 && g.precision != LBM_FP16DEV &&
      g.precision != LBM_FP32DEV) {
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
  const size_t n = size_t(g.nx) * size_t(g.ny);
  for (size_t k = 0; k < n; ++k)
    if (mask[k] > 1) {
      std::snprintf(buf, sizeof buf, "mask byte %zu is %d (must be 0 or 1)", k, int(mask[k]));
      err = buf;
      return LBM_EINVAL;
    }
  p = Plan();
  p.nx = g.nx;
  p.ny = g.ny;
  p.bc_x = g.bc_x;
  p.bc_y = g.bc_y;
  p.has_box = g.box[0] >= 0;
  for (int k = 0; k < 4; ++k) p.box[k] = g.box[k];
  if (p.has_box) {
    const int x0 = g.box[0], x1 = g.box[1], y0 = g.box[2], y1 = g.box[3];
    if (x0 < 1 || y0 < 1 || x1 > g.nx - 1 || y1 > g.ny - 1 || x1 - x0 < 3 || y1 - y0 < 3) {
      err = "control-volume box must lie one node inside the domain and span >= 3 nodes";
      return LBM_EINVAL;
    }
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x)
        if (mask[size_t(y) * g.nx + x] && !(x >= x0 + 1 && x < x1 - 1 && y >= y0 + 1 && y < y1 - 1)) {
          std::snprintf(buf, sizeof buf,
                        "solid node (%d,%d) is not strictly inside the control-volume box", x, y);
          err = buf;
          return LBM_EINVAL;
        }
  }

  // Per-node pull codes.
  p.node.assign(n, 0u);
  for (int y = 0; y < g.ny; ++y)
    for (int x = 0; x < g.nx; ++x) {
      const size_t k = size_t(y) * g.nx + x;
      if (mask[k]) {
        p.node[k] = kSolidBit;
        continue;
      }
      ++p.n_fluid;
      if (in_box(p, x, y)) ++p.n_box;
      uint32_t w = 0;
      for (int i = 1; i < kQ; ++i) w |= classify(p, mask, x, y, i) << (3 * (i - 1));
      p.node[k] = w;
    }

  // Canonical link list: (x, i) with x + c_i a solid mask node, i.e. the pull of the
  // opposite direction bounces back from the body.
  for (int y = 0; y < g.ny; ++y)
    for (int x = 0; x < g.nx; ++x) {
      const size_t k = size_t(y) * g.nx + x;
      if (p.node[k] & kSolidBit) continue;
      for (int i = 1; i < kQ; ++i)
        if (pull_code(p.node[k], kOpp[i]) == kBody) {
          p.links.push_back(int32_t(k));
          p.links.push_back(i);
        }
    }

  // Rectangle of every node off the first and last rows whose codes need the general
  // path.  `band`: the nodes with a control-volume term (the box and the ring around it).
  auto band = [&](int x, int y) {
    return p.has_box && x >= p.box[0] - 1 && x <= p.box[1] && y >= p.box[2] - 1 &&
           y <= p.box[3];
  };
  for (int y = 1; y < g.ny - 1; ++y)
    for (int x = 0; x < g.nx; ++x) {
      if (p.node[size_t(y) * g.nx + x] == edge_word(g.nx, g.bc_x, x)) continue;
      if (p.gx0 > p.gx1) {
        p.gx0 = p.gx1 = x;
        p.gy0 = p.gy1 = y;
      } else {
        p.gx0 = std::min(p.gx0, x);
        p.gx1 = std::max(p.gx1, x);
        p.gy0 = std::min(p.gy0, y);
        p.gy1 = std::max(p.gy1, y);
      }
    }
  // Tiles and strips (strip_class).  General strips holding a link node or a node with a
  // control-volume term own a force-partial slot (kPart sums); box-interior strips own
  // a slot of the box-momentum partials (2 sums).
  p.ntx = (g.nx + kTileW - 1) / kTileW;
  p.nty = (g.ny + kTileH - 1) / kTileH;
  p.ntiles = p.ntx * p.nty;
  p.strip_slot.assign(size_t(p.ntiles) * kStrips, -1);
  for (int ty = 0; ty < p.nty; ++ty)
    for (int tx = 0; tx < p.ntx; ++tx)
      for (int w = 0; w < kStrips; ++w) {
        const int x0 = tx * kTileW + w * kStripW, y0 = ty * kTileH;
        const int cls = p.has_box
                            ? strip_class(g.nx, g.ny, p.gx0, p.gx1, p.gy0, p.gy1, p.box[0],
                                          p.box[1], p.box[2], p.box[3], x0, y0)
                            : strip_class(g.nx, g.ny, p.gx0, p.gx1, p.gy0, p.gy1, 1, 0, 1, 0,
                                          x0, y0);
        if (cls == kStripPlain) continue;
        if (cls == kStripBoxInterior) {
          p.strip_slot[(size_t(ty) * p.ntx + tx) * kStrips + w] = p.njslots++;
          continue;
        }
        ++p.ngeneral;
        bool forces = false;
        for (int y = y0; y < std::min(y0 + kTileH, g.ny); ++y)
          for (int x = x0; x < std::min(x0 + kStripW, g.nx); ++x) {
            const uint32_t wd = p.node[size_t(y) * g.nx + x];
            bool link = false;
            if (!(wd & kSolidBit))
              for (int i = 1; i < kQ; ++i) link = link || pull_code(wd, i) == kBody;
            forces = forces || link || band(x, y);
          }
        if (forces) p.strip_slot[(size_t(ty) * p.ntx + tx) * kStrips + w] = p.nslots++;
      }
  if (p.has_box) {
    p.box_bx = (p.box[1] - p.box[0] + kTileW - 1) / kTileW;
    p.box_rows = p.box[3] - p.box[2];
  }
  return LBM_OK;
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
