// Host-side plan of the three-dimensional path (see plan3.h).
#include "plan3.h"

#include <algorithm>

namespace lbm3 {

namespace {

struct Geo {
  int n[3];
  bool per[3];
  bool wrap(int* p) const {  // wraps periodic axes; false if outside a bounded axis
    for (int a = 0; a < 3; ++a) {
      if (per[a]) p[a] = (p[a] % n[a] + n[a]) % n[a];
      if (p[a] < 0 || p[a] >= n[a]) return false;
    }
    return true;
  }
  int64_t index(const int* p) const { return (int64_t(p[2]) * n[1] + p[1]) * n[0] + p[0]; }
};

}  // namespace

int build_plan3(const lbm3d_grid& g, const uint8_t* mask, Plan3& p, std::string& err) {
  if (g.nx < 2 || g.ny < 2 || g.nz < 2) {
    err = "nx, ny and nz must be >= 2";
    return LBM_EINVAL;
  }
  if (int64_t(g.nx) * g.ny * g.nz >= (int64_t(1) << 31)) {
    err = "nx*ny*nz must be < 2^31";
    return LBM_ENOMEM;
  }
  if ((g.bc_x != LBM_BCX_INLET_OUTLET && g.bc_x != LBM_BCX_PERIODIC) ||
      (g.bc_y != LBM_BCY_WALL && g.bc_y != LBM_BCY_PERIODIC) ||
      (g.bc_z != LBM_BCY_WALL && g.bc_z != LBM_BCY_PERIODIC)) {
    err = "unknown boundary code";
    return LBM_EINVAL;
  }
  p = Plan3();
  p.nx = g.nx;
  p.ny = g.ny;
  p.nz = g.nz;
  p.bc_x = g.bc_x;
  p.bc_y = g.bc_y;
  p.bc_z = g.bc_z;
  const Geo geo{{g.nx, g.ny, g.nz},
                {g.bc_x == LBM_BCX_PERIODIC, g.bc_y == LBM_BCY_PERIODIC,
                 g.bc_z == LBM_BCY_PERIODIC}};
  const int64_t N = int64_t(g.nx) * g.ny * g.nz;
  for (int64_t k = 0; k < N; ++k)
    if (mask[k] > 1) {
      err = "mask values must be 0 or 1";
      return LBM_EINVAL;
    }
  // Control volume, axis by axis.
  p.has_box = g.box[0] >= 0;
  if (p.has_box) {
    for (int a = 0; a < 3; ++a) {
      const int b0 = g.box[2 * a], b1 = g.box[2 * a + 1];
      p.box[2 * a] = b0;
      p.box[2 * a + 1] = b1;
      p.whole[a] = geo.per[a] && b0 == 0 && b1 == geo.n[a];
      if (!p.whole[a] && (b0 < 1 || b1 > geo.n[a] - 1 || b1 - b0 < 3)) {
        err = "control volume must lie one node inside the domain (or span a periodic axis)";
        return LBM_EINVAL;
      }
    }
  }
  auto in_box = [&](const int* q) {
    for (int a = 0; a < 3; ++a)
      if (!p.whole[a] && (q[a] < p.box[2 * a] || q[a] >= p.box[2 * a + 1])) return false;
    return true;
  };
  // Node words: solid bit; bounce-back bits from every solid node to the nodes that
  // pull from it (a source inside the domain is never a wall or inlet case).
  p.word.assign(size_t(N), 0u);
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const int64_t k = (int64_t(z) * g.ny + y) * g.nx + x;
        if (!mask[k]) continue;
        p.word[k] |= kSolid;
        if (p.has_box) {
          const int q[3] = {x, y, z};
          for (int a = 0; a < 3; ++a)
            if (!p.whole[a] && !(q[a] >= p.box[2 * a] + 1 && q[a] < p.box[2 * a + 1] - 1)) {
              err = "every solid node must lie strictly inside the control volume";
              return LBM_EINVAL;
            }
        }
        for (int i = 1; i < kQ; ++i) {
          int t[3] = {x + kCx[i], y + kCy[i], z + kCz[i]};
          if (!geo.wrap(t)) continue;
          p.word[geo.index(t)] |= 1u << i;
        }
      }
  // Outlet ghost plane x = nx: a pull from a ghost node whose copy source is solid
  // bounces back.
  if (g.bc_x == LBM_BCX_INLET_OUTLET)
    for (int z = 0; z < g.nz; ++z)
      for (int y = 0; y < g.ny; ++y)
        for (int i = 1; i < kQ; ++i) {
          if (kCx[i] != -1) continue;
          int s[3] = {g.nx - 1, y - kCy[i], z - kCz[i]};
          if (!geo.wrap(s)) continue;  // a wall comes first
          if (mask[geo.index(s)]) p.word[(int64_t(z) * g.ny + y) * g.nx + g.nx - 1] |= 1u << i;
        }
  // Counts, band (fluid nodes with a neighbour across the box surface), V.
  std::vector<uint8_t> band;
  if (p.has_box) band.assign(size_t(N), 0);
  // Rows (y, z) more than one node from the box in y or z hold no node of V or of its
  // band.
  auto row_near = [&](int y, int z) {
    return p.has_box && (p.whole[1] || (y >= p.box[2] - 1 && y <= p.box[3])) &&
           (p.whole[2] || (z >= p.box[4] - 1 && z <= p.box[5]));
  };
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y) {
      const bool rnear = row_near(y, z);
      for (int x = 0; x < g.nx; ++x) {
        const int64_t k = (int64_t(z) * g.ny + y) * g.nx + x;
        if (mask[k]) continue;
        ++p.n_fluid;
        const uint32_t w = p.word[k];
        if (w)  // most nodes pull plainly in every direction
          for (int i = 1; i < kQ; ++i)
            if ((w >> i) & 1u) {
              int s[3] = {x - kCx[i], y - kCy[i], z - kCz[i]};
              if (geo.wrap(s)) ++p.n_links;
            }
        if (!rnear) continue;
        const int q[3] = {x, y, z};
        const bool in = in_box(q);
        if (in) ++p.n_box;
        bool near = true;  // cheap reject: more than one node from every surface
        for (int a = 0; a < 3 && near; ++a)
          if (!p.whole[a] && (q[a] < p.box[2 * a] - 1 || q[a] > p.box[2 * a + 1]))
            near = false;
        if (!near) continue;
        for (int i = 1; i < kQ; ++i) {
          int t[3] = {x + kCx[i], y + kCy[i], z + kCz[i]};
          if (!geo.wrap(t)) continue;
          if (in_box(t) != in) {
            band[size_t(k)] = 1;
            break;
          }
        }
      }
    }
  // Strips.
  p.ntx = (g.nx + kTileW - 1) / kTileW;
  p.ntiles = int64_t(p.ntx) * g.ny * g.nz;
  p.strip.assign(size_t(p.ntiles) * kStrips, kStripEmpty);
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int tx = 0; tx < p.ntx; ++tx)
        for (int s = 0; s < kStrips; ++s) {
          const int x0 = tx * kTileW + s * kStripW;
          if (x0 >= g.nx) continue;
          const int x1 = std::min(x0 + kStripW, g.nx);
          bool general = x0 == 0 || x1 == g.nx || y == 0 || y == g.ny - 1 || z == 0 ||
                         z == g.nz - 1;
          bool force = false, inV = false;
          const bool rnear = row_near(y, z);
          for (int x = x0; x < x1; ++x) {
            const int64_t k = (int64_t(z) * g.ny + y) * g.nx + x;
            if (p.word[k]) general = force = true;
            if (rnear && band[size_t(k)]) general = force = true;
            if (rnear && !mask[k]) {
              const int q[3] = {x, y, z};
              if (in_box(q)) inV = true;
            }
          }
          const size_t e = (size_t(int64_t(z) * g.ny + y) * p.ntx + tx) * kStrips + s;
          if (general) {
            ++p.ngeneral;
            if (force || inV) {
              p.fstrips.push_back(uint32_t(e));
              p.strip[e] = (kForce << 30) | uint32_t(p.nslots++);
            }
            else
              p.strip[e] = kEdge << 30;
          } else if (inV) {
            p.strip[e] = (kBoxJ << 30) | uint32_t(p.njslots++);
          } else {
            p.strip[e] = kPlain << 30;
          }
        }
  if (p.has_box) {
    const int bw = p.box[1] - p.box[0];
    p.box_bx = (bw + kTileW - 1) / kTileW;
    p.box_rows = (p.box[3] - p.box[2]) * (p.box[5] - p.box[4]);
  }
  return LBM_OK;
}

void plan3_links(const Plan3& p, std::vector<int64_t>& out) {
  out.clear();
  const Geo geo{{p.nx, p.ny, p.nz},
                {p.bc_x == LBM_BCX_PERIODIC, p.bc_y == LBM_BCY_PERIODIC,
                 p.bc_z == LBM_BCY_PERIODIC}};
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const int64_t k = (int64_t(z) * p.ny + y) * p.nx + x;
        const uint32_t w = p.word[size_t(k)];
        if (w & kSolid) continue;
        for (int d = 1; d < kQ; ++d) {
          const int i = opp(d);  // the pull of i comes from x + c_d
          if (!((w >> i) & 1u)) continue;
          int s[3] = {x + kCx[d], y + kCy[d], z + kCz[d]};
          if (!geo.wrap(s)) continue;  // the outlet ghost of a solid node: no link
          out.push_back(k);
          out.push_back(d);
        }
      }
}

}  // namespace lbm3
