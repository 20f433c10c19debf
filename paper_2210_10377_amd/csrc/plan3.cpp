// Host-side plan of the three-dimensional path (see plan3.h).
#include "plan3.h"

#include <algorithm>
#include <cstring>

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



Geo geo_of(const Plan3& p) {
  return Geo{{p.nx, p.ny, p.nz},
             {p.bc_x == LBM_BCX_PERIODIC, p.bc_y == LBM_BCY_PERIODIC, p.bc_z == LBM_BCY_PERIODIC}};
}

bool in_box(const Plan3& p, const int* q) {
  for (int a = 0; a < 3; ++a)
    if (!p.whole[a] && (q[a] < p.box[2 * a] || q[a] >= p.box[2 * a + 1])) return false;
  return true;
}

// Checks that need no plan: sizes, codes, mask bytes, the control volume axis by axis
// (one node inside the domain, or spanning a periodic axis whole) with every solid node
// strictly inside it.  Sets p's geometry and counts the solid nodes.
int validate3(const lbm3d_grid& g, const uint8_t* mask, Plan3& p, int64_t& nsolid,
              std::string& err) {
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
  const Geo geo = geo_of(p);
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
  // Mask bytes (eight fluid bytes skipped at a time) and the solid nodes' bounding box.
  const int64_t N = int64_t(g.nx) * g.ny * g.nz;
  int lo[3] = {g.nx, g.ny, g.nz}, hi[3] = {-1, -1, -1};
  nsolid = 0;
  for (int64_t r = 0; r < int64_t(g.ny) * g.nz; ++r) {
    const uint8_t* row = mask + r * g.nx;
    for (int x = 0; x < g.nx; ++x) {
      if (x + 8 <= g.nx) {
        uint64_t v;
        std::memcpy(&v, row + x, 8);
        if (v == 0) {
          x += 7;
          continue;
        }
      }
      if (row[x] == 0) continue;
      if (row[x] > 1) {
        err = "mask values must be 0 or 1";
        return LBM_EINVAL;
      }
      ++nsolid;
      const int q[3] = {x, int(r % g.ny), int(r / g.ny)};
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], q[a]);
        hi[a] = std::max(hi[a], q[a]);
      }
    }
  }
  (void)N;
  if (p.has_box && nsolid > 0)
    for (int a = 0; a < 3; ++a)
      if (!p.whole[a] && !(lo[a] >= p.box[2 * a] + 1 && hi[a] < p.box[2 * a + 1] - 1)) {
        err = "every solid node must lie strictly inside the control volume";
        return LBM_EINVAL;
      }
  return LBM_OK;
}

// Word of node (x, y, z) from the mask, as build_plan3 scatters it: solid bit; bit i
// when the source of the pull of direction i is a solid node, or, on the last column
// with an outlet, the outlet ghost of a solid node (a wall comes first).
uint32_t word_of(const Plan3& p, const Geo& geo, const uint8_t* mask, int x, int y, int z) {
  const int q[3] = {x, y, z};
  uint32_t w = mask[geo.index(q)] ? kSolid : 0u;  // solid nodes keep their bits too
  for (int i = 1; i < kQ; ++i) {
    int s[3] = {x - kCx[i], y - kCy[i], z - kCz[i]};
    if (geo.wrap(s)) {
      if (mask[geo.index(s)]) w |= 1u << i;
    } else if (p.bc_x == LBM_BCX_INLET_OUTLET && x == p.nx - 1 && kCx[i] == -1) {
      int t[3] = {p.nx - 1, y - kCy[i], z - kCz[i]};
      if (geo.wrap(t) && mask[geo.index(t)]) w |= 1u << i;
    }
  }
  return w;
}

// Body links of a node with word w: bounce-backs whose source is a solid node of the
// domain (not the outlet ghost).
int links_of(const Geo& geo, uint32_t w, int x, int y, int z) {
  if (!w || (w & kSolid)) return 0;
  int n = 0;
  for (int i = 1; i < kQ; ++i)
    if ((w >> i) & 1u) {
      int s[3] = {x - kCx[i], y - kCy[i], z - kCz[i]};
      if (geo.wrap(s)) ++n;
    }
  return n;
}

// A fluid node of the control-volume band: a neighbour lies across the box surface.
// Solid nodes never lie there (they sit strictly inside the box).
bool band_at(const Plan3& p, const Geo& geo, int x, int y, int z) {
  const int q[3] = {x, y, z};
  for (int a = 0; a < 3; ++a)
    if (!p.whole[a] && (q[a] < p.box[2 * a] - 1 || q[a] > p.box[2 * a + 1])) return false;
  const bool in = in_box(p, q);
  for (int i = 1; i < kQ; ++i) {
    int t[3] = {x + kCx[i], y + kCy[i], z + kCz[i]};
    if (!geo.wrap(t)) continue;
    if (in_box(p, t) != in) return true;
  }
  return false;
}

// Class of a strip (slot still unassigned): general path with or without force terms,
// streaming with the control-volume momentum, plain streaming.
uint32_t strip_class_of(const Plan3& p, const Geo& geo, const uint8_t* mask, int y, int z,
                        int x0) {
  const int x1 = std::min(x0 + kStripW, p.nx);
  bool general = x0 == 0 || x1 == p.nx || y == 0 || y == p.ny - 1 || z == 0 || z == p.nz - 1;
  bool force = false, inV = false;
  const bool rnear = p.has_box && (p.whole[1] || (y >= p.box[2] - 1 && y <= p.box[3])) &&
                     (p.whole[2] || (z >= p.box[4] - 1 && z <= p.box[5]));
  for (int x = x0; x < x1; ++x) {
    const int64_t k = (int64_t(z) * p.ny + y) * p.nx + x;
    if (p.word[size_t(k)]) general = force = true;
    if (rnear && !mask[k]) {
      if (band_at(p, geo, x, y, z)) general = force = true;
      const int q[3] = {x, y, z};
      if (in_box(p, q)) inV = true;
    }
  }
  if (general) return (force || inV) ? kForce : kEdge;
  return inV ? kBoxJ : kPlain;
}

// Slots in strip order: force strips number the force slots (and list their strips),
// box-J strips the momentum slots.
void number_slots(Plan3& p) {
  p.fstrips.clear();
  p.nslots = p.njslots = p.ngeneral = 0;
  for (size_t e = 0; e < p.strip.size(); ++e) {
    const uint32_t v = p.strip[e];
    if (v == kStripEmpty) continue;
    const uint32_t c = strip_class(v);
    if (c == kForce) {
      ++p.ngeneral;
      p.fstrips.push_back(uint32_t(e));
      p.strip[e] = (kForce << 30) | uint32_t(p.nslots++);
    } else if (c == kEdge) {
      ++p.ngeneral;
    } else if (c == kBoxJ) {
      p.strip[e] = (kBoxJ << 30) | uint32_t(p.njslots++);
    }
  }
}

void count_box(Plan3& p, const uint8_t* mask) {
  p.n_box = 0;
  p.box_bx = p.box_rows = 0;
  if (!p.has_box) return;
  const int n[3] = {p.nx, p.ny, p.nz};
  int a0[3], a1[3];
  for (int a = 0; a < 3; ++a) {
    a0[a] = p.whole[a] ? 0 : p.box[2 * a];
    a1[a] = p.whole[a] ? n[a] : p.box[2 * a + 1];
  }
  for (int z = a0[2]; z < a1[2]; ++z)
    for (int y = a0[1]; y < a1[1]; ++y)
      for (int x = a0[0]; x < a1[0]; ++x)
        p.n_box += mask[(int64_t(z) * p.ny + y) * p.nx + x] ? 0 : 1;
  const int bw = p.box[1] - p.box[0];
  p.box_bx = (bw + kTileW - 1) / kTileW;
  p.box_rows = (p.box[3] - p.box[2]) * (p.box[5] - p.box[4]);
}

}  // namespace

int build_plan3(const lbm3d_grid& g, const uint8_t* mask, Plan3& p, std::string& err) {
  int64_t nsolid = 0;
  const int rc = validate3(g, mask, p, nsolid, err);
  if (rc != LBM_OK) return rc;
  const Geo geo = geo_of(p);
  const int64_t N = int64_t(g.nx) * g.ny * g.nz;
  // Node words, scattered from every solid node to the nodes that pull from it (a source
  // inside the domain is never a wall or inlet case).
  p.word.assign(size_t(N), 0u);
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const int64_t k = (int64_t(z) * g.ny + y) * g.nx + x;
        if (!mask[k]) continue;
        p.word[k] |= kSolid;
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
  p.n_fluid = N - nsolid;
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const uint32_t w = p.word[(int64_t(z) * g.ny + y) * g.nx + x];
        if (w) p.n_links += links_of(geo, w, x, y, z);
      }
  count_box(p, mask);
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
          const size_t e = (size_t(int64_t(z) * g.ny + y) * p.ntx + tx) * kStrips + s;
          p.strip[e] = strip_class_of(p, geo, mask, y, z, x0) << 30;
        }
  number_slots(p);
  return LBM_OK;
}

int replan3(const lbm3d_grid& g, const uint8_t* mask, const std::vector<int32_t>& changed,
            Plan3& p, Plan3& np, Plan3Delta& d, std::string& err) {
  int64_t nsolid = 0;
  Plan3 q;
  const int rc = validate3(g, mask, q, nsolid, err);
  if (rc != LBM_OK) return rc;
  const Geo geo = geo_of(q);
  const int nx = g.nx, ny = g.ny;
  // Words that can change: the changed nodes, the nodes that pull from them, and on the
  // last column with an outlet the nodes whose ghost copies them.
  std::vector<int64_t> idx;
  idx.reserve(changed.size() * (kQ + 9));
  for (int32_t c : changed) {
    const int x = c % nx, y = (c / nx) % ny, z = c / (nx * ny);
    for (int i = 0; i < kQ; ++i) {
      int t[3] = {x + kCx[i], y + kCy[i], z + kCz[i]};
      if (geo.wrap(t)) idx.push_back(geo.index(t));
      if (g.bc_x == LBM_BCX_INLET_OUTLET && x == nx - 1 && kCx[i] == -1) {
        int u[3] = {nx - 1, y + kCy[i], z + kCz[i]};
        if (geo.wrap(u)) idx.push_back(geo.index(u));
      }
    }
  }
  std::sort(idx.begin(), idx.end());
  idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
  d = Plan3Delta();
  int64_t dlinks = 0;
  for (int64_t k : idx) {
    const int x = int(k % nx), y = int((k / nx) % ny), z = int(k / (int64_t(nx) * ny));
    const uint32_t w = word_of(q, geo, mask, x, y, z), o = p.word[size_t(k)];
    if (w == o) continue;
    dlinks += links_of(geo, w, x, y, z) - links_of(geo, o, x, y, z);
    d.idx.push_back(k);
    d.old_w.push_back(o);
    d.new_w.push_back(w);
  }
  // The new plan: p's words (no copy) with the delta, p's strips re-classified where a
  // word, a node's phase or the control volume changed, slots renumbered.
  apply_delta3(p, d, true);
  np = std::move(q);
  np.word.swap(p.word);
  np.n_fluid = int64_t(nx) * ny * g.nz - nsolid;
  np.n_links = p.n_links + dlinks;
  count_box(np, mask);
  np.ntx = p.ntx;
  np.ntiles = p.ntiles;
  np.strip = p.strip;
  std::vector<int64_t> st;  // strips to re-classify
  auto strip_of = [&](int x, int y, int z) {
    return (int64_t(z) * ny + y) * np.ntx * kStrips + x / kStripW;
  };
  for (int64_t k : d.idx)
    st.push_back(strip_of(int(k % nx), int((k / nx) % ny), int(k / (int64_t(nx) * ny))));
  for (int32_t c : changed) st.push_back(strip_of(c % nx, (c / nx) % ny, c / (nx * ny)));
  bool moved = false;
  for (int k = 0; k < 6; ++k) moved = moved || p.box[k] != np.box[k];
  if (np.has_box && moved) {
    // Every strip within one node of the old or the new box.
    const int n[3] = {nx, ny, g.nz};
    for (const Plan3* b : {&p, &np}) {
      int a0[3], a1[3];
      for (int a = 0; a < 3; ++a) {
        a0[a] = b->whole[a] ? 0 : std::max(b->box[2 * a] - 1, 0);
        a1[a] = b->whole[a] ? n[a] - 1 : std::min(b->box[2 * a + 1], n[a] - 1);
      }
      for (int z = a0[2]; z <= a1[2]; ++z)
        for (int y = a0[1]; y <= a1[1]; ++y)
          for (int x = a0[0] / kStripW * kStripW; x <= a1[0]; x += kStripW)
            st.push_back(strip_of(x, y, z));
    }
  }
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  for (int64_t e : st) {
    const int64_t row = e / (int64_t(np.ntx) * kStrips);
    const int x0 = int(e % (int64_t(np.ntx) * kStrips)) * kStripW;
    if (x0 >= nx) continue;
    np.strip[size_t(e)] = strip_class_of(np, geo, mask, int(row % ny), int(row / ny), x0) << 30;
  }
  number_slots(np);
  return LBM_OK;
}

void apply_delta3(Plan3& p, const Plan3Delta& d, bool forward) {
  for (size_t j = 0; j < d.idx.size(); ++j)
    p.word[size_t(d.idx[j])] = forward ? d.new_w[j] : d.old_w[j];
}

void undo_replan3(Plan3& p, Plan3& np, const Plan3Delta& d) {
  p.word.swap(np.word);
  apply_delta3(p, d, false);
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
