// The C ABI of include/lbm.h: handle life cycle, workspace layout, step scheduling,
// the force ring, state transfer and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "adjoint.h"
#include "handle.h"
#include "trace.h"
#include "kernels.h"
#include "lbm.h"
#include "plan.h"

using namespace lbm;

namespace {

#ifndef LBM_PITCH_PAD
#define LBM_PITCH_PAD 128
#endif
// The reverse sweep overlaps the recomputation of the next segment with the reverse
// launches of the current one only on grids of at most this many tiles: a launch of
// 2,048 tiles (1024 x 512) is one wave of workgroups over the chip and leaves room
// beside it, while a launch of 131,072 (8192 x 4096) fills the chip and HBM alone.
#ifndef LBM_ADJ_OVERLAP_MAX_TILES
#define LBM_ADJ_OVERLAP_MAX_TILES 16384
#endif
#ifndef LBM_PLANE_PAD_ROWS
#define LBM_PLANE_PAD_ROWS 0
#endif
#ifndef LBM_PLANE_PAD_BYTES
#define LBM_PLANE_PAD_BYTES 512
#endif

constexpr int kRow = kRingRow;
constexpr uint64_t kStateMagic = 0x4c424d5332443951ull;  // "LBMS2D9Q"

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Padded row of the device layout, and whether the row-interleaved layout keeps every
// offset within a buffer below 2^31.
int64_t padded_row(int32_t nx) { return (int64_t(nx) + 63) / 64 * 64 + LBM_PITCH_PAD; }
bool rows_fit(const lbm_grid& g) {
  return int64_t(g.ny) * kQ * padded_row(g.nx) < (int64_t(1) << 31);
}

size_t elem_bytes(int precision) {
  return precision == LBM_FP64 ? 8 : (precision == LBM_FP16DEV ? 2 : 4);
}

bool is_dev(int precision) { return precision == LBM_FP16DEV || precision == LBM_FP32DEV; }

std::string g_create_error;

struct StateHeader {
  uint64_t magic;
  int32_t nx, ny, precision, pad;
  int64_t plane;
  int32_t pitch, pad2;
  int64_t steps_done;
};

// Lattice weight (Table I) of direction i: the base of the deviation storages.
double host_weight(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

}  // namespace


extern "C" {

int lbm_create(const lbm_grid* grid, const uint8_t* solid_mask, double tau,
               const lbm_inlet* inlet, lbm_t** out) {
  g_create_error.clear();
  if (!grid || !solid_mask || !out) {
    g_create_error = "null argument";
    return LBM_EINVAL;
  }
  *out = nullptr;
  if (!std::isfinite(tau) || tau <= 0.5) {
    g_create_error = "tau must be finite and > 1/2";
    return LBM_EINVAL;
  }
  const lbm_grid& g = *grid;
  std::vector<double> uin;
  double rho_w = 1.0;
  if (g.bc_x == LBM_BCX_INLET_OUTLET) {
    if (!inlet || !inlet->ux) {
      g_create_error = "an inlet profile is required when bc_x is inlet/outlet";
      return LBM_EINVAL;
    }
    if (g.ny > 0) uin.assign(inlet->ux, inlet->ux + g.ny);
    for (double v : uin)
      if (!std::isfinite(v)) {
        g_create_error = "inlet velocity is not finite";
        return LBM_EINVAL;
      }
    rho_w = inlet->rho_w;
    if (!std::isfinite(rho_w) || rho_w <= 0.0) {
      g_create_error = "inlet wall density must be finite and > 0";
      return LBM_EINVAL;
    }
  }
  if (g.layout != LBM_LAYOUT_AUTO && g.layout != LBM_LAYOUT_ROWS &&
      g.layout != LBM_LAYOUT_PLANES) {
    g_create_error = "unknown layout";
    return LBM_EINVAL;
  }
  if (g.layout == LBM_LAYOUT_ROWS && g.nx >= 3 && g.ny >= 3 && !rows_fit(g)) {
    g_create_error = "grid too large for the row-interleaved layout (9 ny row >= 2^31)";
    return LBM_ENOMEM;
  }
  lbm_t* h = new (std::nothrow) lbm_t();
  if (!h) return LBM_ENOMEM;
  std::string perr;
  const int rc = build_plan(g, solid_mask, h->plan, perr);
  if (rc != LBM_OK) {
    g_create_error = perr;
    delete h;
    return rc;
  }
  h->g = g;
  h->mask.assign(solid_mask, solid_mask + size_t(g.nx) * size_t(g.ny));
  h->tau = tau;
  h->omega = 1.0 / tau;
  h->rho_w = rho_w;
  h->uin = uin;
  h->uin.resize(size_t(g.ny), 0.0);
  // Device layout (offsets within a buffer are 32-bit in the kernels).  Rows padded to
  // 64 elements plus LBM_PITCH_PAD.  Row-interleaved: the nine directions of a row side
  // by side ([ny][9][row]), so a tile touches few pages.  Planar ([9][ny][row]): planes
  // padded so that consecutive planes do not sit a power of two apart.
  h->esz = elem_bytes(g.precision);
  const int64_t row = padded_row(g.nx);
  if (g.layout == LBM_LAYOUT_ROWS || (g.layout == LBM_LAYOUT_AUTO && rows_fit(g))) {
    h->plane = row;
    h->pitch = int32_t(row * kQ);
    h->buf_elems = int64_t(g.ny) * row * kQ;
  } else {
    h->pitch = int32_t(row);
    const int64_t raw = row * (g.ny + LBM_PLANE_PAD_ROWS);
    const int64_t quantum = int64_t(4096 / h->esz);
    h->plane = (raw + quantum - 1) / quantum * quantum + int64_t(LBM_PLANE_PAD_BYTES / h->esz);
    h->buf_elems = h->plane * kQ;
    if (h->plane >= (int64_t(1) << 31)) {
      g_create_error = "grid too large: a direction plane must hold fewer than 2^31 elements";
      delete h;
      return LBM_ENOMEM;
    }
  }
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    h->off_buf[k] = off;
    off = align256(off + h->buf_bytes());
  }
  h->off_node = off;
  off = align256(off + h->plan.node.size() * sizeof(uint32_t));
  h->off_tiles = off;
  off = align256(off + h->plan.strip_slot.size() * sizeof(int32_t));
  h->off_uin = off;
  off = align256(off + size_t(g.ny) * sizeof(double));
  h->off_motion = off;
  off = align256(off + sizeof(BodyMotion));
  // Force partials of two steps, with room for masks that need up to twice the slots
  // of this one (plus 4096 doubles): a body moving through the grid keeps the layout.
  h->part_cap = 2 * h->part_doubles() + 4096;
  h->off_part = off;
  off = align256(off + 2 * h->part_cap * sizeof(double));
  h->njblocks = h->plan.has_box ? h->plan.box_bx * h->plan.box_rows : 0;
  h->jcap = h->njblocks;
  h->off_jpart = off;
  off = align256(off + size_t(h->jcap) * 2 * sizeof(double));
  h->off_ring = off;
  off = align256(off + size_t(g.max_record) * kRow * sizeof(double));
  h->total = off;
  *out = h;
  return LBM_OK;
}

int lbm_workspace_bytes(const lbm_t* h, size_t* bytes) {
  if (!h || !bytes) return LBM_EINVAL;
  *bytes = h->total;
  return LBM_OK;
}

int lbm_bind(lbm_t* h, void* device_workspace, size_t bytes, void* hip_stream) {
  if (!h) return LBM_EINVAL;
  if (!device_workspace) return h->fail(LBM_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(device_workspace) % 256)
    return h->fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < h->total) return h->fail(LBM_ENOMEM, "workspace smaller than lbm_workspace_bytes");
  h->ws = static_cast<char*>(device_workspace);
  h->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  e = hipMemcpyAsync(h->ws + h->off_node, h->plan.node.data(),
                     h->plan.node.size() * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload node codes");
  e = hipMemcpyAsync(h->ws + h->off_tiles, h->plan.strip_slot.data(),
                     h->plan.strip_slot.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload tiles");
  e = hipMemcpyAsync(h->ws + h->off_uin, h->uin.data(), h->uin.size() * sizeof(double),
                     hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload inlet");
  e = hipMemcpyAsync(h->ws + h->off_motion, &h->motion, sizeof(BodyMotion),
                     hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload body motion");
  for (int k = 0; k < 2; ++k) {
    e = launch_fill_rest(h->g.precision, h->buf(k), h->buf_elems, h->plane, h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "fill rest state");
  }
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "bind synchronize");
  h->bound = true;
  h->cur = 0;
  h->steps_done = 0;
  h->nrec = 0;
  h->rec_scheme.clear();
  return LBM_OK;
}

}  // extern "C"

namespace lbm {

DevTables ws_tables(const lbm_t* h) {
  DevTables t{};
  t.node = reinterpret_cast<const uint32_t*>(h->ws + h->off_node);
  t.strip_slot = reinterpret_cast<const int32_t*>(h->ws + h->off_tiles);
  t.uin = reinterpret_cast<const double*>(h->ws + h->off_uin);
  t.motion = h->motion_dev();
  t.part[0] = h->part(0);
  t.part[1] = h->part(1);
  t.jpart = reinterpret_cast<double*>(h->ws + h->off_jpart);
  return t;
}

StepArgs step_args(const lbm_t* h) { return step_args(h, ws_tables(h)); }

StepArgs step_args(const lbm_t* h, const DevTables& t) {
  const Plan& p = h->plan;
  StepArgs a{};
  a.plane = h->plane;
  a.buf_bytes = h->buf_bytes32();
  a.pitch = h->pitch;
  a.nx = p.nx;
  a.ny = p.ny;
  a.bc_x = p.bc_x;
  a.bc_y = p.bc_y;
  a.tile_rows = p.tile_rows;
  a.ntx = p.ntx;
  a.nty = p.nty;
  a.gx0 = p.gx0;
  a.gx1 = p.gx1;
  a.gy0 = p.gy0;
  a.gy1 = p.gy1;
  a.ntiles = p.ntiles;
  if (p.has_box) {
    a.bx0 = p.box[0];
    a.bx1 = p.box[1];
    a.by0 = p.box[2];
    a.by1 = p.box[3];
  } else {
    a.bx0 = 1;
    a.bx1 = 0;
    a.by0 = 1;
    a.by1 = 0;
  }
  a.node = t.node;
  a.strip_slot = t.strip_slot;
  a.uin = t.uin;
  a.rho_w6 = 6.0 * h->rho_w;
  a.motion = t.motion;
  a.omega = h->omega;
  a.collision = h->g.collision;
  a.nslots = p.nslots;
  a.njslots = p.njslots;
  return a;
}

bool row_forces(const double* r, uint32_t sch, bool has_box, double* o) {
  // DRTT: J(t) - J(t+1) + Phi(t) with J(t) before collision; DRTT-post: the same with
  // J(t) after collision (the stored populations).
  const double v[2 * kSchemes] = {r[0], r[1], r[2], r[3], r[4] - r[kJnext] + r[6],
                                  r[5] - r[kJnext + 1] + r[7], r[8], r[9],
                                  r[kJpost] - r[kJnext] + r[6], r[kJpost + 1] - r[kJnext + 1] + r[7]};
  const bool want[kSchemes] = {(sch & LBM_FORCE_MEA_A) != 0, (sch & LBM_FORCE_MEA_B) != 0,
                               (sch & LBM_FORCE_DRTT) != 0 && has_box, (sch & LBM_FORCE_SI) != 0,
                               (sch & LBM_FORCE_DRTT_POST) != 0 && has_box};
  bool finite = true;
  for (int s = 0; s < kSchemes; ++s)
    for (int c = 0; c < 2; ++c) {
      o[2 * s + c] = want[s] ? v[2 * s + c] : std::nan("");
      if (want[s] && !std::isfinite(v[2 * s + c])) finite = false;
    }
  return finite;
}

BoxArgs box_args(const lbm_t* h, const void* src) { return box_args(h, src, ws_tables(h)); }

BoxArgs box_args(const lbm_t* h, const void* src, const DevTables& t) {
  const Plan& p = h->plan;
  BoxArgs b{};
  b.src = src;
  b.plane = h->plane;
  b.buf_bytes = h->buf_bytes32();
  b.pitch = h->pitch;
  b.nx = p.nx;
  b.ny = p.ny;
  b.bx0 = p.box[0];
  b.bx1 = p.box[1];
  b.by0 = p.box[2];
  b.by1 = p.box[3];
  b.box_bx = p.box_bx;
  b.node = t.node;
  b.uin = t.uin;
  b.rho_w6 = 6.0 * h->rho_w;
  b.motion = t.motion;
  b.jpart = t.jpart;
  return b;
}

}  // namespace lbm

namespace {

// Enqueue n >= 1 steps; step k reads io(k).first and writes io(k).second.  With a
// non-null ring, the force row of step k goes to ring row k (rows are self-contained:
// the J of the following step, or of the pull after the last one, is stored with it).
template <class IO>
int enqueue_steps(lbm_t* h, const DevTables& t, hipStream_t stream, int32_t n, double* ring,
                  int64_t step0, IO&& io) {
  const Plan& p = h->plan;
  const bool forces = ring != nullptr;
  StepArgs a = step_args(h, t);
  const void* last = nullptr;
  for (int32_t k = 0; k < n; ++k) {
    const auto sd = io(k);
    a.src = sd.first;
    a.dst = sd.second;
    a.step_key = sr_step_key(step0 + k);
    last = sd.second;
    a.part_out = forces ? t.part[k & 1] : nullptr;
    a.red_in = nullptr;
    a.red_row = nullptr;
    a.red_prev_jnext = nullptr;
    if (forces && k >= 1) {
      a.red_in = t.part[(k - 1) & 1];
      a.red_row = ring + int64_t(k - 1) * kRow;
      a.red_prev_jnext = k >= 2 ? ring + int64_t(k - 2) * kRow + kJnext : nullptr;
    }
    hipError_t e = launch_step(h->g.precision, forces, a, stream);
    if (e != hipSuccess) return h->hip_fail(e, "launch step");
  }
  if (forces) {
    if (p.has_box) {
      const BoxArgs b = box_args(h, last, t);
      hipError_t e = launch_box_momentum(h->g.precision, b, h->njblocks, stream);
      if (e != hipSuccess) return h->hip_fail(e, "launch box momentum");
    }
    FinalArgs f{};
    f.red_in = t.part[(n - 1) & 1];
    f.nslots = p.nslots;
    f.njslots = p.njslots;
    f.row = ring + int64_t(n - 1) * kRow;
    f.prev_jnext = n >= 2 ? ring + int64_t(n - 2) * kRow + kJnext : nullptr;
    f.jpart = p.has_box ? t.jpart : nullptr;
    f.njblocks = h->njblocks;
    hipError_t e = launch_finalize(f, stream);
    if (e != hipSuccess) return h->hip_fail(e, "launch finalize");
  }
  return LBM_OK;
}

// n steps on the handle's own ping-pong state buffers.
int enqueue_own_steps(lbm_t* h, int32_t n, double* ring) {
  const int c0 = h->cur;
  const int rc = enqueue_steps(h, ws_tables(h), h->stream, n, ring, h->steps_done, [&](int32_t k) {
    const int s = (c0 + k) & 1;
    return std::pair<const void*, void*>(h->buf(s), h->buf(1 - s));
  });
  if (rc == LBM_OK) {
    h->cur = (c0 + n) & 1;
    h->steps_done += n;
  }
  return rc;
}

}  // namespace

namespace lbm {

int enqueue_pingpong(lbm_t* h, const DevTables& t, void* b0, void* b1, hipStream_t stream,
                     int32_t n, double* ring) {
  return enqueue_steps(h, t, stream, n, ring, 0, [&](int32_t k) {
    return (k & 1) ? std::pair<const void*, void*>(b1, b0) : std::pair<const void*, void*>(b0, b1);
  });
}

}  // namespace lbm

extern "C" {

int lbm_step(lbm_t* h, int32_t n, uint32_t force_scheme) {
  TraceRange range("lbm_step");
  if (!h) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  if (n < 0) return h->fail(LBM_EINVAL, "n must be >= 0");
  if (force_scheme & ~LBM_FORCE_ALL) return h->fail(LBM_EINVAL, "unknown force scheme bits");
  const bool forces = force_scheme != 0;
  if (forces && h->nrec + n > h->g.max_record)
    return h->fail(LBM_EOVERFLOW, "force ring would overflow; read lbm_forces first");
  if (n == 0) return LBM_OK;
  h->adj_valid = false;
  const int rc = enqueue_own_steps(h, n, forces ? h->ring() + h->nrec * kRow : nullptr);
  if (rc != LBM_OK) return rc;
  if (forces) {
    h->nrec += n;
    h->rec_scheme.insert(h->rec_scheme.end(), size_t(n), force_scheme);
  }
  return LBM_OK;
}

int lbm_forces(lbm_t* h, double* out, int64_t cap, int64_t* k_out) {
  TraceRange range("lbm_forces");
  if (!h) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  if (k_out) *k_out = h->nrec;
  if (h->nrec == 0) return LBM_OK;
  if (!out || cap < h->nrec) return h->fail(LBM_EINVAL, "output holds fewer rows than recorded");
  std::vector<double> rows(size_t(h->nrec) * kRow);
  hipError_t e = hipMemcpyAsync(rows.data(), h->ring(), rows.size() * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download force ring");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "forces synchronize");
  bool finite = true;
  for (int64_t t = 0; t < h->nrec; ++t)
    finite = row_forces(&rows[size_t(t) * kRow], h->rec_scheme[size_t(t)], h->plan.has_box,
                        out + t * 2 * kSchemes) && finite;
  h->nrec = 0;
  h->rec_scheme.clear();
  if (!finite) return h->fail(LBM_ENONFINITE, "a recorded force is not finite");
  return LBM_OK;
}

int lbm_coefficients(const lbm_t* h, const double* forces, int64_t k, double* out) {
  if (!h || (k > 0 && (!forces || !out)) || k < 0) return LBM_EINVAL;
  const double q = 0.5 * h->g.rho_ref * h->g.u_ref * h->g.u_ref * h->g.l_ref;
  for (int64_t j = 0; j < k * 2 * kSchemes; ++j) out[j] = forces[j] / q;
  return LBM_OK;
}

int lbm_destroy(lbm_t* h) {
  delete h;
  return LBM_OK;
}

int lbm_get_links(const lbm_t* h, int32_t* node_dir, int64_t cap, int64_t* n) {
  if (!h || !n) return LBM_EINVAL;
  const int64_t L = int64_t(h->plan.links.size() / 2);
  *n = L;
  const int64_t m = L < cap ? L : cap;
  if (m > 0) {
    if (!node_dir) return LBM_EINVAL;
    std::memcpy(node_dir, h->plan.links.data(), size_t(m) * 2 * sizeof(int32_t));
  }
  return LBM_OK;
}

int lbm_get_info(const lbm_t* h, lbm_info* info) {
  if (!h || !info) return LBM_EINVAL;
  info->n_fluid = h->plan.n_fluid;
  info->n_links = int64_t(h->plan.links.size() / 2);
  info->n_tiles = h->plan.ntiles;
  info->n_general = h->plan.ngeneral;
  info->n_box = h->plan.n_box;
  info->steps_done = h->steps_done;
  info->n_recorded = h->nrec;
  info->tile_w = kTileW / h->plan.tile_rows;
  info->tile_h = h->plan.tile_rows;
  info->plane_stride = h->plane;
  info->pitch = h->pitch;
  info->elem_bytes = int32_t(h->esz);
  return LBM_OK;
}

int lbm_get_populations(lbm_t* h, double* out) {
  if (!h || !out) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  const size_t bytes = h->buf_bytes();
  std::vector<unsigned char> raw(bytes);
  hipError_t e = hipMemcpyAsync(raw.data(), h->buf(h->cur), bytes, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download populations");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "populations synchronize");
  const int nx = h->g.nx, ny = h->g.ny, prec = h->g.precision;
  for (int i = 0; i < kQ; ++i) {
    const double base = is_dev(prec) ? host_weight(i) : 0.0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t k = size_t(i) * h->plane + size_t(y) * h->pitch + x;
        double v;
        if (prec == LBM_FP64) {
          std::memcpy(&v, &raw[k * 8], 8);
        } else if (prec == LBM_FP16DEV) {
          _Float16 hv;
          std::memcpy(&hv, &raw[k * 2], 2);
          v = double(hv);
        } else {
          float f;
          std::memcpy(&f, &raw[k * 4], 4);
          v = f;
        }
        out[(size_t(i) * ny + y) * nx + x] = base + v;
      }
  }
  return LBM_OK;
}

int lbm_set_populations(lbm_t* h, const double* in) {
  if (!h || !in) return LBM_EINVAL;
  h->adj_valid = false;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  const size_t bytes = h->buf_bytes();
  std::vector<unsigned char> raw(bytes, 0);
  const int nx = h->g.nx, ny = h->g.ny, prec = h->g.precision;
  for (int i = 0; i < kQ; ++i) {
    const double base = is_dev(prec) ? host_weight(i) : 0.0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t k = size_t(i) * h->plane + size_t(y) * h->pitch + x;
        const double v = in[(size_t(i) * ny + y) * nx + x] - base;
        if (prec == LBM_FP64) {
          std::memcpy(&raw[k * 8], &v, 8);
        } else if (prec == LBM_FP16DEV) {
          const _Float16 hv = _Float16(v);
          std::memcpy(&raw[k * 2], &hv, 2);
        } else {
          const float f = float(v);
          std::memcpy(&raw[k * 4], &f, 4);
        }
      }
  }
  hipError_t e = hipMemcpyAsync(h->buf(h->cur), raw.data(), bytes, hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload populations");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "populations synchronize");
  return LBM_OK;
}

int lbm_state_bytes(const lbm_t* h, size_t* bytes) {
  if (!h || !bytes) return LBM_EINVAL;
  *bytes = sizeof(StateHeader) + h->buf_bytes();
  return LBM_OK;
}

int lbm_get_state(lbm_t* h, void* blob, size_t cap) {
  if (!h || !blob) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  size_t need = 0;
  lbm_state_bytes(h, &need);
  if (cap < need) return h->fail(LBM_EINVAL, "state buffer too small");
  StateHeader hd{};
  hd.magic = kStateMagic;
  hd.nx = h->g.nx;
  hd.ny = h->g.ny;
  hd.precision = h->g.precision;
  hd.plane = h->plane;
  hd.pitch = h->pitch;
  hd.steps_done = h->steps_done;
  std::memcpy(blob, &hd, sizeof hd);
  hipError_t e = hipMemcpyAsync(static_cast<char*>(blob) + sizeof hd, h->buf(h->cur),
                                need - sizeof hd, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download state");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "state synchronize");
  return LBM_OK;
}

int lbm_set_state(lbm_t* h, const void* blob, size_t n) {
  if (!h || !blob) return LBM_EINVAL;
  h->adj_valid = false;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  size_t need = 0;
  lbm_state_bytes(h, &need);
  StateHeader hd{};
  if (n < sizeof hd) return h->fail(LBM_EINVAL, "state blob too small");
  std::memcpy(&hd, blob, sizeof hd);
  if (hd.magic != kStateMagic || hd.nx != h->g.nx || hd.ny != h->g.ny ||
      hd.precision != h->g.precision || hd.plane != h->plane || hd.pitch != h->pitch || n != need)
    return h->fail(LBM_EINVAL, "state blob does not match this handle");
  hipError_t e = hipMemcpyAsync(h->buf(h->cur), static_cast<const char*>(blob) + sizeof hd,
                                need - sizeof hd, hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload state");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "state synchronize");
  h->steps_done = hd.steps_done;
  return LBM_OK;
}

int lbm_set_inlet(lbm_t* h, const double* ux) {
  if (!h || !ux) return LBM_EINVAL;
  for (int y = 0; y < h->g.ny; ++y)
    if (!std::isfinite(ux[y])) return h->fail(LBM_EINVAL, "inlet velocity is not finite");
  h->uin.assign(ux, ux + h->g.ny);
  h->adj_valid = false;
  if (h->bound) {
    hipError_t e = hipMemcpyAsync(h->ws + h->off_uin, h->uin.data(), h->uin.size() * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "upload inlet");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "inlet synchronize");
  }
  return LBM_OK;
}

int lbm_set_tau(lbm_t* h, double tau) {
  if (!h) return LBM_EINVAL;
  if (!std::isfinite(tau) || tau <= 0.5) return h->fail(LBM_EINVAL, "tau must be finite and > 1/2");
  h->tau = tau;
  h->omega = 1.0 / tau;
  h->adj_valid = false;
  return LBM_OK;
}

int lbm_set_body_motion(lbm_t* h, double ux, double uy, double omega, double xc, double yc) {
  if (!h) return LBM_EINVAL;
  for (double v : {ux, uy, omega, xc, yc})
    if (!std::isfinite(v)) return h->fail(LBM_EINVAL, "body motion must be finite");
  h->motion = BodyMotion{ux, uy, omega, xc, yc,
                         (ux != 0.0 || uy != 0.0 || omega != 0.0) ? 1 : 0};
  h->adj_valid = false;
  if (h->bound) {
    hipError_t e = hipMemcpyAsync(h->ws + h->off_motion, &h->motion, sizeof(BodyMotion),
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "upload body motion");
  }
  return LBM_OK;
}

int lbm_set_mask(lbm_t* h, const uint8_t* solid_mask, const int32_t* box, double* impulse) {
  TraceRange range("lbm_set_mask");
  if (!h || !solid_mask) return LBM_EINVAL;
  lbm_grid g = h->g;
  if (box) {
    if ((box[0] >= 0) != (g.box[0] >= 0))
      return h->fail(LBM_EINVAL, "a control volume can be moved, not added or removed");
    for (int k = 0; k < 4; ++k) g.box[k] = box[k];
  }
  // Nodes that swap between fluid and solid (bit 31 of a list entry: uncovered), and
  // the nodes fluid in both masks (read by the refill).
  // Compared with the mask of the plan eight bytes at a time (bytes other than 0/1 are
  // refused by replan before anything changes).
  const int nx = g.nx, ny = g.ny;
  const size_t n = size_t(nx) * ny;
  std::vector<int32_t> changed, list;
  const uint8_t* old = h->mask.data();
  size_t k = 0;
  for (; k + 8 <= n; k += 8) {
    uint64_t a, b;
    std::memcpy(&a, old + k, 8);
    std::memcpy(&b, solid_mask + k, 8);
    if (a == b) continue;
    for (size_t j = k; j < k + 8; ++j)
      if ((old[j] != 0) != (solid_mask[j] != 0)) changed.push_back(int32_t(j));
  }
  for (; k < n; ++k)
    if ((old[k] != 0) != (solid_mask[k] != 0)) changed.push_back(int32_t(k));
  list.reserve(changed.size());
  for (int32_t c : changed) list.push_back(int32_t(uint32_t(c) | (old[c] ? 0x80000000u : 0u)));
  std::vector<uint8_t> valid(h->bound && !list.empty() ? n : 0);
  for (size_t j = 0; j < valid.size(); ++j) valid[j] = (old[j] | solid_mask[j]) == 0;
  // Scratch in the other state buffer, which the next step overwrites anyway.
  const int blocks = int(std::min<size_t>((list.size() + 255) / 256, 1024));
  const size_t off_list = align256(n), off_blk = align256(off_list + list.size() * 4),
               off_res = align256(off_blk + size_t(std::max(blocks, 1)) * 16);
  if (h->bound && off_res + 16 > h->buf_bytes())
    return h->fail(LBM_ENOMEM, "too many nodes change at once");
  // Re-classify only around the changed nodes; the new plan takes the old node words.
  Plan np;
  PlanDelta d;
  std::string perr;
  const int rc = replan(g, solid_mask, changed, h->plan, np, d, perr);
  if (rc != LBM_OK) return h->fail(rc, perr);
  const int nj = np.has_box ? np.box_bx * np.box_rows : 0;
  if (size_t(np.nslots) * kPart + size_t(np.njslots) * kBoxPart > h->part_cap || nj > h->jcap) {
    undo_replan(h->plan, np, d);
    return h->fail(LBM_ENOMEM, nj > h->jcap
                                   ? "the new control volume is larger than the one at create"
                                   : "the new mask needs more force-partial slots than "
                                     "reserved at create; create a handle for it");
  }
  auto commit = [&]() {
    h->plan = std::move(np);
    std::memcpy(h->mask.data(), solid_mask, n);
    h->g = g;
    h->njblocks = nj;
    h->adj_valid = false;
    h->adj_codes.clear();  // the adjoint codes invert the pull codes of the old mask
    ++h->plan_gen;         // tables built from the plan elsewhere (a batch) are stale
  };
  double P[2] = {0.0, 0.0};
  if (h->bound) {
    // Nothing in flight (on any stream, a batch holding the handle included) may still
    // read the old node codes or the state.
    hipError_t e = hipDeviceSynchronize();
    char* scr = static_cast<char*>(h->buf(1 - h->cur));
    if (e == hipSuccess && !list.empty()) {
      e = hipMemcpyAsync(scr, valid.data(), n, hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(scr + off_list, list.data(), list.size() * 4, hipMemcpyHostToDevice,
                           h->stream);
      RemaskArgs a{};
      a.state = h->buf(h->cur);
      a.plane = h->plane;
      a.pitch = h->pitch;
      a.nx = nx;
      a.ny = ny;
      a.bc_x = g.bc_x;
      a.bc_y = g.bc_y;
      a.list = reinterpret_cast<const int32_t*>(scr + off_list);
      a.n = int32_t(list.size());
      a.valid = reinterpret_cast<const uint8_t*>(scr);
      a.rho_w = h->rho_w;
      a.motion = h->motion;
      a.block_out = reinterpret_cast<double*>(scr + off_blk);
      double* res = reinterpret_cast<double*>(scr + off_res);
      if (e == hipSuccess) e = launch_remask(g.precision, a, blocks, res, h->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(P, res, sizeof(P), hipMemcpyDeviceToHost, h->stream);
    }
    // Upload the rewritten node words (one contiguous index range) and the strip slots.
    if (e == hipSuccess && !d.idx.empty()) {
      const size_t lo = size_t(d.idx.front()), cnt = size_t(d.idx.back()) - lo + 1;
      e = hipMemcpyAsync(h->ws + h->off_node + lo * sizeof(uint32_t), np.node.data() + lo,
                         cnt * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->ws + h->off_tiles, np.strip_slot.data(),
                         np.strip_slot.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                         h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      commit();  // the state is undefined; the plan is the new mask's
      return h->hip_fail(e, "mask change");
    }
  }
  commit();
  if (impulse) {
    impulse[0] = P[0];
    impulse[1] = P[1];
  }
  return LBM_OK;
}

int lbm_boundary_cp(lbm_t* h, int32_t x_inf, int32_t y_inf, double* cp, int32_t* nodes,
                    int64_t cap, int64_t* n) {
  TraceRange range("lbm_boundary_cp");
  if (!h || !n) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  const int nx = h->g.nx, ny = h->g.ny;
  int32_t ref = -1;
  if (x_inf >= 0) {
    if (x_inf >= nx || y_inf < 0 || y_inf >= ny || h->mask[size_t(y_inf) * nx + x_inf])
      return h->fail(LBM_EINVAL, "the reference node must be a fluid node of the grid");
    ref = y_inf * nx + x_inf;
  }
  if (!std::isfinite(h->g.rho_ref) || !std::isfinite(h->g.u_ref) || h->g.rho_ref * h->g.u_ref == 0.0)
    return h->fail(LBM_EINVAL, "rho_ref and u_ref must be finite and non-zero");
  // The boundary fluid nodes: the distinct nodes of the canonical link list (sorted by
  // node, so row-major).
  std::vector<int32_t> list;
  const std::vector<int32_t>& L = h->plan.links;
  for (size_t k = 0; k < L.size(); k += 2)
    if (list.empty() || list.back() != L[k]) list.push_back(L[k]);
  *n = int64_t(list.size());
  if (list.empty()) return LBM_OK;
  if (!cp || cap < *n) return h->fail(LBM_EINVAL, "output holds fewer values than boundary nodes");
  if (nodes) std::memcpy(nodes, list.data(), list.size() * sizeof(int32_t));
  // Scratch in the idle state buffer, which the next step overwrites anyway.
  const size_t off_out = align256(list.size() * sizeof(int32_t));
  if (off_out + list.size() * sizeof(double) > h->buf_bytes())
    return h->fail(LBM_ENOMEM, "boundary node list larger than the scratch buffer");
  char* scr = static_cast<char*>(h->buf(1 - h->cur));
  hipError_t e = hipMemcpyAsync(scr, list.data(), list.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, h->stream);
  CpArgs a{};
  a.state = h->buf(h->cur);
  a.plane = h->plane;
  a.pitch = h->pitch;
  a.nx = nx;
  a.nodes = reinterpret_cast<const int32_t*>(scr);
  a.n = int32_t(list.size());
  a.ref_node = ref;
  a.p_ref = h->g.rho_ref * (1.0 / 3.0);
  a.q = 0.5 * h->g.rho_ref * h->g.u_ref * h->g.u_ref;
  a.out = reinterpret_cast<double*>(scr + off_out);
  if (e == hipSuccess) e = launch_boundary_cp(h->g.precision, a, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cp, a.out, list.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "boundary pressure coefficient");
  return LBM_OK;
}

int lbm_reset(lbm_t* h) {
  if (!h) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  for (int k = 0; k < 2; ++k) {
    hipError_t e = launch_fill_rest(h->g.precision, h->buf(k), h->buf_elems, h->plane, h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "fill rest state");
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "reset synchronize");
  h->cur = 0;
  h->steps_done = 0;
  h->nrec = 0;
  h->rec_scheme.clear();
  h->adj_valid = false;
  return LBM_OK;
}

}  // extern "C"

namespace {

struct AdjLayout {
  size_t state = 0, mu = 0;  // bytes of one state / adjoint buffer
  int32_t ncp = 0;           // checkpoints
  int32_t nstore = 1;        // segment stores (two when there are two segments or more)
  size_t off_cp = 0, off_seg = 0, off_mu = 0, off_adj = 0, off_dom = 0, off_duin = 0,
         off_ring = 0, total = 0;
};

// The second stream and the events of the reverse sweep, created at first use on the
// device that holds the handle's workspace.
int ensure_aux(lbm_t* h) {
  if (h->aux) return LBM_OK;
  hipPointerAttribute_t attr{};
  hipError_t e = hipPointerGetAttributes(&attr, h->ws);
  if (e != hipSuccess) return h->hip_fail(e, "workspace device");
  int prev = 0;
  if ((e = hipGetDevice(&prev)) != hipSuccess) return h->hip_fail(e, "current device");
  if (attr.device != prev && (e = hipSetDevice(attr.device)) != hipSuccess)
    return h->hip_fail(e, "select workspace device");
  e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
  hipEvent_t* evs[] = {&h->ev_go, &h->ev_rec[0], &h->ev_rec[1], &h->ev_adj[0], &h->ev_adj[1]};
  for (hipEvent_t* ev : evs)
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  const hipError_t e2 = attr.device != prev ? hipSetDevice(prev) : hipSuccess;
  if (e != hipSuccess || e2 != hipSuccess) {
    h->release_aux();
    return h->hip_fail(e != hipSuccess ? e : e2, "create the recomputation stream");
  }
  return LBM_OK;
}

AdjLayout adj_layout(const lbm_t* h, int32_t n, int32_t every) {
  AdjLayout L;
  const size_t cbytes = h->g.precision == LBM_FP64 ? 8 : 4;
  L.state = h->buf_bytes();
  L.mu = size_t(h->buf_elems) * cbytes;
  L.ncp = (n + every - 1) / every;
  size_t off = 0;
  L.off_cp = off;
  off = align256(off + size_t(L.ncp) * align256(L.state));
  L.nstore = L.ncp >= 2 && h->plan.ntiles <= LBM_ADJ_OVERLAP_MAX_TILES ? 2 : 1;
  L.off_seg = off;
  off = align256(off + size_t(L.nstore) * size_t(every - 1) * align256(L.state));
  L.off_mu = off;
  off = align256(off + 2 * align256(L.mu));
  L.off_adj = off;
  off = align256(off + size_t(h->g.nx) * h->g.ny * sizeof(uint32_t));
  L.off_dom = off;
  off = align256(off + size_t(h->plan.ntiles) * kStrips * sizeof(double));
  L.off_duin = off;
  off = align256(off + size_t(h->g.ny) * sizeof(double));
  L.off_ring = off;
  off = align256(off + size_t(n) * kRow * sizeof(double));
  L.total = off;
  return L;
}

uint32_t bytes32(size_t b) { return b < (uint64_t(1) << 32) - 4096 ? uint32_t(b) : 0u; }

}  // namespace

extern "C" {

int lbm_adjoint_bytes(const lbm_t* h, int32_t n_steps, int32_t every, size_t* bytes) {
  if (!h || !bytes || n_steps < 1 || every < 1 || every > n_steps) return LBM_EINVAL;
  *bytes = adj_layout(h, n_steps, every).total;
  return LBM_OK;
}

int lbm_adjoint_forward(lbm_t* h, void* ws, size_t bytes, int32_t n_steps, int32_t every,
                        int32_t t0, int32_t T, double wx, double wy, double* J) {
  TraceRange range("lbm_adjoint_forward");
  if (!h) return LBM_EINVAL;
  if (h->g.precision == LBM_FP16DEV)
    return h->fail(LBM_EINVAL, "the adjoint covers the 32-bit and FP64 storages");
  if (h->g.collision != LBM_COLL_BGK)
    return h->fail(LBM_EINVAL, "the adjoint covers the BGK collision only");
  if (h->motion.moving) return h->fail(LBM_EINVAL, "the adjoint covers bodies at rest only");
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  if (!ws || !J || n_steps < 1 || every < 1 || every > n_steps || t0 < 0 || T < 1 ||
      int64_t(t0) + T > n_steps || !std::isfinite(wx) || !std::isfinite(wy))
    return h->fail(LBM_EINVAL, "invalid adjoint run parameters");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return h->fail(LBM_EINVAL, "adjoint workspace must be 256-byte aligned");
  const AdjLayout L = adj_layout(h, n_steps, every);
  if (bytes < L.total) return h->fail(LBM_ENOMEM, "adjoint workspace smaller than lbm_adjoint_bytes");
  h->adj_valid = false;
  char* aws = static_cast<char*>(ws);
  if (h->adj_codes.empty()) build_adjoint_codes(h->plan, h->adj_codes);
  hipError_t e = hipMemcpyAsync(aws + L.off_adj, h->adj_codes.data(),
                                h->adj_codes.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload adjoint codes");
  double* ring = reinterpret_cast<double*>(aws + L.off_ring);
  // Step s of the run is the handle's step adj_base + s: the recomputation replays it
  // with the same number (the stochastically rounded storage draws from it).
  h->adj_base = h->steps_done;
  for (int32_t c = 0; c < L.ncp; ++c) {
    const int32_t s0 = c * every;
    const int32_t len = std::min(every, n_steps - s0);
    e = hipMemcpyAsync(aws + L.off_cp + size_t(c) * align256(L.state), h->buf(h->cur), L.state,
                       hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "store checkpoint");
    // Force sums only where the objective reads them (steps t0 .. t0 + T - 1): the
    // populations do not depend on them.
    const int32_t w0 = std::clamp(t0 - s0, 0, len), w1 = std::clamp(t0 + T - s0, 0, len);
    int rc = w0 > 0 ? enqueue_own_steps(h, w0, nullptr) : LBM_OK;
    if (rc == LBM_OK && w1 > w0)
      rc = enqueue_own_steps(h, w1 - w0, ring + int64_t(s0 + w0) * kRow);
    if (rc == LBM_OK && len > w1) rc = enqueue_own_steps(h, len - w1, nullptr);
    if (rc != LBM_OK) return rc;
  }
  std::vector<double> rows(size_t(T) * kRow);
  e = hipMemcpyAsync(rows.data(), ring + int64_t(t0) * kRow, rows.size() * sizeof(double),
                     hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download forces");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "adjoint forward synchronize");
  double acc = 0.0;
  for (int32_t t = 0; t < T; ++t) acc += wx * rows[size_t(t) * kRow + 2] + wy * rows[size_t(t) * kRow + 3];
  *J = acc / T;
  h->aws = aws;
  h->aws_bytes = bytes;
  h->adj_n = n_steps;
  h->adj_every = every;
  h->adj_t0 = t0;
  h->adj_T = T;
  h->adj_wx = wx;
  h->adj_wy = wy;
  h->adj_valid = true;
  if (!std::isfinite(*J)) return h->fail(LBM_ENONFINITE, "objective is not finite");
  return LBM_OK;
}

int lbm_adjoint_backward(lbm_t* h, double dJ, double* grad_uin, double* grad_tau) {
  TraceRange range("lbm_adjoint_backward");
  if (!h) return LBM_EINVAL;
  if (h->g.precision == LBM_FP16DEV)
    return h->fail(LBM_EINVAL, "the adjoint covers the 32-bit and FP64 storages");
  if (h->g.collision != LBM_COLL_BGK)
    return h->fail(LBM_EINVAL, "the adjoint covers the BGK collision only");
  if (h->motion.moving) return h->fail(LBM_EINVAL, "the adjoint covers bodies at rest only");
  if (!h->adj_valid)
    return h->fail(LBM_ESTATE, "no adjoint forward run matches the handle's current parameters");
  if (!grad_uin || !grad_tau || !std::isfinite(dJ)) return h->fail(LBM_EINVAL, "invalid arguments");
  const AdjLayout L = adj_layout(h, h->adj_n, h->adj_every);
  char* aws = h->aws;
  const Plan& p = h->plan;
  const size_t cbytes = h->g.precision == LBM_FP64 ? 8 : 4;
  void* mu[2] = {aws + L.off_mu, aws + L.off_mu + align256(L.mu)};
  double* dom = reinterpret_cast<double*>(aws + L.off_dom);
  double* duin = reinterpret_cast<double*>(aws + L.off_duin);
  hipError_t e = hipSuccess;
  // Both adjoint fields start at zero: mu(n) = 0, and no entry of a solid node is ever
  // written, so neither buffer keeps values of an earlier run or geometry.
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = cbytes == 8 ? launch_zero_f64(static_cast<double*>(mu[k]), int64_t(L.mu / 8), h->stream)
                    : launch_zero_f32(static_cast<float*>(mu[k]), int64_t(L.mu / 4), h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "zero adjoint");
  if ((e = launch_zero_f64(dom, int64_t(p.ntiles) * kStrips, h->stream)) != hipSuccess)
    return h->hip_fail(e, "zero adjoint sums");
  if ((e = launch_zero_f64(duin, p.ny, h->stream)) != hipSuccess)
    return h->hip_fail(e, "zero adjoint sums");
  AdjArgs a{};
  a.plane = h->plane;
  a.state_bytes = bytes32(L.state);
  a.mu_bytes = bytes32(L.mu);
  a.pitch = h->pitch;
  a.nx = p.nx;
  a.ny = p.ny;
  a.ntx = p.ntx;
  a.tile_rows = p.tile_rows;
  a.ntiles = p.ntiles;
  a.gx0 = p.gx0;
  a.gx1 = p.gx1;
  a.gy0 = p.gy0;
  a.gy1 = p.gy1;
  a.node = reinterpret_cast<const uint32_t*>(h->ws + h->off_node);
  a.adj = reinterpret_cast<const uint32_t*>(aws + L.off_adj);
  a.uin = reinterpret_cast<const double*>(h->ws + h->off_uin);
  a.rho_w6 = 6.0 * h->rho_w;
  a.omega = h->omega;
  a.domega = dom;
  a.duin = duin;
  const int32_t every = h->adj_every;
  auto seg_len = [&](int32_t c) { return std::min(every, h->adj_n - c * every); };
  // seg(c, j) = S(c * every - 1 + j): the checkpoint of segment c, then its recomputed
  // states, in segment store c % nstore.
  auto seg = [&](int32_t c, int32_t j) -> void* {
    return j == 0 ? static_cast<void*>(aws + L.off_cp + size_t(c) * align256(L.state))
                  : static_cast<void*>(aws + L.off_seg +
                                       (size_t(c % L.nstore) * (every - 1) + size_t(j - 1)) *
                                           align256(L.state));
  };
  auto recompute = [&](int32_t c, hipStream_t s) -> int {
    const int32_t len = seg_len(c);
    if (len <= 1) return LBM_OK;
    // Recomputed step k of segment c is step c * every + k of the forward run.
    return enqueue_steps(h, ws_tables(h), s, len - 1, nullptr, h->adj_base + int64_t(c) * every,
                         [&](int32_t k) {
      return std::pair<const void*, void*>(seg(c, k), seg(c, k + 1));
    });
  };
  // With two segment stores (small grids, LBM_ADJ_OVERLAP_MAX_TILES) the recomputation
  // of segment c - 1 (second stream) runs while the reverse launches of segment c (the
  // handle's stream) read the other store: neither kernel fills the GPU alone there.
  // Events order each recomputation after the reverse sweep that last read its store,
  // and each sweep after its recomputation.
  const bool overlap = L.nstore == 2;
  if (overlap) {
    int rc = ensure_aux(h);
    if (rc != LBM_OK) return rc;
    if ((e = hipEventRecord(h->ev_go, h->stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(h->aux, h->ev_go, 0)) != hipSuccess)
      return h->hip_fail(e, "order the recomputation stream");
    if ((rc = recompute(L.ncp - 1, h->aux)) != LBM_OK) return rc;
    if ((e = hipEventRecord(h->ev_rec[(L.ncp - 1) & 1], h->aux)) != hipSuccess)
      return h->hip_fail(e, "record recomputation");
  }
  int cur = 0;  // mu[cur] holds mu(t+1)
  for (int32_t c = L.ncp - 1; c >= 0; --c) {
    const int32_t t_first = c * every;
    const int32_t len = seg_len(c);
    if (overlap) {
      if (c >= 1) {
        if (c + 1 < L.ncp && (e = hipStreamWaitEvent(h->aux, h->ev_adj[(c + 1) & 1], 0)) != hipSuccess)
          return h->hip_fail(e, "order the recomputation stream");
        const int rc = recompute(c - 1, h->aux);
        if (rc != LBM_OK) return rc;
        if ((e = hipEventRecord(h->ev_rec[(c - 1) & 1], h->aux)) != hipSuccess)
          return h->hip_fail(e, "record recomputation");
      }
      if ((e = hipStreamWaitEvent(h->stream, h->ev_rec[c & 1], 0)) != hipSuccess)
        return h->hip_fail(e, "wait for recomputation");
    } else {
      const int rc = recompute(c, h->stream);
      if (rc != LBM_OK) return rc;
    }
    for (int32_t t = t_first + len - 1; t >= t_first; --t) {
      const bool in_window = t >= h->adj_t0 && t < h->adj_t0 + h->adj_T;
      const double g = in_window ? dJ * 2.0 / h->adj_T : 0.0;
      a.gx = g * h->adj_wx;
      a.gy = g * h->adj_wy;
      a.state = seg(c, t - t_first);
      a.mu_in = mu[cur];
      a.mu_out = mu[1 - cur];
      e = launch_adjoint(h->g.precision, a, h->stream);
      if (e != hipSuccess) return h->hip_fail(e, "launch adjoint");
      cur = 1 - cur;
    }
    if (overlap && (e = hipEventRecord(h->ev_adj[c & 1], h->stream)) != hipSuccess)
      return h->hip_fail(e, "record reverse sweep");
  }
  std::vector<double> hdom(size_t(p.ntiles) * kStrips);
  e = hipMemcpyAsync(hdom.data(), dom, hdom.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download adjoint sums");
  e = hipMemcpyAsync(grad_uin, duin, size_t(p.ny) * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download adjoint sums");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "adjoint synchronize");
  double domega = 0.0;
  for (double v : hdom) domega += v;
  // omega = 1 / tau
  *grad_tau = -domega / (h->tau * h->tau);
  bool finite = std::isfinite(*grad_tau);
  for (int y = 0; y < p.ny; ++y) finite = finite && std::isfinite(grad_uin[y]);
  if (!finite) return h->fail(LBM_ENONFINITE, "gradient is not finite");
  return LBM_OK;
}

const char* lbm_last_error(const lbm_t* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
