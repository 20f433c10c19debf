// C ABI of the three-dimensional (D3Q27) path (include/lbm3d.h): planning, device
// layout, stepping with per-step forces, readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "kernels3.h"
#include "lbm3d.h"
#include "plan3.h"
#include "trace.h"

using namespace lbm3;

struct lbm3d {
  lbm3d_grid g;
  double tau = 0.0, rho_w = 1.0;
  double mu[3] = {0.0, 0.0, 0.0}, mw[3] = {0.0, 0.0, 0.0}, mc[3] = {0.0, 0.0, 0.0};
  bool moving = false;
  std::vector<double> uin;  // [nz][ny]
  Plan3 plan;
  std::vector<uint8_t> mask;  // the body mask of the plan ([nz][ny][nx], 0/1)
  // Population i of node (x, y, z) at i * dstride + (z * ny + y) * rstride + x.
  int32_t rstride = 0;
  int64_t dstride = 0;
  int64_t buf_elems = 0;  // elements of one state buffer
  size_t esz = 0;
  size_t off_buf[2] = {0, 0}, off_word = 0, off_strip = 0, off_fstrip = 0, off_uin = 0, off_part = 0,
         off_jpart = 0, off_ring = 0, total = 0;
  int njblocks = 0;
  // Reserved at create so that a mask change can re-plan in place: force slots (strip
  // indices), doubles of one force-partial buffer, control-volume sweep blocks.
  size_t fcap = 0, part_cap = 0;
  int jcap = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int cur = 0;
  int64_t steps_done = 0, nrec = 0;
  std::vector<uint32_t> rec_scheme;
  std::string err;

  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EHIP;
  }
  void* buf(int k) const { return ws + off_buf[k]; }
  size_t buf_bytes() const { return size_t(buf_elems) * esz; }
  size_t part_doubles() const {
    return size_t(plan.nslots) * kPart + size_t(plan.njslots) * 3;
  }
  double* part(int k) const {
    return reinterpret_cast<double*>(ws + off_part) + size_t(k) * part_cap;
  }
  double* ring() const { return reinterpret_cast<double*>(ws + off_ring); }
};

namespace {

std::string g_err3;

constexpr uint64_t kState3Magic = 0x4c424d5333443237ull;  // "LBMS3D27"

// Header of a checkpoint blob; the raw state buffer follows.
struct State3Header {
  uint64_t magic;
  int32_t nx, ny, nz, precision;
  int64_t dstride;
  int32_t rstride, pad;
  int64_t steps_done;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }
size_t elem_bytes(int p) { return p == LBM_FP64 ? 8 : (p == LBM_FP16DEV ? 2 : 4); }
bool is_dev(int p) { return p == LBM_FP16DEV || p == LBM_FP32DEV; }
double host_w27(int i) {
  double w = 1.0;
  w *= kCx[i] == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
  w *= kCy[i] == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
  w *= kCz[i] == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
  return w;
}

// Padded row of the row-interleaved layout, and whether that layout fits 32-bit offsets.
int64_t rows_row(int32_t nx) {
  const int64_t row64 = (int64_t(nx) + 63) / 64 * 64;
  return row64 + (row64 % 1024 == 0 ? 64 : 0);
}
bool rows_fit(const lbm3d_grid& g) {
  return int64_t(g.ny) * g.nz * kQ * rows_row(g.nx) < (int64_t(1) << 31);
}

Geom3 geom(const lbm3d* h) {
  const Plan3& p = h->plan;
  Geom3 g{};
  g.dstride = h->dstride;
  g.rstride = h->rstride;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.bc_x = p.bc_x;
  g.bc_y = p.bc_y;
  g.bc_z = p.bc_z;
  for (int k = 0; k < 6; ++k) g.box[k] = p.box[k];
  for (int a = 0; a < 3; ++a) g.whole[a] = p.whole[a] ? 1 : 0;
  g.has_box = p.has_box ? 1 : 0;
  g.word = reinterpret_cast<const uint32_t*>(h->ws + h->off_word);
  g.uin = reinterpret_cast<const double*>(h->ws + h->off_uin);
  g.rho_w6 = 6.0 * h->rho_w;
  for (int k = 0; k < 3; ++k) {
    g.mu[k] = h->mu[k];
    g.mw[k] = h->mw[k];
    g.mc[k] = h->mc[k];
  }
  g.moving = h->moving ? 1 : 0;
  return g;
}

// Enqueue n >= 1 steps on the ping-pong buffers; with a ring, step k's row is ring row k.
int enqueue3(lbm3d* h, int32_t n, double* ring) {
  const Plan3& p = h->plan;
  const bool forces = ring != nullptr;
  Step3Args a{};
  a.g = geom(h);
  a.ntx = p.ntx;
  a.ntiles = p.ntiles;
  a.strip = reinterpret_cast<const uint32_t*>(h->ws + h->off_strip);
  a.fstrips = reinterpret_cast<const uint32_t*>(h->ws + h->off_fstrip);
  a.omega = 1.0 / h->tau;
  a.collision = h->g.collision;
  a.nslots = p.nslots;
  a.njslots = p.njslots;
  const int c0 = h->cur;
  for (int32_t k = 0; k < n; ++k) {
    const int s = (c0 + k) & 1;
    a.src = h->buf(s);
    a.dst = h->buf(1 - s);
    a.step_key = lbm::sr_step_key(h->steps_done + k);
    a.part_out = forces ? h->part(k & 1) : nullptr;
    a.red_in = nullptr;
    a.red_row = nullptr;
    a.red_prev_jnext = nullptr;
    if (forces && k >= 1) {
      a.red_in = h->part((k - 1) & 1);
      a.red_row = ring + int64_t(k - 1) * kRow;
      a.red_prev_jnext = k >= 2 ? ring + int64_t(k - 2) * kRow + kPart : nullptr;
    }
    hipError_t e = launch_step3(h->g.precision, forces, a, h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "launch step");
  }
  const void* last = h->buf((c0 + n) & 1);
  if (forces) {
    if (p.has_box) {
      Box3Args b{};
      b.g = geom(h);
      b.src = last;
      b.jpart = reinterpret_cast<double*>(h->ws + h->off_jpart);
      hipError_t e = launch_box3(h->g.precision, b, h->njblocks, h->stream);
      if (e != hipSuccess) return h->hip_fail(e, "launch box momentum");
    }
    Final3Args f{};
    f.red_in = h->part((n - 1) & 1);
    f.nslots = p.nslots;
    f.njslots = p.njslots;
    f.row = ring + int64_t(n - 1) * kRow;
    f.prev_jnext = n >= 2 ? ring + int64_t(n - 2) * kRow + kPart : nullptr;
    f.jpart = p.has_box ? reinterpret_cast<const double*>(h->ws + h->off_jpart) : nullptr;
    f.njblocks = h->njblocks;
    hipError_t e = launch_final3(f, h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "launch finalize");
  }
  h->cur = (c0 + n) & 1;
  h->steps_done += n;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm3d_create(const lbm3d_grid* grid, const uint8_t* mask, double tau, const double* uin,
                 double rho_w, lbm3d_t** out) {
  g_err3.clear();
  if (!grid || !mask || !out) {
    g_err3 = "null argument";
    return LBM_EINVAL;
  }
  *out = nullptr;
  const lbm3d_grid& g = *grid;
  if (!std::isfinite(tau) || tau <= 0.5) {
    g_err3 = "tau must be finite and > 1/2";
    return LBM_EINVAL;
  }
  if (g.precision != LBM_FP64 && g.precision != LBM_FP32 && g.precision != LBM_FP32DEV &&
      g.precision != LBM_FP16DEV && g.precision != LBM_FP32SR) {
    g_err3 = "unknown precision";
    return LBM_EINVAL;
  }
  if (g.max_record < 1) {
    g_err3 = "max_record must be >= 1";
    return LBM_EINVAL;
  }
  if (g.collision != LBM_COLL_BGK && g.collision != LBM_COLL_REGULARIZED) {
    g_err3 = "unknown collision (BGK or regularized)";
    return LBM_EINVAL;
  }
  if (g.layout != LBM_LAYOUT_AUTO && g.layout != LBM_LAYOUT_ROWS &&
      g.layout != LBM_LAYOUT_PLANES) {
    g_err3 = "unknown layout";
    return LBM_EINVAL;
  }
  if (g.layout == LBM_LAYOUT_ROWS && g.nx >= 2 && g.ny >= 2 && g.nz >= 2 && !rows_fit(g)) {
    g_err3 = "grid too large for the row-interleaved layout (27 ny nz row >= 2^31)";
    return LBM_ENOMEM;
  }
  lbm3d* h = new (std::nothrow) lbm3d();
  if (!h) return LBM_ENOMEM;
  std::string perr;
  const int rc = build_plan3(g, mask, h->plan, perr);
  if (rc != LBM_OK) {
    g_err3 = perr;
    delete h;
    return rc;
  }
  h->g = g;
  h->mask.assign(mask, mask + size_t(g.nx) * g.ny * g.nz);
  h->tau = tau;
  h->uin.assign(size_t(g.ny) * g.nz, 0.0);
  if (g.bc_x == LBM_BCX_INLET_OUTLET) {
    if (!uin || !std::isfinite(rho_w) || rho_w <= 0.0) {
      g_err3 = "an inlet plane and a wall density > 0 are required when bc_x is inlet/outlet";
      delete h;
      return LBM_EINVAL;
    }
    for (size_t k = 0; k < h->uin.size(); ++k) {
      if (!std::isfinite(uin[k])) {
        g_err3 = "inlet velocity is not finite";
        delete h;
        return LBM_EINVAL;
      }
      h->uin[k] = uin[k];
    }
    h->rho_w = rho_w;
  }
  // Layout.  Offsets within a buffer are 32-bit in the kernels.  Row-interleaved
  // ([nz][ny][27][row]: the 27 directions of a row side by side, so a tile touches few
  // pages), rows padded to 64 elements, plus 64 when the padded row is a multiple of
  // 1024 (the directions of a row then do not sit a power of two apart).  Planar
  // ([27][nz][ny][row]), rows padded to 64, planes padded so that they do not sit a
  // power of two apart.
  h->esz = elem_bytes(g.precision);
  const int64_t row64 = (int64_t(g.nx) + 63) / 64 * 64;
  const int64_t rrow = rows_row(g.nx);
  const int64_t rows = int64_t(g.ny) * g.nz;
  if (g.layout == LBM_LAYOUT_ROWS || (g.layout == LBM_LAYOUT_AUTO && rows_fit(g))) {
    h->dstride = rrow;
    h->rstride = int32_t(rrow * kQ);
    h->buf_elems = rows * rrow * kQ;
  } else {
    const int64_t raw = row64 * rows;
    const int64_t quantum = int64_t(4096 / h->esz);
    h->rstride = int32_t(row64);
    h->dstride = (raw + quantum - 1) / quantum * quantum + int64_t(512 / h->esz);
    h->buf_elems = h->dstride * kQ;
    if (h->dstride >= (int64_t(1) << 31)) {
      g_err3 = "grid too large: a direction plane must hold fewer than 2^31 elements";
      delete h;
      return LBM_ENOMEM;
    }
  }
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    h->off_buf[k] = off;
    off = align256(off + h->buf_bytes());
  }
  h->off_word = off;
  off = align256(off + h->plan.word.size() * sizeof(uint32_t));
  h->off_strip = off;
  off = align256(off + h->plan.strip.size() * sizeof(uint32_t));
  h->fcap = 2 * h->plan.fstrips.size() + 256;
  h->part_cap = 2 * h->part_doubles() + 4096;
  h->njblocks = h->plan.has_box ? h->plan.box_bx * h->plan.box_rows : 0;
  h->jcap = h->njblocks;
  h->off_fstrip = off;
  off = align256(off + h->fcap * sizeof(uint32_t));
  h->off_uin = off;
  off = align256(off + h->uin.size() * sizeof(double));
  h->off_part = off;
  off = align256(off + 2 * h->part_cap * sizeof(double));
  h->off_jpart = off;
  off = align256(off + size_t(h->jcap) * 3 * sizeof(double));
  h->off_ring = off;
  off = align256(off + size_t(g.max_record) * kRow * sizeof(double));
  h->total = off;
  *out = h;
  return LBM_OK;
}

int lbm3d_workspace_bytes(const lbm3d_t* h, size_t* bytes) {
  if (!h || !bytes) return LBM_EINVAL;
  *bytes = h->total;
  return LBM_OK;
}

int lbm3d_bind(lbm3d_t* h, void* ws, size_t bytes, void* stream) {
  if (!h) return LBM_EINVAL;
  if (!ws) return h->fail(LBM_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return h->fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < h->total) return h->fail(LBM_ENOMEM, "workspace smaller than lbm3d_workspace_bytes");
  h->ws = static_cast<char*>(ws);
  h->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(h->ws + h->off_word, h->plan.word.data(),
                                h->plan.word.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->ws + h->off_strip, h->plan.strip.data(),
                       h->plan.strip.size() * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && !h->plan.fstrips.empty())
    e = hipMemcpyAsync(h->ws + h->off_fstrip, h->plan.fstrips.data(),
                       h->plan.fstrips.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                       h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->ws + h->off_uin, h->uin.data(), h->uin.size() * sizeof(double),
                       hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload plan");
  for (int k = 0; k < 2; ++k) {
    e = launch_fill_rest3(h->g.precision, h->buf(k), h->buf_elems, h->dstride, h->stream);
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

int lbm3d_step(lbm3d_t* h, int32_t n, uint32_t scheme) {
  lbm::TraceRange range("lbm3d_step");
  if (!h) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  if (n < 0) return h->fail(LBM_EINVAL, "n must be >= 0");
  if (scheme & ~LBM3D_FORCE_ALL) return h->fail(LBM_EINVAL, "unknown force scheme bits");
  const bool forces = scheme != 0;
  if (forces && h->nrec + n > h->g.max_record)
    return h->fail(LBM_EOVERFLOW, "force ring would overflow; read lbm3d_forces first");
  if (n == 0) return LBM_OK;
  const int rc = enqueue3(h, n, forces ? h->ring() + h->nrec * kRow : nullptr);
  if (rc != LBM_OK) return rc;
  if (forces) {
    h->nrec += n;
    h->rec_scheme.insert(h->rec_scheme.end(), size_t(n), scheme);
  }
  return LBM_OK;
}

int lbm3d_forces(lbm3d_t* h, double* out, int64_t cap, int64_t* got) {
  lbm::TraceRange range("lbm3d_forces");
  if (!h) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  if (got) *got = h->nrec;
  if (h->nrec == 0) return LBM_OK;
  if (!out || cap < h->nrec) return h->fail(LBM_EINVAL, "output holds fewer rows than recorded");
  std::vector<double> rows(size_t(h->nrec) * kRow);
  hipError_t e = hipMemcpyAsync(rows.data(), h->ring(), rows.size() * sizeof(double),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download force ring");
  bool finite = true;
  for (int64_t t = 0; t < h->nrec; ++t) {
    const double* r = &rows[size_t(t) * kRow];
    const uint32_t sch = h->rec_scheme[size_t(t)];
    double v[12];
    for (int c = 0; c < 3; ++c) {
      v[c] = r[c];
      v[3 + c] = r[3 + c];
      v[6 + c] = r[6 + c] - r[kPart + c] + r[9 + c];
      v[9 + c] = r[12 + c];
    }
    const bool want[4] = {(sch & LBM_FORCE_MEA_A) != 0, (sch & LBM_FORCE_MEA_B) != 0,
                          (sch & LBM_FORCE_DRTT) != 0 && h->plan.has_box,
                          (sch & LBM_FORCE_SI) != 0};
    double* o = out + t * 12;
    for (int s = 0; s < 4; ++s)
      for (int c = 0; c < 3; ++c) {
        o[3 * s + c] = want[s] ? v[3 * s + c] : std::nan("");
        if (want[s] && !std::isfinite(v[3 * s + c])) finite = false;
      }
  }
  h->nrec = 0;
  h->rec_scheme.clear();
  if (!finite) return h->fail(LBM_ENONFINITE, "a recorded force is not finite");
  return LBM_OK;
}

int lbm3d_get_populations(lbm3d_t* h, double* out) {
  if (!h || !out) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  const size_t bytes = h->buf_bytes();
  std::vector<unsigned char> raw(bytes);
  hipError_t e = hipMemcpyAsync(raw.data(), h->buf(h->cur), bytes, hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download populations");
  const int nx = h->g.nx, ny = h->g.ny, nz = h->g.nz, prec = h->g.precision;
  for (int i = 0; i < kQ; ++i) {
    const double base = is_dev(prec) ? host_w27(i) : 0.0;
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const size_t k = size_t(i) * h->dstride + (size_t(z) * ny + y) * h->rstride + x;
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
          out[((size_t(i) * nz + z) * ny + y) * nx + x] = base + v;
        }
  }
  return LBM_OK;
}

int lbm3d_set_populations(lbm3d_t* h, const double* in) {
  if (!h || !in) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  const size_t bytes = h->buf_bytes();
  std::vector<unsigned char> raw(bytes, 0);
  const int nx = h->g.nx, ny = h->g.ny, nz = h->g.nz, prec = h->g.precision;
  for (int i = 0; i < kQ; ++i) {
    const double base = is_dev(prec) ? host_w27(i) : 0.0;
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const size_t k = size_t(i) * h->dstride + (size_t(z) * ny + y) * h->rstride + x;
          const double v = in[((size_t(i) * nz + z) * ny + y) * nx + x] - base;
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
  hipError_t e = hipMemcpyAsync(h->buf(h->cur), raw.data(), bytes, hipMemcpyHostToDevice,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload populations");
  return LBM_OK;
}

int lbm3d_get_links(const lbm3d_t* h, int64_t* out, int64_t cap, int64_t* n) {
  if (!h || !n) return LBM_EINVAL;
  std::vector<int64_t> L;
  plan3_links(h->plan, L);
  *n = int64_t(L.size() / 2);
  const int64_t m = *n < cap ? *n : cap;
  if (m > 0) {
    if (!out) return LBM_EINVAL;
    std::memcpy(out, L.data(), size_t(m) * 2 * sizeof(int64_t));
  }
  return LBM_OK;
}

int lbm3d_get_info(const lbm3d_t* h, lbm3d_info* info) {
  if (!h || !info) return LBM_EINVAL;
  info->n_fluid = h->plan.n_fluid;
  info->n_links = h->plan.n_links;
  info->n_box = h->plan.n_box;
  info->steps_done = h->steps_done;
  info->n_recorded = h->nrec;
  info->n_general = h->plan.ngeneral;
  info->n_strips = int32_t(h->plan.strip.size());
  return LBM_OK;
}

int lbm3d_set_body_motion(lbm3d_t* h, const double* u, const double* omega,
                          const double* centre) {
  if (!h) return LBM_EINVAL;
  if (!u || !omega || !centre) return h->fail(LBM_EINVAL, "null motion vector");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(u[k]) || !std::isfinite(omega[k]) || !std::isfinite(centre[k]))
      return h->fail(LBM_EINVAL, "body motion must be finite");
  bool moving = false;
  for (int k = 0; k < 3; ++k) {
    h->mu[k] = u[k];
    h->mw[k] = omega[k];
    h->mc[k] = centre[k];
    moving = moving || u[k] != 0.0 || omega[k] != 0.0;
  }
  h->moving = moving;
  return LBM_OK;
}

int lbm3d_set_mask(lbm3d_t* h, const uint8_t* mask, const int32_t* box, double* impulse) {
  lbm::TraceRange range("lbm3d_set_mask");
  if (!h || !mask) return LBM_EINVAL;
  lbm3d_grid g = h->g;
  if (box) {
    if ((box[0] >= 0) != (g.box[0] >= 0))
      return h->fail(LBM_EINVAL, "a control volume can be moved, not added or removed");
    for (int k = 0; k < 6; ++k) g.box[k] = box[k];
  }
  // Nodes that swap between fluid and solid, from the mask of the plan compared eight
  // bytes at a time (bytes other than 0/1 are refused by replan3 before anything
  // changes); bit 31 of a list entry: uncovered.
  const size_t n = size_t(g.nx) * g.ny * g.nz;
  const uint8_t* old = h->mask.data();
  std::vector<int32_t> changed, list;
  size_t k = 0;
  for (; k + 8 <= n; k += 8) {
    uint64_t a, b;
    std::memcpy(&a, old + k, 8);
    std::memcpy(&b, mask + k, 8);
    if (a == b) continue;
    for (size_t j = k; j < k + 8; ++j)
      if ((old[j] != 0) != (mask[j] != 0)) changed.push_back(int32_t(j));
  }
  for (; k < n; ++k)
    if ((old[k] != 0) != (mask[k] != 0)) changed.push_back(int32_t(k));
  list.reserve(changed.size());
  for (int32_t c : changed) list.push_back(int32_t(uint32_t(c) | (old[c] ? 0x80000000u : 0u)));
  // Scratch in the other state buffer, which the next step overwrites anyway.
  const int blocks = int(std::min<size_t>((list.size() + 255) / 256, 1024));
  const size_t off_list = align256(n), off_blk = align256(off_list + list.size() * 4),
               off_res = align256(off_blk + size_t(std::max(blocks, 1)) * 24);
  if (h->bound && off_res + 24 > h->buf_bytes())
    return h->fail(LBM_ENOMEM, "too many nodes change at once");
  // Re-classify around the changed nodes; the new plan takes the old words.
  Plan3 np;
  Plan3Delta d;
  std::string perr;
  const int rc = replan3(g, mask, changed, h->plan, np, d, perr);
  if (rc != LBM_OK) return h->fail(rc, perr);
  const int nj = np.has_box ? np.box_bx * np.box_rows : 0;
  if (np.fstrips.size() > h->fcap ||
      size_t(np.nslots) * kPart + size_t(np.njslots) * 3 > h->part_cap || nj > h->jcap) {
    undo_replan3(h->plan, np, d);
    return h->fail(LBM_ENOMEM, nj > h->jcap
                                   ? "the new control volume is larger than the one at create"
                                   : "the new mask needs more force slots than reserved at "
                                     "create; create a handle for it");
  }
  auto commit = [&]() {
    h->plan = std::move(np);
    std::memcpy(h->mask.data(), mask, n);
    h->g = g;
    h->njblocks = nj;
  };
  double P[3] = {0.0, 0.0, 0.0};
  if (h->bound) {
    // Nothing in flight may still read the old node words or the state.
    hipError_t e = hipStreamSynchronize(h->stream);
    char* scr = static_cast<char*>(h->buf(1 - h->cur));
    if (e == hipSuccess && !list.empty()) {
      std::vector<uint8_t> valid(n);  // fluid in both masks
      for (size_t j = 0; j < n; ++j) valid[j] = (old[j] | mask[j]) == 0;
      e = hipMemcpyAsync(scr, valid.data(), n, hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(scr + off_list, list.data(), list.size() * 4, hipMemcpyHostToDevice,
                           h->stream);
      Remask3Args a{};
      a.g = geom(h);
      a.state = h->buf(h->cur);
      a.list = reinterpret_cast<const int32_t*>(scr + off_list);
      a.n = int32_t(list.size());
      a.valid = reinterpret_cast<const uint8_t*>(scr);
      a.rho_w = h->rho_w;
      a.block_out = reinterpret_cast<double*>(scr + off_blk);
      double* res = reinterpret_cast<double*>(scr + off_res);
      if (e == hipSuccess) e = launch_remask3(g.precision, a, blocks, res, h->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(P, res, sizeof(P), hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      // The scratch buffer back to the rest state (its solid nodes are never written).
      if (e == hipSuccess) e = launch_fill_rest3(g.precision, scr, h->buf_elems, h->dstride, h->stream);
    }
    // The rewritten node words (one contiguous index range), the strip table and the
    // force-strip list.
    if (e == hipSuccess && !d.idx.empty()) {
      const size_t lo = size_t(d.idx.front()), cnt = size_t(d.idx.back()) - lo + 1;
      e = hipMemcpyAsync(h->ws + h->off_word + lo * sizeof(uint32_t), np.word.data() + lo,
                         cnt * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->ws + h->off_strip, np.strip.data(), np.strip.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && !np.fstrips.empty())
      e = hipMemcpyAsync(h->ws + h->off_fstrip, np.fstrips.data(),
                         np.fstrips.size() * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      commit();  // the state is undefined; the plan is the new mask's
      return h->hip_fail(e, "mask change");
    }
  }
  commit();
  if (impulse)
    for (int c = 0; c < 3; ++c) impulse[c] = P[c];
  return LBM_OK;
}

int lbm3d_state_bytes(const lbm3d_t* h, size_t* bytes) {
  if (!h || !bytes) return LBM_EINVAL;
  *bytes = sizeof(State3Header) + h->buf_bytes();
  return LBM_OK;
}

int lbm3d_get_state(lbm3d_t* h, void* blob, size_t cap) {
  if (!h || !blob) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  size_t need = 0;
  lbm3d_state_bytes(h, &need);
  if (cap < need) return h->fail(LBM_EINVAL, "state buffer too small");
  State3Header hd{};
  hd.magic = kState3Magic;
  hd.nx = h->g.nx;
  hd.ny = h->g.ny;
  hd.nz = h->g.nz;
  hd.precision = h->g.precision;
  hd.dstride = h->dstride;
  hd.rstride = h->rstride;
  hd.steps_done = h->steps_done;
  std::memcpy(blob, &hd, sizeof hd);
  hipError_t e = hipMemcpyAsync(static_cast<char*>(blob) + sizeof hd, h->buf(h->cur),
                                need - sizeof hd, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "download state");
  return LBM_OK;
}

int lbm3d_set_state(lbm3d_t* h, const void* blob, size_t n) {
  if (!h || !blob) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  size_t need = 0;
  lbm3d_state_bytes(h, &need);
  State3Header hd{};
  if (n < sizeof hd) return h->fail(LBM_EINVAL, "state blob too small");
  std::memcpy(&hd, blob, sizeof hd);
  if (hd.magic != kState3Magic || hd.nx != h->g.nx || hd.ny != h->g.ny || hd.nz != h->g.nz ||
      hd.precision != h->g.precision || hd.dstride != h->dstride ||
      hd.rstride != h->rstride || n != need)
    return h->fail(LBM_EINVAL, "state blob does not match this handle");
  hipError_t e = hipMemcpyAsync(h->buf(h->cur), static_cast<const char*>(blob) + sizeof hd,
                                need - sizeof hd, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "upload state");
  h->steps_done = hd.steps_done;
  return LBM_OK;
}

int lbm3d_reset(lbm3d_t* h) {
  if (!h) return LBM_EINVAL;
  if (!h->bound) return h->fail(LBM_ESTATE, "handle is not bound to a workspace");
  for (int k = 0; k < 2; ++k) {
    hipError_t e = launch_fill_rest3(h->g.precision, h->buf(k), h->buf_elems, h->dstride,
                                     h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "fill rest state");
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "reset synchronize");
  h->cur = 0;
  h->steps_done = 0;
  h->nrec = 0;
  h->rec_scheme.clear();
  return LBM_OK;
}

int lbm3d_set_tau(lbm3d_t* h, double tau) {
  if (!h) return LBM_EINVAL;
  if (!std::isfinite(tau) || tau <= 0.5) return h->fail(LBM_EINVAL, "tau must be finite and > 1/2");
  h->tau = tau;
  return LBM_OK;
}

int lbm3d_set_inlet(lbm3d_t* h, const double* uin) {
  if (!h || !uin) return LBM_EINVAL;
  if (h->g.bc_x != LBM_BCX_INLET_OUTLET) return h->fail(LBM_EINVAL, "the lattice has no inlet");
  for (size_t k = 0; k < h->uin.size(); ++k)
    if (!std::isfinite(uin[k])) return h->fail(LBM_EINVAL, "inlet velocity is not finite");
  h->uin.assign(uin, uin + h->uin.size());
  if (h->bound) {
    hipError_t e = hipMemcpyAsync(h->ws + h->off_uin, h->uin.data(),
                                  h->uin.size() * sizeof(double), hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "upload inlet");
  }
  return LBM_OK;
}

void lbm3d_destroy(lbm3d_t* h) { delete h; }

const char* lbm3d_last_error(const lbm3d_t* h) { return h ? h->err.c_str() : g_err3.c_str(); }

}  // extern "C"
