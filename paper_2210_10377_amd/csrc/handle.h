// The handle of the C ABI (include/lbm.h), shared by the single-lattice entry points
// (api.hip) and the batched ones (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.h"
#include "lbm.h"
#include "plan.h"

struct lbm_t {
  lbm_grid g;
  double tau = 0.0, omega = 0.0, rho_w = 1.0;
  lbm::BodyMotion motion{0.0, 0.0, 0.0, 0.0, 0.0, 0};
  std::vector<double> uin;
  lbm::Plan plan;
  std::vector<uint8_t> mask;  // the body mask of the plan ([ny][nx], 0/1)
  // device layout
  // Population i of node (x, y) at i * plane + y * pitch + x (elements): row-interleaved
  // (plane = padded row, pitch = 9 rows) or planar (plane = padded plane, pitch = row).
  int32_t pitch = 0;
  int64_t plane = 0;
  int64_t buf_elems = 0;  // elements of one state buffer
  size_t esz = 0;
  size_t off_buf[2] = {0, 0}, off_node = 0, off_tiles = 0, off_uin = 0, off_motion = 0, off_part = 0,
         off_jpart = 0, off_ring = 0, total = 0;
  int njblocks = 0;
  // Reserved at create so that a new mask (a body moving through the grid) fits the
  // same layout: doubles of one step's force partials, blocks of the box sweep.
  size_t part_cap = 0;
  int jcap = 0;
  // binding
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int cur = 0;  // buffer holding the current state
  int64_t steps_done = 0;
  uint64_t plan_gen = 0;  // counts plan replacements (mask changes)
  int64_t nrec = 0;
  std::vector<uint32_t> rec_scheme;  // scheme mask per recorded row
  std::string err;
  // adjoint: workspace and the forward run it holds
  bool adj_valid = false;
  char* aws = nullptr;
  size_t aws_bytes = 0;
  int32_t adj_n = 0, adj_every = 0, adj_t0 = 0, adj_T = 0;
  int64_t adj_base = 0;  // step count at the forward run's start (its first step's number)
  double adj_wx = 0.0, adj_wy = 0.0;
  std::vector<uint32_t> adj_codes;
  // reverse sweep: recomputation stream and its events (created at first use)
  hipStream_t aux = nullptr;
  hipEvent_t ev_go = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};

  lbm_t() = default;
  lbm_t(const lbm_t&) = delete;
  lbm_t& operator=(const lbm_t&) = delete;
  ~lbm_t() { release_aux(); }
  void release_aux() {
    for (hipEvent_t* ev : {&ev_go, &ev_rec[0], &ev_rec[1], &ev_adj[0], &ev_adj[1]}) {
      if (*ev) (void)hipEventDestroy(*ev);
      *ev = nullptr;
    }
    if (aux) (void)hipStreamDestroy(aux);
    aux = nullptr;
  }

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EHIP;
  }
  void* buf(int k) const { return ws + off_buf[k]; }
  size_t buf_bytes() const { return size_t(buf_elems) * esz; }
  // Size of one state buffer for buffer-resource addressing, or 0 when it needs 64-bit
  // addresses.
  uint32_t buf_bytes32() const {
    const uint64_t b = buf_bytes();
    return b < (uint64_t(1) << 32) - 4096 ? uint32_t(b) : 0u;
  }
  double* ring() const { return reinterpret_cast<double*>(ws + off_ring); }
  // The body motion as the kernels read it (device), or null for a body at rest.
  const lbm::BodyMotion* motion_dev() const {
    return motion.moving ? reinterpret_cast<const lbm::BodyMotion*>(ws + off_motion) : nullptr;
  }
  // Doubles of one step's force partials: general strips, then box-interior strips.
  size_t part_doubles() const {
    return size_t(plan.nslots) * lbm::kPart + size_t(plan.njslots) * lbm::kBoxPart;
  }
  double* part(int k) const {
    return reinterpret_cast<double*>(ws + off_part) + size_t(k) * part_cap;
  }
};

namespace lbm {

// Device tables a step reads besides the state buffers, and the force scratch it writes:
// in the handle's workspace (ws_tables), or elsewhere (the static scratch of the
// allocation-free entry point).
struct DevTables {
  const uint32_t* node;        // per-node pull codes
  const int32_t* strip_slot;   // per-strip force slots
  const double* uin;           // [ny] inlet profile
  const BodyMotion* motion;    // body motion (device), or null at rest
  double* part[2];             // force partials of alternate steps
  double* jpart;               // box-sweep partials
};
DevTables ws_tables(const lbm_t* h);

// Kernel arguments of the handle's step (src, dst and the force buffers unset).
StepArgs step_args(const lbm_t* h);
StepArgs step_args(const lbm_t* h, const DevTables& t);
// Control-volume sweep arguments of the handle over the state `src`.
BoxArgs box_args(const lbm_t* h, const void* src);
BoxArgs box_args(const lbm_t* h, const void* src, const DevTables& t);
// Enqueue n >= 1 steps alternating between two state buffers (step k reads b[k & 1]
// and writes the other) with the tables t; with a non-null ring, step k's force row
// goes to ring row k.  Leaves the handle's own buffers and counters alone.
int enqueue_pingpong(lbm_t* h, const DevTables& t, void* b0, void* b1, hipStream_t stream,
                     int32_t n, double* ring);
// One ring row -> forces [A, B, DRTT, SI, DRTT-post][x, y] (NaN for schemes not
// recorded, and for the DRTT forms without a control volume); returns false if a
// recorded force is not finite.
bool row_forces(const double* row, uint32_t scheme, bool has_box, double* out);

}  // namespace lbm
