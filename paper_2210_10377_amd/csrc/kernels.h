// Launch interface between the C ABI (api.hip) and the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace lbm {

// Arguments of one fused time step.
struct StepArgs {
  const void* src;  // post-collision state of the previous step (storage type)
  void* dst;        // post-collision state of this step
  int64_t plane;    // population plane stride, elements
  uint32_t buf_bytes;  // bytes of one state buffer when below 4 GiB (buffer-resource
                       // addressing), 0 for 64-bit global addressing
  int32_t pitch;    // row pitch, elements
  int32_t nx, ny;
  int32_t ntx, nty, ntiles;
  int32_t gx0, gx1, gy0, gy1;  // node rectangle (inclusive) of every non-border node that
                               // needs the general path; empty when gx0 > gx1
  int32_t bx0, bx1, by0, by1;  // control-volume box; bx0 > bx1 when there is none
  const uint32_t* node;        // per-node pull codes
  const int32_t* strip_slot;   // per 64-node strip: force partial slot, or -1
  const double* uin;           // [ny] inlet velocity
  double rho_w6;               // 2 rho_w / c_s^2 = 6 rho_w
  double omega;                // 1 / tau_lb
  double* part_out;            // [nslots][8] force partials of this step, or null
  const double* red_in;        // [nslots][8] partials of the previous step, or null
  int32_t nslots;
  double* red_row;             // ring row receiving the reduced previous step
  double* red_prev_jnext;      // Jnext slot of the row before that, or null
};

// Control-volume momentum of the populations one pull of `src` gives (the J(t+1) of
// the last recorded step).
struct BoxArgs {
  const void* src;
  int64_t plane;
  uint32_t buf_bytes;
  int32_t pitch, nx, ny;
  int32_t bx0, bx1, by0, by1;
  int32_t box_bx;             // blocks per box row
  const uint32_t* node;
  const double* uin;
  double rho_w6;
  double* jpart;              // [blocks][2]
};

struct FinalArgs {
  const double* red_in;   // [nslots][8] partials of the last step
  int32_t nslots;
  double* row;            // ring row of the last step
  double* prev_jnext;     // Jnext slot of the row before, or null
  const double* jpart;    // [njblocks][2], or null when there is no box
  int32_t njblocks;
};

hipError_t launch_step(int precision, bool forces, const StepArgs& a, hipStream_t s);
hipError_t launch_box_momentum(int precision, const BoxArgs& a, int blocks, hipStream_t s);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
// Rest state w_i in every element of a population buffer (padding included).
hipError_t launch_fill_rest(int precision, void* buf, int64_t plane, hipStream_t s);

}  // namespace lbm
