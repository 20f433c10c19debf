// Launch interface of the adjoint kernel (adjoint.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace lbm {

// One reverse step t: mu(t) from mu(t+1) and the stored state S(t-1).
struct AdjArgs {
  const void* state;     // S(t-1), storage type, state layout
  const void* mu_in;     // mu(t+1), arithmetic type, same layout (zero at the end)
  void* mu_out;          // mu(t)
  int64_t plane;         // elements between directions (state and adjoint share it)
  uint32_t state_bytes;  // bytes of a state buffer below 4 GiB (buffer addressing), else 0
  uint32_t mu_bytes;     // bytes of an adjoint buffer below 4 GiB, else 0
  int32_t pitch, nx, ny, ntx, ntiles;
  int32_t tile_rows;           // rows of a tile: 1 (256 x 1) or 4 (64 x 4)
  int32_t gx0, gx1, gy0, gy1;  // node rectangle of the general path (as the step kernel)
  const uint32_t* node;        // forward pull codes
  const uint32_t* adj;         // adjoint codes (readers of each population)
  const double* uin;
  double rho_w6;
  double omega;
  double gx, gy;     // dJ/dS on a body link (s, k): gx c_kx + gy c_ky (0 outside the window)
  double* domega;    // [ntiles * strips] running sums of dJ/domega
  double* duin;      // [ny] running sums of dJ/du_in
};

hipError_t launch_adjoint(int precision, const AdjArgs& a, hipStream_t s);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s);

}  // namespace lbm
