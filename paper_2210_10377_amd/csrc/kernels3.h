// Kernel arguments and launchers of the three-dimensional (D3Q27) path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm3 {

// Geometry and tables of a lattice as the kernels read them.
struct Geom3 {
  // A state buffer holds population i of node (x, y, z) at
  // i * dstride + (z * ny + y) * rstride + x (row-interleaved: dstride = padded row,
  // rstride = 27 rows; planar: dstride = padded plane, rstride = padded row).
  int64_t dstride;      // elements between directions of a node
  int32_t rstride;      // elements between rows (fixed y, z)
  int32_t nx, ny, nz;
  int32_t bc_x, bc_y, bc_z;
  int32_t box[6];       // control volume (has_box)
  int32_t whole[3];     // box spans the whole (periodic) axis
  int32_t has_box;
  const uint32_t* word; // [nz][ny][nx] node words
  const double* uin;    // [nz][ny] inlet x-velocity
  double rho_w6;        // 6 rho_w: inlet term 2 rho_w w_i (c_i . u_w) / theta0
  // Rigid motion of the body (moving != 0): the wall velocity at a point x is
  // mu + mw x (x - mc).
  double mu[3], mw[3], mc[3];
  int32_t moving;
};

struct Step3Args {
  Geom3 g;
  const void* src;
  void* dst;
  int32_t ntx;               // tiles per row
  int64_t ntiles;
  const uint32_t* strip;     // [ntiles * 4] strip table
  const uint32_t* fstrips;   // [nslots] strip index of each force slot
  double omega;
  int32_t collision;         // LBM_COLL_BGK or LBM_COLL_REGULARIZED
  int32_t nslots, njslots;   // force slots (15 doubles), J slots (3 doubles)
  double* part_out;          // partials of this step: [nslots][15] then [njslots][3]
  // Reducer (last block of the launch): the previous step's partials into its ring row,
  // and its J into the J(t+1) of the row before.
  const double* red_in;
  double* red_row;
  double* red_prev_jnext;
  uint32_t step_key;         // stochastically rounded storage: key of the step number
};

struct Box3Args {
  Geom3 g;
  const void* src;
  double* jpart;  // [blocks][3]
};

struct Final3Args {
  const double* red_in;
  int32_t nslots, njslots;
  double* row;
  double* prev_jnext;
  const double* jpart;  // J of the pull after the last step, per box-sweep block
  int32_t njblocks;
};

// A mask change of a body moving through the grid, over the current state buffer.
struct Remask3Args {
  Geom3 g;                // geometry and the rigid motion (wall velocity of refills)
  void* state;            // current state buffer
  const int32_t* list;    // [n] node index (z*ny + y)*nx + x; bit 31: uncovered
  int32_t n;
  const uint8_t* valid;   // [nz][ny][nx] 1 where fluid in both masks
  double rho_w;           // density of a refill without valid neighbours
  double* block_out;      // [blocks][3] covered minus refilled momentum per block
};

hipError_t launch_step3(int precision, bool forces, const Step3Args& a, hipStream_t s);
// Refill the uncovered nodes and sum, in a fixed order, the momentum of the covered
// ones minus that of the refilled ones into out[3].
hipError_t launch_remask3(int precision, const Remask3Args& a, int blocks, double* out,
                          hipStream_t s);
hipError_t launch_box3(int precision, const Box3Args& a, int blocks, hipStream_t s);
hipError_t launch_final3(const Final3Args& a, hipStream_t s);
// Rest state w_i in all n elements of a buffer with direction stride dstride.
hipError_t launch_fill_rest3(int precision, void* buf, int64_t n, int64_t dstride, hipStream_t s);

}  // namespace lbm3
