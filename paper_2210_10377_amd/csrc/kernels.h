// Launch interface between the C ABI (api.hip) and the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace lbm {

// Force partial of one strip, and the per-step sums: FAx FAy FBx FBy Jx Jy Phix Phiy
// SIx SIy Jpx Jpy (J before collision, Jp after it, both over the control volume).
constexpr int kPart = 12;
constexpr int kJpost = 10;
// Partial of a box-interior strip: Jx Jy Jpx Jpy.
constexpr int kBoxPart = 4;
// Force-ring row: the kPart sums, then Jnext_x Jnext_y (the J of the following step).
constexpr int kRingRow = 14;
constexpr int kJnext = 12;
// Estimators of a force row as lbm_forces reports them: A, B, DRTT, SI, DRTT-post.
constexpr int kSchemes = 5;

// 32-bit finalizer of MurmurHash3 (A. Appleby, public domain): a bijection of 32-bit
// words in which every input bit flips every output bit with probability close to 1/2.
constexpr uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
// Key of step number t (counted from the handle's creation or last reset) for the
// stochastically rounded storage.
constexpr uint32_t sr_step_key(int64_t t) {
  return fmix32(fmix32(uint32_t(t)) ^ uint32_t(uint64_t(t) >> 32) ^ 0x2545f491u);
}

// Rigid motion of the body: velocity U + Omega e_z x (x - c) at a point x.  Kernels read
// it from device memory, and only on body links, through a pointer that is null for a
// body at rest.
struct BodyMotion {
  double ux, uy, omega, xc, yc;
  int32_t moving;
};

// Arguments of one fused time step.
struct StepArgs {
  const void* src;  // post-collision state of the previous step (storage type)
  void* dst;        // post-collision state of this step
  int64_t plane;    // elements between the directions of a node (i * plane + y * pitch + x)
  uint32_t buf_bytes;  // bytes of one state buffer when below 4 GiB (buffer-resource
                       // addressing), 0 for 64-bit global addressing
  int32_t pitch;    // elements between rows
  int32_t nx, ny;
  int32_t bc_x, bc_y;  // LBM_BCX_*, LBM_BCY_*
  int32_t tile_rows;   // rows of a tile: 1 (256 x 1) or 4 (64 x 4)
  int32_t ntx, nty, ntiles;
  int32_t gx0, gx1, gy0, gy1;  // node rectangle (inclusive) of every non-border node that
                               // needs the general path; empty when gx0 > gx1
  int32_t bx0, bx1, by0, by1;  // control-volume box; bx0 > bx1 when there is none
  const uint32_t* node;        // per-node pull codes
  const int32_t* strip_slot;   // per 64-node strip: force partial slot, or -1
  const double* uin;           // [ny] inlet velocity
  double rho_w6;               // 2 rho_w / c_s^2 = 6 rho_w
  const BodyMotion* motion;    // body motion (device), or null for a body at rest
  double omega;                // 1 / tau_lb
  int32_t collision;           // LBM_COLL_*
  double* part_out;            // force partials of this step ([nslots][kPart] of the
                               // general strips, then [njslots][kBoxPart] box momenta),
                               // or null
  const double* red_in;        // partials of the previous step (same layout), or null
  int32_t nslots, njslots;
  double* red_row;             // ring row receiving the reduced previous step
  double* red_prev_jnext;      // Jnext slot of the row before that, or null
  uint32_t step_key;           // stochastically rounded storage: fmix32 of the step number
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
  const BodyMotion* motion;   // device, or null
  double* jpart;              // [blocks][2]
};

struct FinalArgs {
  const double* red_in;   // partials of the last step (StepArgs layout)
  int32_t nslots, njslots;
  double* row;            // ring row of the last step
  double* prev_jnext;     // Jnext slot of the row before, or null
  const double* jpart;    // [njblocks][2], or null when there is no box
  int32_t njblocks;
};

// One instance of a batch, as the batched kernels read it from device memory.
struct BatchInst {
  StepArgs a;               // geometry, tables and physics (src/dst/partials unused)
  void* buf[2];             // the two state buffers
  double* part[2];          // force partial buffers of alternate steps
  double* ring;             // this instance's force row of step 0 ([rows][n_inst][kRingRow])
  BoxArgs box;              // control-volume sweep (src chosen per launch)
  int32_t njblocks;         // blocks of that sweep (0 without a box)
  BodyMotion mot;           // the member's body motion; a.motion and box.motion point here
  int64_t step_off;         // the member's step count less the batch's (step keys)
};

// Tiles taken per atomic of the batch's tile queue.
constexpr int kQueueChunk = 16;

struct BatchLaunch {
  const BatchInst* inst;     // [n_inst], device
  const int32_t* tile_inst;  // [total_tiles] instance of each tile, device
  const int32_t* tile_local; // [total_tiles] tile index inside its instance, device
  const int32_t* box_inst;   // [total_box_blocks] instance of each box-sweep block
  const int32_t* box_local;  // [total_box_blocks] block index inside its instance's sweep
  const int32_t* ctl;        // {first force row of the launch sequence, steps of the call
                             // before it, the batch's step count at the call (low, high)}
  int32_t* queue;            // two tile counters of the queue schedule (launch parity), or null
  int32_t n_inst, nred;      // instances; reducer blocks (n_inst rounded up to 8)
  int32_t total_tiles, total_box_blocks;
  int32_t grid_blocks;       // tile blocks per launch (0: one block per tile)
  int32_t collision;         // LBM_COLL_* of every instance
  int32_t moving;            // some instance has a body in motion
};

// A mask change of a body moving through the grid, over the current state buffer.
struct RemaskArgs {
  void* state;            // current state buffer (stored populations)
  int64_t plane;          // elements between the directions of a node
  int32_t pitch, nx, ny, bc_x, bc_y;
  const int32_t* list;    // [n] y * nx + x; bit 31 set: uncovered (refill), clear: covered
  int32_t n;
  const uint8_t* valid;   // [ny * nx] 1 where the node is fluid in both masks
  double rho_w;           // density of a refilled node without valid neighbours
  BodyMotion motion;      // wall velocity of the refilled nodes (all zero at rest)
  double* block_out;      // [blocks][2] covered minus refilled momentum of each block
};

// Pressure coefficient at listed nodes of a state buffer (see launch_boundary_cp).
struct CpArgs {
  const void* state;      // current state buffer (stored populations)
  int64_t plane;          // elements between the directions of a node
  int32_t pitch, nx;
  const int32_t* nodes;   // [n] y * nx + x
  int32_t n;
  int32_t ref_node;       // y * nx + x of the reference node, or -1
  double p_ref;           // reference pressure when ref_node < 0
  double q;               // dynamic pressure rho_ref u_ref^2 / 2
  double* out;            // [n]
};

hipError_t launch_step(int precision, bool forces, const StepArgs& a, hipStream_t s);
// C_p = (rho/3 - p_inf) / q at every listed node, rho the sum of the node's stored
// populations in binary64, p_inf = rho/3 of the reference node (or p_ref).
hipError_t launch_boundary_cp(int precision, const CpArgs& a, hipStream_t s);
// Refill the uncovered nodes and sum, in a fixed order, the momentum of the covered
// ones minus that of the refilled ones into out[2] (block_out as scratch).
hipError_t launch_remask(int precision, const RemaskArgs& a, int blocks, double* out,
                         hipStream_t s);
hipError_t launch_batch_step(int precision, bool forces, const BatchLaunch& b, int32_t parity,
                             int32_t k, hipStream_t s);
hipError_t launch_batch_ctl(int32_t* ctl, int32_t row_base, int32_t nprev, int64_t base,
                            hipStream_t s);
// Zeroes both tile counters of the queue schedule (before a call's first launch).
hipError_t launch_batch_queue_reset(int32_t* queue, hipStream_t s);
// Control-volume sweeps over buffer `parity` and finalization of force row `row` of every
// instance (the last step of a call; its partials are in part[part_parity]).
hipError_t launch_batch_tail(int precision, const BatchLaunch& b, int32_t parity, int32_t row,
                             int32_t part_parity, bool has_prev, hipStream_t s);
hipError_t launch_box_momentum(int precision, const BoxArgs& a, int blocks, hipStream_t s);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
// Rest state w_i in every element of a population buffer (padding included).
// Rest state w_i in all n elements of a state buffer whose directions sit plane elements
// apart.
hipError_t launch_fill_rest(int precision, void* buf, int64_t n, int64_t plane, hipStream_t s);

}  // namespace lbm
