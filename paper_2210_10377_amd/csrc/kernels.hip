// HIP kernels for gfx950: the fused D2Q9 pull-stream + BGK collision step with the
// per-step momentum-exchange (algorithms A and B) and DRTT force sums.
//
// Kaushal, Succi & Ansumali, arXiv:2210.10377: Eq. CollideAdv (collide, then stream),
// the second-order equilibrium and Table I (Sec. II), stationary and moving-wall
// bounce-back (Sec. II), the momentum exchange of Sec. III with the two operator
// orders of Eq. rtt4, and the control-volume balance of the second Eq. rtt7.
//
// Data layout (HBM): structure of arrays, x fastest; population i of node (x, y) sits at
// i * plane + y * pitch + x, with the strides from the host (row-interleaved: the nine
// directions of a row side by side; or one plane per direction).  Every node is updated
// by one thread of a 256-thread block; each wave of a block covers a strip of 64 nodes
// of one row, the four strips of a block side by side (256 x 1 tiles) or one above the
// other (64 x 4 tiles, for grids with short rows).
// Strips of plain fluid (all pulls plain streaming, away from the control-volume band)
// take a branch-free path that reads no per-node metadata; the other strips read a
// 32-bit word of pull codes per node, apply the boundary rules, and accumulate the
// force sums in FP64.  Waves never wait for each other: a strip with force terms
// reduces them over the wave and writes one partial slot; the slots are reduced in a
// fixed order by one extra block (dispatched first) of the next step's launch, or by
// the finalize kernel, so every force is deterministic.
//
// Addressing: when a state buffer is below 4 GiB its populations are read and written
// through buffer resources (one descriptor per buffer, the direction offsets in scalar
// registers, 32-bit per-lane offsets); out-of-range offsets read zero and drop writes.
// Larger buffers use 64-bit global addresses.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace lbm {

namespace {

using namespace dev;

__device__ __forceinline__ bool in_box(const StepArgs& a, int x, int y) {
  return x >= a.bx0 && x < a.bx1 && y >= a.by0 && y < a.by1;
}

__device__ __forceinline__ int lane_id() { return int(threadIdx.x) & 63; }

// Interior strip at (x0, y0): plain pull streaming in every direction, no metadata; the
// nine loads are issued together.
template <int P, bool BUF>
__device__ __forceinline__ void interior_load(const StepArgs& a, int x0, int y0,
                                              typename Storage<P>::T (&v)[kQ]) {
  using T = typename Storage<P>::T;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const int pitch = a.pitch;
  const int32_t o0 = y0 * pitch + x0 + lane_id();
#pragma unroll
  for (int i = 0; i < kQ; ++i) v[i] = src.ld(i, o0 - kCy[i] * pitch - kCx[i]);
}

// Collision and store of an interior strip; with JP the momentum of the stored
// (post-collision) populations is added to jp (binary64).
template <int P, bool BUF, int COLL, bool JP = false>
__device__ __forceinline__ void interior_finish(const StepArgs& a, int x0, int y0,
                                                const typename Storage<P>::T (&v)[kQ],
                                                double* jp = nullptr) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> dst(a.dst, a.plane, a.buf_bytes);
  const int32_t o = y0 * a.pitch + x0 + lane_id();
  C f[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) f[i] = unpack<P>(v[i], i);
  C g[kQ];
  collide<C, S::kDev, COLL, S::kExactW>(f, C(a.omega), g);
  const uint32_t word = S::kSR ? sr_node_word(a.step_key, a.nx, x0 + lane_id(), y0) : 0u;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const T q = pack_sr<P>(g[i], i, word);
    dst.st(i, o, q);
    if constexpr (JP) {
      if (i > 0) {
        const double fi = to_f64<P>(q, i);
        jp[0] += kCx[i] * fi;
        jp[1] += kCy[i] * fi;
      }
    }
  }
}

// Plain strip on the first or last row, or holding x = 0, x = nx - 1 or lanes past the
// row end: the pull codes are those of edge_word (walls or wrap, inlet or wrap, outlet
// or wrap, plain streaming elsewhere), made from the lane's coordinates alone, with no
// per-node metadata; no forces.
template <int P, bool BUF, int COLL>
__device__ __forceinline__ void edge_strip(const StepArgs& a, int x0, int y) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const Planes<T, BUF> dst(a.dst, a.plane, a.buf_bytes);
  const int pitch = a.pitch;
  const int x = x0 + lane_id();
  if (x >= a.nx) return;
  const uint32_t w = edge_word_bits(a.nx, a.ny, a.bc_x, a.bc_y, x, y);
  C f[kQ];
  pull_all<P>(src, pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, f);
  C g[kQ];
  collide<C, S::kDev, COLL, S::kExactW>(f, C(a.omega), g);
  const int32_t o = y * pitch + x;
  const uint32_t word = S::kSR ? sr_node_word(a.step_key, a.nx, x, y) : 0u;
#pragma unroll
  for (int i = 0; i < kQ; ++i) dst.st(i, o, pack_sr<P>(g[i], i, word));
}

// Control-volume terms of fluid node (x, y) (second Eq. rtt7) added to acc: the
// momentum of its populations before collision (f) and as stored after it (s) when it
// lies in the control volume, and the stored populations crossing the box surface:
// entering V (+) from a node outside, leaving V (-) from a node inside.
template <int P>
__device__ __forceinline__ void box_terms(const StepArgs& a, int x, int y,
                                          const typename Storage<P>::C (&f)[kQ],
                                          const typename Storage<P>::T (&s)[kQ],
                                          double (&acc)[kPart]) {
  using S = Storage<P>;
  if (in_box(a, x, y)) {
    double jx = 0.0, jy = 0.0, px = 0.0, py = 0.0;
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
      const double fi = pre_f64<P>(f[i], i);
      jx += kCx[i] * fi;
      jy += kCy[i] * fi;
      const double sv = to_f64<P>(s[i], i);
      px += kCx[i] * sv;
      py += kCy[i] * sv;
    }
    acc[4] += jx;
    acc[5] += jy;
    acc[kJpost] += px;
    acc[kJpost + 1] += py;
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      if (!in_box(a, x + kCx[i], y + kCy[i])) {
        const double sv = to_f64<P>(s[i], i);
        acc[6] -= kCx[i] * sv;
        acc[7] -= kCy[i] * sv;
      }
  } else {
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      if (in_box(a, x + kCx[i], y + kCy[i])) {
        const double sv = to_f64<P>(s[i], i);
        acc[6] += kCx[i] * sv;
        acc[7] += kCy[i] * sv;
      }
  }
}

// Interior strip touching the control-volume surface: plain pulls (the loaded v),
// collision and store as interior_finish, and the control-volume terms of every node.
template <int P, bool BUF, int COLL>
__device__ __forceinline__ void ring_finish(const StepArgs& a, int x0, int y0,
                                            const typename Storage<P>::T (&v)[kQ],
                                            double (&acc)[kPart]) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> dst(a.dst, a.plane, a.buf_bytes);
  const int x = x0 + lane_id();
  const int32_t o = y0 * a.pitch + x;
  C f[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) f[i] = unpack<P>(v[i], i);
  C g[kQ];
  collide<C, S::kDev, COLL, S::kExactW>(f, C(a.omega), g);
  const uint32_t word = S::kSR ? sr_node_word(a.step_key, a.nx, x, y0) : 0u;
  T s[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    s[i] = pack_sr<P>(g[i], i, word);
    dst.st(i, o, s[i]);
  }
  box_terms<P>(a, x, y0, f, s, acc);
}

// General path of one lane of a strip: boundary rules from the pull codes, and (when
// `forces`) the force sums of its node added to acc.
template <int P, bool BUF, int COLL, bool MOV>
__device__ __forceinline__ void general_strip(const StepArgs& a, int x0, int y, bool forces,
                                              double (&acc)[kPart]) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const Planes<T, BUF> dst(a.dst, a.plane, a.buf_bytes);
  const int pitch = a.pitch;
  const int x = x0 + lane_id();
  {
    if (x >= a.nx) return;
    const uint32_t w = a.node[int64_t(y) * a.nx + x];
    if (w & kSolidBit) return;
    const int32_t o = y * pitch + x;
    C f[kQ];
    pull_all<P>(src, pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, f, MOV ? a.motion : nullptr);
    C g[kQ];
    collide<C, S::kDev, COLL, S::kExactW>(f, C(a.omega), g);
    const uint32_t word = S::kSR ? sr_node_word(a.step_key, a.nx, x, y) : 0u;
    T s[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      s[i] = pack_sr<P>(g[i], i, word);
      dst.st(i, o, s[i]);
    }
    if (forces) {
      // Momentum exchange on the links of this node (Sec. III; Eq. rtt4): the
      // population leaving along c_i towards the body is f_i before collision (A) or
      // f~_i after it (B); the body returns f~_i (as stored) along -c_i, less the
      // moving-wall term of that return when the body moves.
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        if (pull_code(w, kOpp[i]) != kBody) continue;
        const double sv = to_f64<P>(s[i], i);
        const double back =
            (MOV && a.motion) ? sv + body_wall_term(*a.motion, a.rho_w6, kOpp[i], x, y) : sv;
        const double fa = pre_f64<P>(f[i], i) + back;
        acc[0] += kCx[i] * fa;
        acc[1] += kCy[i] * fa;
        acc[2] += kCx[i] * (sv + back);
        acc[3] += kCy[i] * (sv + back);
      }
      // Control volume (second Eq. rtt7).
      box_terms<P>(a, x, y, f, s, acc);
      // Stress integration (Sec. III, Eq. stress_int): each axis link of this node is a
      // unit face of the staircase surface with normal -c_i out of the body; the
      // traction (-p I + sigma) . n uses p = rho/3 and sigma = -(1 - omega/2) Pi^neq of
      // the pre-collision populations (Pi^neq = sum c c f - rho u u - rho I/3), in
      // binary64.  Faces are linear in n, so the node adds the traction of their sum.
      int nsx = 0, nsy = 0;
#pragma unroll
      for (int i = 1; i <= 4; ++i)
        if (pull_code(w, kOpp[i]) == kBody) {
          nsx -= kCx[i];
          nsy -= kCy[i];
        }
      if (nsx != 0 || nsy != 0) {
        double fd[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i)
          fd[i] = pre_f64<P>(f[i], i);
        const double rho = ((fd[0] + fd[1]) + (fd[2] + fd[3])) + ((fd[4] + fd[5]) + (fd[6] + fd[7])) + fd[8];
        const double ux = ((fd[1] + fd[5] + fd[8]) - (fd[3] + fd[6] + fd[7])) / rho;
        const double uy = ((fd[2] + fd[5] + fd[6]) - (fd[4] + fd[7] + fd[8])) / rho;
        const double diag = (fd[5] + fd[6]) + (fd[7] + fd[8]);
        const double p = rho * (1.0 / 3.0);
        const double visc = -(1.0 - 0.5 * a.omega);
        const double sxx = visc * (((fd[1] + fd[3]) + diag) - rho * ux * ux - p);
        const double syy = visc * (((fd[2] + fd[4]) + diag) - rho * uy * uy - p);
        const double sxy = visc * (((fd[5] + fd[7]) - (fd[6] + fd[8])) - rho * ux * uy);
        acc[8] += (sxx - p) * nsx + sxy * nsy;
        acc[9] += sxy * nsx + (syy - p) * nsy;
      }
    }
  }
}

// Force row of the previous step from its partial slots (fixed order).
__device__ __forceinline__ void reduce_row(const double* red_in, int nslots, int njslots,
                                           double* row, double* prev_jnext) {
  // General strips, then the box momenta of the box-interior strips (J before and after
  // collision, added to the two J sums).
  double t = reduce_partials<kPart>(red_in, nslots);
  const double tj = reduce_partials<kBoxPart>(red_in + int64_t(nslots) * kPart, njslots);
  const int tid = int(threadIdx.x);
  const bool pre = tid == 4 || tid == 5, post = tid == kJpost || tid == kJpost + 1;
  const double tjs = __shfl(tj, pre ? tid - 4 : (post ? tid - kJpost + 2 : 0), 64);
  if (pre || post) t += tjs;
  if (threadIdx.x < kPart) {
    row[threadIdx.x] = t;
    if (prev_jnext && (threadIdx.x == 4 || threadIdx.x == 5)) prev_jnext[threadIdx.x - 4] = t;
  }
}

// One tile of a step: each 64-lane wave takes one strip.
template <int P, bool BUF, bool FORCES, int COLL, bool MOV>
__device__ __forceinline__ void step_tile(const StepArgs& a, int tile,
                                          const int32_t* __restrict__ strip_slot) {
  // Each wave's strip is classified from its coordinates alone (no memory access before
  // the first population load).
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  int x0 = 0, y0 = 0;
  strip_origin(tile, wave, a.ntx, a.tile_rows, x0, y0);
  if (y0 >= a.ny) return;
  const int cls = strip_class(a.nx, a.ny, a.gx0, a.gx1, a.gy0, a.gy1, a.bx0, a.bx1, a.by0,
                              a.by1, x0, y0);
  if (cls != kStripGeneral) {
    if (!strip_is_interior(a.nx, a.ny, x0, y0)) {
      edge_strip<P, BUF, COLL>(a, x0, y0);
      return;
    }
    typename Storage<P>::T v[kQ];
    interior_load<P, BUF>(a, x0, y0, v);
    if (FORCES && cls == kStripBoxRing) {
      // Plain pulls, with the control-volume terms of every node from its coordinates.
      double acc[kPart] = {};
      ring_finish<P, BUF, COLL>(a, x0, y0, v, acc);
      const int slot = strip_slot[tile * kStrips + wave];
      if (slot >= 0) wave_sum_store<kPart>(acc, a.part_out + int64_t(slot) * kPart);
      return;
    }
    if (FORCES && cls == kStripBoxInterior) {
      // Every node is in the control volume and streams plainly: its pre-collision
      // populations are the loaded values; only the box momentum J is accumulated,
      // before collision and after it (of the stored values).
      double acc[kBoxPart] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const double fi = to_f64<P>(v[i], i);
        acc[0] += kCx[i] * fi;
        acc[1] += kCy[i] * fi;
      }
      interior_finish<P, BUF, COLL, true>(a, x0, y0, v, acc + 2);
      wave_sum_store<kBoxPart>(acc, a.part_out + int64_t(a.nslots) * kPart +
                                        int64_t(strip_slot[tile * kStrips + wave]) * kBoxPart);
      return;
    }
    interior_finish<P, BUF, COLL>(a, x0, y0, v);
    return;
  }
  const int slot = FORCES ? strip_slot[tile * kStrips + wave] : -1;
  // FA(x,y), FB(x,y), J(x,y), Phi(x,y), SI(x,y), Jpost(x,y)
  double acc[kPart] = {};
  general_strip<P, BUF, COLL, MOV>(a, x0, y0, slot >= 0, acc);
  if (slot >= 0) wave_sum_store<kPart>(acc, a.part_out + int64_t(slot) * kPart);
}

template <int P, bool BUF, bool FORCES, int COLL, bool MOV>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs a,
                                                        const int32_t* __restrict__ strip_slot) {
  constexpr int kGroup = kStepGroup * 4 / int(sizeof(typename Storage<P>::T));
  int tile = block_tile<kGroup>(blockIdx.x, a.ntiles + (a.red_in ? 1 : 0));
  if (a.red_in) {
    // Block 0 is dispatched first: it reduces the previous step's force partials while
    // the tiles stream.
    if (tile == 0) {
      reduce_row(a.red_in, a.nslots, a.njslots, a.red_row, a.red_prev_jnext);
      return;
    }
    --tile;
  }
  step_tile<P, BUF, FORCES, COLL, MOV>(a, tile, strip_slot);
}

// Batched step: every instance of a batch advances one step in one launch.  The first
// b.nred blocks (when forces are recorded) reduce the previous step's force row, one
// instance each; the other blocks sweep the concatenated tile list of all instances,
// `stride` tiles apart (a persistent sweep when the grid is smaller than the tile count,
// one tile per block otherwise).  nred and a persistent grid are multiples of 8, so the
// tile a block takes lies on the block's own XCD in the grouping of block_tile.
// Step k of a launch sequence writes force row ctl[0] + k; ctl[1] counts the steps of
// the same call enqueued before the sequence (their last row is still to be reduced);
// ctl[2..3] hold the batch's step count at the call, from which the stochastically
// rounded storage takes each member's step number.
__device__ __forceinline__ uint32_t batch_step_key(const BatchLaunch& b, const BatchInst& I,
                                                   int32_t k) {
  const int64_t base = int64_t(uint32_t(b.ctl[2])) | (int64_t(b.ctl[3]) << 32);
  return sr_step_key(base + I.step_off + b.ctl[1] + k);
}
template <int P, bool FORCES, bool PERSIST, int COLL, bool MOV>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(P == LBM_FP64 ? 1 : 7)))
void batch_step_kernel(
    const BatchInst* __restrict__ inst, const int32_t* __restrict__ tile_inst,
    const int32_t* __restrict__ tile_local, BatchLaunch b, int32_t parity, int32_t k) {
  const int nred = FORCES ? b.nred : 0;
  if (int(blockIdx.x) < nred) {
    if (int(blockIdx.x) >= b.n_inst) return;
    const int32_t row_base = b.ctl[0], nprev = b.ctl[1];
    if (k == 0 && nprev == 0) return;
    const BatchInst& I = inst[blockIdx.x];
    const int64_t r = int64_t(row_base) + k - 1;
    const int64_t rs = int64_t(b.n_inst) * kRingRow;  // rows are step-major
    reduce_row(I.part[(k - 1) & 1], I.a.nslots, I.a.njslots, I.ring + r * rs,
               k + nprev >= 2 ? I.ring + (r - 1) * rs + kJnext : nullptr);
    return;
  }
  if (PERSIST && b.queue) {
    // Tile queue: each workgroup takes the next chunk of kQueueChunk consecutive tiles of
    // the list from counter k & 1 (one global atomic per chunk: the counter's atomics
    // are serialised, one per ~13 ns, so a tile each would bound a launch of 50 k tiles
    // at 0.65 ms) until the list is exhausted; the first tile workgroup zeroes the other
    // counter for the next launch (the launch before this one, its last user, has
    // completed).
    __shared__ int32_t next;
    if (int(blockIdx.x) == nred && threadIdx.x == 0) b.queue[(k + 1) & 1] = 0;
    for (;;) {
      if (threadIdx.x == 0) next = atomicAdd(&b.queue[k & 1], 1);
      __syncthreads();
      const int t0 = next * kQueueChunk;
      __syncthreads();
      if (t0 >= b.total_tiles) return;
      const int t1 = min(t0 + kQueueChunk, b.total_tiles);
      for (int t = t0; t < t1; ++t) {
        const BatchInst& I = inst[tile_inst[t]];
        StepArgs a = I.a;
        a.src = I.buf[parity];
        a.dst = I.buf[1 - parity];
        a.part_out = I.part[k & 1];
        if constexpr (Storage<P>::kSR) a.step_key = batch_step_key(b, I, k);
        step_tile<P, true, FORCES, COLL, MOV>(a, tile_local[t], a.strip_slot);
      }
    }
  }
  const int stride = PERSIST ? int(gridDim.x) - nred : b.total_tiles;
  for (int v = int(blockIdx.x) - nred; v < b.total_tiles; v += stride) {
    const int t = block_tile<kBatchGroup>(v, b.total_tiles);
    const BatchInst& I = inst[tile_inst[t]];
    StepArgs a = I.a;
    a.src = I.buf[parity];
    a.dst = I.buf[1 - parity];
    a.part_out = I.part[k & 1];
    if constexpr (Storage<P>::kSR) a.step_key = batch_step_key(b, I, k);
    step_tile<P, true, FORCES, COLL, MOV>(a, tile_local[t], a.strip_slot);
  }
}

__global__ void batch_ctl_kernel(int32_t* ctl, int32_t row_base, int32_t nprev, int64_t base) {
  if (threadIdx.x == 0) {
    ctl[0] = row_base;
    ctl[1] = nprev;
    ctl[2] = int32_t(uint32_t(uint64_t(base)));
    ctl[3] = int32_t(uint32_t(uint64_t(base) >> 32));
  }
}

// J over the control volume of the populations one pull of src gives: block `blk` of
// the box sweep (kTileW nodes of one box row) writes its two partial sums.
template <int P, bool BUF>
__device__ __forceinline__ void box_block(const BoxArgs& a, int blk) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const int row = blk / a.box_bx;
  const int x = a.bx0 + (blk - row * a.box_bx) * kTileW + int(threadIdx.x);
  const int y = a.by0 + row;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (x < a.bx1) {
    const uint32_t w = a.node[int64_t(y) * a.nx + x];
    if (!(w & kSolidBit)) {
      C f[kQ];
      pull_all<P>(src, a.pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, f, a.motion);
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const double fi = pre_f64<P>(f[i], i);
        v[0] += kCx[i] * fi;
        v[1] += kCy[i] * fi;
      }
    }
  }
  __shared__ double out[8];
  block_sum8(v, out);
  if (threadIdx.x < 2) a.jpart[int64_t(blk) * 2 + threadIdx.x] = out[threadIdx.x];
}

template <int P, bool BUF>
__global__ __launch_bounds__(kThreads) void box_momentum_kernel(BoxArgs a) {
  box_block<P, BUF>(a, blockIdx.x);
}

// Box sweeps of all instances of a batch (block b -> instance box_inst[b]).
template <int P>
__global__ __launch_bounds__(kThreads) void batch_box_kernel(BatchLaunch b, int32_t parity) {
  const BatchInst& I = b.inst[b.box_inst[blockIdx.x]];
  BoxArgs x = I.box;
  x.src = I.buf[parity];
  box_block<P, true>(x, b.box_local[blockIdx.x]);
}

__device__ __forceinline__ void finalize_body(const FinalArgs& a) {
  reduce_row(a.red_in, a.nslots, a.njslots, a.row, a.prev_jnext);
  if (a.jpart) {
    __syncthreads();
    __shared__ double red[kThreads][2];
    double jx = 0.0, jy = 0.0;
    for (int j = threadIdx.x; j < a.njblocks; j += kThreads) {
      jx += a.jpart[2 * int64_t(j)];
      jy += a.jpart[2 * int64_t(j) + 1];
    }
    red[threadIdx.x][0] = jx;
    red[threadIdx.x][1] = jy;
    __syncthreads();
    if (threadIdx.x < 2) {
      double s = 0.0;
      for (int k = 0; k < kThreads; ++k) s += red[k][threadIdx.x];
      a.row[kJnext + threadIdx.x] = s;
    }
  } else if (threadIdx.x < 2) {
    a.row[kJnext + threadIdx.x] = __builtin_nan("");
  }
}

__global__ __launch_bounds__(kThreads) void finalize_kernel(FinalArgs a) { finalize_body(a); }

// Finalize of every instance of a batch (one block each): force row `row` from the
// partials part[part_parity] and, without a box, NaN for its Jnext.
__global__ __launch_bounds__(kThreads) void batch_finalize_kernel(BatchLaunch b, int32_t row,
                                                                  int32_t part_parity,
                                                                  int32_t has_prev) {
  const BatchInst& I = b.inst[blockIdx.x];
  FinalArgs f{};
  f.red_in = I.part[part_parity];
  f.nslots = I.a.nslots;
  f.njslots = I.a.njslots;
  const int64_t rs = int64_t(b.n_inst) * kRingRow;  // rows are step-major
  f.row = I.ring + int64_t(row) * rs;
  f.prev_jnext = has_prev ? I.ring + (int64_t(row) - 1) * rs + kJnext : nullptr;
  f.jpart = I.njblocks > 0 ? I.box.jpart : nullptr;
  f.njblocks = I.njblocks;
  finalize_body(f);
}

template <int P>
__global__ __launch_bounds__(kThreads) void fill_rest_kernel(void* buf, int64_t n,
                                                               int64_t plane) {
  using S = Storage<P>;
  using T = typename S::T;
  T* p = static_cast<T*>(buf);
  // Both layouts repeat the nine directions every 9 * plane elements.
  const int64_t period = plane * kQ;
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * kThreads) {
    const int i = int((k % period) / plane);
    p[k] = (S::kDev && !S::kStoreF) ? T(0) : T(weight<typename S::C>(i));
  }
}

// Mask change: one thread per listed node.  A covered node contributes its momentum; an
// uncovered one is refilled with f^eq(rho, u_w), rho the mean density of its lattice
// neighbours that are fluid in both masks (periodic edges wrap, other edges do not
// count; rho_w when none is) and u_w the rigid-body velocity at the node, and
// contributes minus the momentum it now stores.  Refills read valid neighbours only, so
// no thread reads what another writes.
template <int P>
__global__ __launch_bounds__(kThreads) void remask_kernel(RemaskArgs a) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  T* st = static_cast<T*>(a.state);
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < a.n;
       k += int64_t(gridDim.x) * kThreads) {
    const uint32_t e = uint32_t(a.list[k]);
    const int32_t node = int32_t(e & 0x7fffffffu);
    const int y = node / a.nx, x = node - y * a.nx;
    const int64_t at = int64_t(y) * a.pitch + x;
    if (!(e >> 31)) {
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        const double f = to_f64<P>(st[i * a.plane + at], i);
        v[0] += kCx[i] * f;
        v[1] += kCy[i] * f;
      }
      continue;
    }
    double rsum = 0.0;
    int cnt = 0;
    for (int i = 1; i < kQ; ++i) {
      int ax = x + kCx[i], ay = y + kCy[i];
      if (a.bc_x == LBM_BCX_PERIODIC) ax = (ax + a.nx) % a.nx;
      if (a.bc_y == LBM_BCY_PERIODIC) ay = (ay + a.ny) % a.ny;
      if (ax < 0 || ax >= a.nx || ay < 0 || ay >= a.ny || !a.valid[int64_t(ay) * a.nx + ax])
        continue;
      const int64_t nb = int64_t(ay) * a.pitch + ax;
      double r = 0.0;
      for (int j = 0; j < kQ; ++j) r += to_f64<P>(st[j * a.plane + nb], j);
      rsum += r;
      ++cnt;
    }
    const double rho = cnt > 0 ? rsum / double(cnt) : a.rho_w;
    const double ux = a.motion.ux - a.motion.omega * (double(y) - a.motion.yc);
    const double uy = a.motion.uy + a.motion.omega * (double(x) - a.motion.xc);
    const double uu = ux * ux + uy * uy;
    for (int i = 0; i < kQ; ++i) {
      const double cu = kCx[i] * ux + kCy[i] * uy;
      const double feq = weight<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      const T q = S::kStoreF ? T(feq) : pack<P>(C(feq - weight<double>(i)), i);
      st[i * a.plane + at] = q;
      const double f = to_f64<P>(q, i);
      v[0] -= kCx[i] * f;
      v[1] -= kCy[i] * f;
    }
  }
  __shared__ double out[8];
  block_sum8(v, out);
  __syncthreads();
  if (threadIdx.x < 2) a.block_out[2 * blockIdx.x + threadIdx.x] = out[threadIdx.x];
}

// Sum of the per-block momenta in a fixed order (one block).
__global__ __launch_bounds__(kThreads) void remask_sum_kernel(const double* block_out, int nb,
                                                              double* res) {
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    v[0] += block_out[2 * b];
    v[1] += block_out[2 * b + 1];
  }
  __shared__ double out[8];
  block_sum8(v, out);
  __syncthreads();
  if (threadIdx.x < 2) res[threadIdx.x] = out[threadIdx.x];
}

// Boundary pressure coefficient (Sec. V, the C_p equation: over the boundary fluid
// nodes, no extrapolation), one thread per listed node: p = rho theta0 with rho the sum
// of the stored populations (binary64), p_inf the same at the reference node.
template <int P>
__global__ __launch_bounds__(kThreads) void boundary_cp_kernel(CpArgs a) {
  using T = typename Storage<P>::T;
  const T* st = static_cast<const T*>(a.state);
  auto density = [&](int32_t node) {
    const int y = node / a.nx, x = node - y * a.nx;
    const int64_t at = int64_t(y) * a.pitch + x;
    double rho = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) rho += to_f64<P>(st[i * a.plane + at], i);
    return rho;
  };
  const int k = int(blockIdx.x) * kThreads + int(threadIdx.x);
  if (k >= a.n) return;
  const double p_inf = a.ref_node >= 0 ? density(a.ref_node) * (1.0 / 3.0) : a.p_ref;
  a.out[k] = (density(a.nodes[k]) * (1.0 / 3.0) - p_inf) / a.q;
}

template <int P, bool BUF, int COLL>
hipError_t step_dispatch3(bool forces, const StepArgs& a, hipStream_t s) {
  const dim3 grid(a.ntiles + (a.red_in ? 1 : 0));
  // Bodies in motion take their own instantiation, so the moving-wall arithmetic costs
  // the resting case no registers.
  if (forces) {
    if (a.motion)
      hipLaunchKernelGGL((step_kernel<P, BUF, true, COLL, true>), grid, dim3(kThreads), 0, s, a,
                         a.strip_slot);
    else
      hipLaunchKernelGGL((step_kernel<P, BUF, true, COLL, false>), grid, dim3(kThreads), 0, s, a,
                         a.strip_slot);
  } else {
    if (a.motion)
      hipLaunchKernelGGL((step_kernel<P, BUF, false, COLL, true>), grid, dim3(kThreads), 0, s, a,
                         a.strip_slot);
    else
      hipLaunchKernelGGL((step_kernel<P, BUF, false, COLL, false>), grid, dim3(kThreads), 0, s,
                         a, a.strip_slot);
  }
  return hipGetLastError();
}

template <int P, bool BUF>
hipError_t step_dispatch2(bool forces, const StepArgs& a, hipStream_t s) {
  switch (a.collision) {
    case LBM_COLL_REGULARIZED: return step_dispatch3<P, BUF, LBM_COLL_REGULARIZED>(forces, a, s);
    case LBM_COLL_KBC: return step_dispatch3<P, BUF, LBM_COLL_KBC>(forces, a, s);
    default: return step_dispatch3<P, BUF, LBM_COLL_BGK>(forces, a, s);
  }
}

template <int P>
hipError_t step_dispatch(bool forces, const StepArgs& a, hipStream_t s) {
  return a.buf_bytes ? step_dispatch2<P, true>(forces, a, s) : step_dispatch2<P, false>(forces, a, s);
}

template <int P>
hipError_t box_dispatch(const BoxArgs& a, int blocks, hipStream_t s) {
  if (a.buf_bytes)
    hipLaunchKernelGGL((box_momentum_kernel<P, true>), dim3(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((box_momentum_kernel<P, false>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int precision, bool forces, const StepArgs& a, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: return step_dispatch<LBM_FP64>(forces, a, s);
    case LBM_FP32: return step_dispatch<LBM_FP32>(forces, a, s);
    case LBM_FP32DEV: return step_dispatch<LBM_FP32DEV>(forces, a, s);
    case LBM_FP32SR: return step_dispatch<LBM_FP32SR>(forces, a, s);
    case LBM_FP16DEV: return step_dispatch<LBM_FP16DEV>(forces, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_box_momentum(int precision, const BoxArgs& a, int blocks, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: return box_dispatch<LBM_FP64>(a, blocks, s);
    case LBM_FP32: return box_dispatch<LBM_FP32>(a, blocks, s);
    case LBM_FP32DEV: return box_dispatch<LBM_FP32DEV>(a, blocks, s);
    case LBM_FP32SR: return box_dispatch<LBM_FP32SR>(a, blocks, s);
    case LBM_FP16DEV: return box_dispatch<LBM_FP16DEV>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_step(int precision, bool forces, const BatchLaunch& b, int32_t parity,
                             int32_t k, hipStream_t s) {
  const bool persist = b.grid_blocks > 0 && b.grid_blocks < b.total_tiles;
  const int tiles = persist ? b.grid_blocks : b.total_tiles;
  const dim3 grid((forces ? b.nred : 0) + tiles);
#define LBM_BATCH_GO4(P, F, R, K, M) \
  hipLaunchKernelGGL((batch_step_kernel<P, F, R, K, M>), grid, dim3(kThreads), 0, s, b.inst, \
                     b.tile_inst, b.tile_local, b, parity, k)
#define LBM_BATCH_GO3(P, F, R, K)                        \
  do {                                                   \
    if (b.moving) LBM_BATCH_GO4(P, F, R, K, true);       \
    else LBM_BATCH_GO4(P, F, R, K, false);               \
  } while (0)
#define LBM_BATCH_GO(P, F, R)                                                         \
  do {                                                                                \
    if (b.collision == LBM_COLL_REGULARIZED) LBM_BATCH_GO3(P, F, R, LBM_COLL_REGULARIZED); \
    else if (b.collision == LBM_COLL_KBC) LBM_BATCH_GO3(P, F, R, LBM_COLL_KBC);      \
    else LBM_BATCH_GO3(P, F, R, LBM_COLL_BGK);                                        \
  } while (0)
#define LBM_BATCH_LAUNCH(P)                                          \
  if (forces) {                                                      \
    if (persist) LBM_BATCH_GO(P, true, true); else LBM_BATCH_GO(P, true, false);   \
  } else {                                                           \
    if (persist) LBM_BATCH_GO(P, false, true); else LBM_BATCH_GO(P, false, false); \
  }
  switch (precision) {
    case LBM_FP64: LBM_BATCH_LAUNCH(LBM_FP64) break;
    case LBM_FP32: LBM_BATCH_LAUNCH(LBM_FP32) break;
    case LBM_FP32DEV: LBM_BATCH_LAUNCH(LBM_FP32DEV) break;
    case LBM_FP32SR: LBM_BATCH_LAUNCH(LBM_FP32SR) break;
    case LBM_FP16DEV: LBM_BATCH_LAUNCH(LBM_FP16DEV) break;
    default: return hipErrorInvalidValue;
  }
#undef LBM_BATCH_LAUNCH
#undef LBM_BATCH_GO
#undef LBM_BATCH_GO3
#undef LBM_BATCH_GO4
  return hipGetLastError();
}

__global__ void batch_queue_reset_kernel(int32_t* queue) {
  if (threadIdx.x < 2) queue[threadIdx.x] = 0;
}

hipError_t launch_batch_queue_reset(int32_t* queue, hipStream_t s) {
  hipLaunchKernelGGL(batch_queue_reset_kernel, dim3(1), dim3(64), 0, s, queue);
  return hipGetLastError();
}

hipError_t launch_batch_ctl(int32_t* ctl, int32_t row_base, int32_t nprev, int64_t base,
                            hipStream_t s) {
  hipLaunchKernelGGL(batch_ctl_kernel, dim3(1), dim3(64), 0, s, ctl, row_base, nprev, base);
  return hipGetLastError();
}

hipError_t launch_batch_tail(int precision, const BatchLaunch& b, int32_t parity, int32_t row,
                             int32_t part_parity, bool has_prev, hipStream_t s) {
  if (b.total_box_blocks > 0) {
    const dim3 grid(b.total_box_blocks);
    switch (precision) {
      case LBM_FP64:
        hipLaunchKernelGGL(batch_box_kernel<LBM_FP64>, grid, dim3(kThreads), 0, s, b, parity);
        break;
      case LBM_FP32:
        hipLaunchKernelGGL(batch_box_kernel<LBM_FP32>, grid, dim3(kThreads), 0, s, b, parity);
        break;
      case LBM_FP32DEV:
        hipLaunchKernelGGL(batch_box_kernel<LBM_FP32DEV>, grid, dim3(kThreads), 0, s, b, parity);
        break;
      case LBM_FP32SR:
        hipLaunchKernelGGL(batch_box_kernel<LBM_FP32SR>, grid, dim3(kThreads), 0, s, b, parity);
        break;
      case LBM_FP16DEV:
        hipLaunchKernelGGL(batch_box_kernel<LBM_FP16DEV>, grid, dim3(kThreads), 0, s, b, parity);
        break;
      default:
        return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(b.n_inst), dim3(kThreads), 0, s, b, row,
                     part_parity, int32_t(has_prev ? 1 : 0));
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_remask(int precision, const RemaskArgs& a, int blocks, double* out,
                         hipStream_t s) {
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(remask_kernel<LBM_FP64>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(remask_kernel<LBM_FP32>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32DEV:
      hipLaunchKernelGGL(remask_kernel<LBM_FP32DEV>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32SR:
      hipLaunchKernelGGL(remask_kernel<LBM_FP32SR>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP16DEV:
      hipLaunchKernelGGL(remask_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(remask_sum_kernel, dim3(1), dim3(kThreads), 0, s,
                     static_cast<const double*>(a.block_out), blocks, out);
  return hipGetLastError();
}

hipError_t launch_boundary_cp(int precision, const CpArgs& a, hipStream_t s) {
  const dim3 grid((a.n + kThreads - 1) / kThreads);
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(boundary_cp_kernel<LBM_FP64>, grid, dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(boundary_cp_kernel<LBM_FP32>, grid, dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32DEV:
      hipLaunchKernelGGL(boundary_cp_kernel<LBM_FP32DEV>, grid, dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32SR:
      hipLaunchKernelGGL(boundary_cp_kernel<LBM_FP32SR>, grid, dim3(kThreads), 0, s, a);
      break;
    case LBM_FP16DEV:
      hipLaunchKernelGGL(boundary_cp_kernel<LBM_FP16DEV>, grid, dim3(kThreads), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_rest(int precision, void* buf, int64_t n, int64_t plane, hipStream_t s) {
  const int blocks = 2048;
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP64>, dim3(blocks), dim3(kThreads), 0, s, buf, n, plane);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP32>, dim3(blocks), dim3(kThreads), 0, s, buf, n, plane);
      break;
    case LBM_FP32DEV:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP32DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, n, plane);
      break;
    case LBM_FP32SR:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP32SR>, dim3(blocks), dim3(kThreads), 0, s, buf, n, plane);
      break;
    case LBM_FP16DEV:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, n, plane);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbm
