// HIP kernels for gfx950: the fused D2Q9 pull-stream + BGK collision step with the
// per-step momentum-exchange (algorithms A and B) and DRTT force sums.
//
// Kaushal, Succi & Ansumali, arXiv:2210.10377: Eq. CollideAdv (collide, then stream),
// the second-order equilibrium and Table I (Sec. II), stationary and moving-wall
// bounce-back (Sec. II), the momentum exchange of Sec. III with the two operator
// orders of Eq. rtt4, and the control-volume balance of the second Eq. rtt7.
//
// Data layout (HBM): structure of arrays, one plane per direction, x fastest; plane
// stride and row pitch come from the host.  Every node is updated by one thread of a
// 256-thread block; a block covers a 256 x kTileH tile, each wave a 64 x kTileH strip.
// Strips of plain fluid (all pulls plain streaming, away from the control-volume band)
// take a branch-free path that reads no per-node metadata; the other strips read a
// 32-bit word of pull codes per node, apply the boundary rules, and accumulate the
// force sums in FP64.  Waves never wait for each other: a strip with force terms
// reduces them over the wave and writes one partial slot; the slots are reduced in a
// fixed order by one extra block (dispatched first) of the next step's launch, or by
// the finalize kernel, so every force is deterministic.
//
// Addressing: when a state buffer is below 4 GiB its populations are read and written
// through buffer resources (one descriptor per buffer, the plane offsets in scalar
// registers, 32-bit per-lane offsets); out-of-range offsets read zero and drop writes.
// Larger buffers use 64-bit global addresses.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace lbm {

namespace {

using namespace dev;

__device__ __forceinline__ bool in_box(const StepArgs& a, int x, int y) {
  return x >= a.bx0 && x < a.bx1 && y >= a.by0 && y < a.by1;
}

// Interior tile: plain pull streaming in every direction, no metadata.  All rows of
// the tile are loaded before any is collided, so each lane keeps 9 * kTileH loads in
// flight.
template <int P, bool BUF>
__device__ __forceinline__ void interior_load(const StepArgs& a, int tx, int ty,
                                              typename Storage<P>::T (&v)[kTileH][kQ]) {
  using T = typename Storage<P>::T;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const int pitch = a.pitch;
  const int32_t o0 = (ty * kTileH) * pitch + tx * kTileW + int(threadIdx.x);
#pragma unroll
  for (int r = 0; r < kTileH; ++r)
#pragma unroll
    for (int i = 0; i < kQ; ++i) v[r][i] = src.ld(i, o0 + (r - kCy[i]) * pitch - kCx[i]);
}

template <int P, bool BUF>
__device__ __forceinline__ void interior_finish(const StepArgs& a, int tx, int ty,
                                                const typename Storage<P>::T (&v)[kTileH][kQ]) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> dst(a.dst, a.plane, a.buf_bytes);
  const int pitch = a.pitch;
  const int32_t o0 = (ty * kTileH) * pitch + tx * kTileW + int(threadIdx.x);
#pragma unroll
  for (int r = 0; r < kTileH; ++r) {
    C f[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) f[i] = unpack<P>(v[r][i]);
    C g[kQ];
    collide<C, S::kDev>(f, C(a.omega), g);
#pragma unroll
    for (int i = 0; i < kQ; ++i) dst.st(i, o0 + r * pitch, pack<P>(g[i]));
  }
}

// General path of one lane's column of the tile: boundary rules from the pull codes,
// and (when `forces`) the force sums of its nodes added to acc.
template <int P, bool BUF>
__device__ __forceinline__ void general_rows(const StepArgs& a, int tx, int ty, bool forces,
                                             double (&acc)[8]) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const Planes<T, BUF> dst(a.dst, a.plane, a.buf_bytes);
  const int pitch = a.pitch;
  const int x = tx * kTileW + int(threadIdx.x);
  for (int r = 0; r < kTileH; ++r) {
    const int y = ty * kTileH + r;
    if (x >= a.nx || y >= a.ny) continue;
    const uint32_t w = a.node[int64_t(y) * a.nx + x];
    if (w & kSolidBit) continue;
    const int32_t o = y * pitch + x;
    C f[kQ];
    pull_all<P>(src, pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, f);
    C g[kQ];
    collide<C, S::kDev>(f, C(a.omega), g);
    T s[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      s[i] = pack<P>(g[i]);
      dst.st(i, o, s[i]);
    }
    if (forces) {
      // Momentum exchange on the links of this node (Sec. III; Eq. rtt4): the
      // population leaving along c_i towards the body is f_i before collision (A) or
      // f~_i after it (B); the body returns f~_i (as stored) along -c_i.
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        if (pull_code(w, kOpp[i]) != kBody) continue;
        const double sv = to_f64<P>(s[i], i);
        const double fa = (S::kDev ? weight<double>(i) + double(f[i]) : double(f[i])) + sv;
        acc[0] += kCx[i] * fa;
        acc[1] += kCy[i] * fa;
        acc[2] += kCx[i] * (sv + sv);
        acc[3] += kCy[i] * (sv + sv);
      }
      // Control volume (second Eq. rtt7): momentum before collision, and the
      // populations crossing the box surface after collision.
      if (in_box(a, x, y)) {
        double jx = 0.0, jy = 0.0;
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
          const double fi = S::kDev ? weight<double>(i) + double(f[i]) : double(f[i]);
          jx += kCx[i] * fi;
          jy += kCy[i] * fi;
        }
        acc[4] += jx;
        acc[5] += jy;
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
  }
}

template <int P, bool BUF, bool FORCES>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs a,
                                                        const int32_t* __restrict__ strip_slot) {
  int tile = block_tile(blockIdx.x, a.ntiles + (a.red_in ? 1 : 0));
  if (a.red_in) {
    // Block 0 is dispatched first: it reduces the previous step's force partials while
    // the tiles stream.
    if (tile == 0) {
      const double t = reduce_partials8(a.red_in, a.nslots);
      if (threadIdx.x < 8) {
        a.red_row[threadIdx.x] = t;
        if (a.red_prev_jnext && (threadIdx.x == 4 || threadIdx.x == 5))
          a.red_prev_jnext[threadIdx.x - 4] = t;
      }
      return;
    }
    --tile;
  }
  const int ty = tile / a.ntx, tx = tile - ty * a.ntx;
  // Each 64-lane wave covers a 64 x kTileH strip, classified from its coordinates
  // alone (no memory access before the first population load).
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  if (strip_is_plain(a.nx, a.ny, a.gx0, a.gx1, a.gy0, a.gy1, tx * kTileW + 64 * wave,
                     ty * kTileH)) {
    typename Storage<P>::T v[kTileH][kQ];
    interior_load<P, BUF>(a, tx, ty, v);
    interior_finish<P, BUF>(a, tx, ty, v);
    return;
  }
  const int slot = FORCES ? strip_slot[tile * (kTileW / 64) + wave] : -1;
  // FA(x,y), FB(x,y), J(x,y), Phi(x,y)
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  general_rows<P, BUF>(a, tx, ty, slot >= 0, acc);
  if (slot >= 0) wave_sum8_store(acc, a.part_out + int64_t(slot) * 8);
}

// J over the control volume of the populations one pull of src gives.
template <int P, bool BUF>
__global__ __launch_bounds__(kThreads) void box_momentum_kernel(BoxArgs a) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Planes<T, BUF> src(a.src, a.plane, a.buf_bytes);
  const int row = blockIdx.x / a.box_bx;
  const int x = a.bx0 + (blockIdx.x - row * a.box_bx) * kTileW + int(threadIdx.x);
  const int y = a.by0 + row;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (x < a.bx1) {
    const uint32_t w = a.node[int64_t(y) * a.nx + x];
    if (!(w & kSolidBit)) {
      C f[kQ];
      pull_all<P>(src, a.pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, f);
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const double fi = S::kDev ? weight<double>(i) + double(f[i]) : double(f[i]);
        v[0] += kCx[i] * fi;
        v[1] += kCy[i] * fi;
      }
    }
  }
  __shared__ double out[8];
  block_sum8(v, out);
  if (threadIdx.x < 2) a.jpart[int64_t(blockIdx.x) * 2 + threadIdx.x] = out[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void finalize_kernel(FinalArgs a) {
  const double t = reduce_partials8(a.red_in, a.nslots);
  if (threadIdx.x < 8) {
    a.row[threadIdx.x] = t;
    if (a.prev_jnext && (threadIdx.x == 4 || threadIdx.x == 5)) a.prev_jnext[threadIdx.x - 4] = t;
  }
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
      a.row[8 + threadIdx.x] = s;
    }
  } else if (threadIdx.x < 2) {
    a.row[8 + threadIdx.x] = __builtin_nan("");
  }
}

template <int P>
__global__ __launch_bounds__(kThreads) void fill_rest_kernel(void* buf, int64_t plane) {
  using S = Storage<P>;
  using T = typename S::T;
  T* p = static_cast<T*>(buf);
  const int64_t n = plane * kQ;
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * kThreads) {
    const int i = int(k / plane);
    p[k] = S::kDev ? T(0) : T(weight<typename S::C>(i));
  }
}

template <int P, bool BUF>
hipError_t step_dispatch2(bool forces, const StepArgs& a, hipStream_t s) {
  const int grid = a.ntiles + (a.red_in ? 1 : 0);
  if (forces)
    hipLaunchKernelGGL((step_kernel<P, BUF, true>), dim3(grid), dim3(kThreads), 0, s, a, a.strip_slot);
  else
    hipLaunchKernelGGL((step_kernel<P, BUF, false>), dim3(grid), dim3(kThreads), 0, s, a, a.strip_slot);
  return hipGetLastError();
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
    default: return step_dispatch<LBM_FP16DEV>(forces, a, s);
  }
}

hipError_t launch_box_momentum(int precision, const BoxArgs& a, int blocks, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: return box_dispatch<LBM_FP64>(a, blocks, s);
    case LBM_FP32: return box_dispatch<LBM_FP32>(a, blocks, s);
    case LBM_FP32DEV: return box_dispatch<LBM_FP32DEV>(a, blocks, s);
    default: return box_dispatch<LBM_FP16DEV>(a, blocks, s);
  }
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_rest(int precision, void* buf, int64_t plane, hipStream_t s) {
  const int blocks = 2048;
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP64>, dim3(blocks), dim3(kThreads), 0, s, buf, plane);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP32>, dim3(blocks), dim3(kThreads), 0, s, buf, plane);
      break;
    case LBM_FP32DEV:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP32DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, plane);
      break;
    default:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, plane);
  }
  return hipGetLastError();
}

}  // namespace lbm
