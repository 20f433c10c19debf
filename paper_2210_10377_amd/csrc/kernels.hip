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
// 256-thread block; a block covers a 256 x kTileH tile.  Interior tiles (all fluid,
// all pulls plain streaming, away from the control-volume band) take a branch-free
// path that reads no per-node metadata; the other tiles read a 32-bit word of pull
// codes per node, apply the boundary rules, and accumulate the force sums in FP64.
// Force partial sums go to one slot per general tile and are reduced in a fixed order
// by one extra block of the next step's launch (or by the finalize kernel), so every
// force is deterministic.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "plan.h"

namespace lbm {

namespace {

constexpr int kThreads = kTileW;

template <class C>
__device__ __forceinline__ constexpr C weight(int i) {
  return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

// Storage of a population and the arithmetic type it is computed in.
template <int P>
struct Storage;

template <>
struct Storage<LBM_FP64> {
  using T = double;
  using C = double;
  static __device__ __forceinline__ C unpack(T v, int) { return v; }
  static __device__ __forceinline__ T pack(C v, int) { return v; }
};

template <>
struct Storage<LBM_FP32> {
  using T = float;
  using C = float;
  static __device__ __forceinline__ C unpack(T v, int) { return v; }
  static __device__ __forceinline__ T pack(C v, int) { return v; }
};

// Deviation from the lattice weight stored in binary16 (round to nearest even);
// arithmetic in binary32.
template <>
struct Storage<LBM_FP16DEV> {
  using T = _Float16;
  using C = float;
  static __device__ __forceinline__ C unpack(T v, int i) { return weight<float>(i) + float(v); }
  static __device__ __forceinline__ T pack(C v, int i) { return T(v - weight<float>(i)); }
};

// BGK collision of one node (Eq. CollideAdv, first line, with 2 beta = omega) towards
// the second-order equilibrium w_i rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2].
template <class C>
__device__ __forceinline__ void collide(const C (&f)[kQ], C omega, C (&g)[kQ]) {
  const C rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const C jx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const C jy = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const C ir = C(1) / rho;
  const C ux = jx * ir, uy = jy * ir;
  const C usq = C(1.5) * (ux * ux + uy * uy);
  const C om = omega;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const C cu = C(kCx[i]) * ux + C(kCy[i]) * uy;
    const C feq = weight<C>(i) * rho * (C(1) + C(3) * cu + C(4.5) * cu * cu - usq);
    g[i] = f[i] + om * (feq - f[i]);
  }
}

template <class T>
__device__ __forceinline__ void store_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Block index -> tile index such that each XCD (blocks are dealt round-robin over the
// 8 XCDs) walks a contiguous run of row-major tiles, so the neighbouring tiles that
// share cache lines of the +-1-shifted pulls sit in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int xcd = b & 7, k = b >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + k;
}

__device__ __forceinline__ bool in_box(const StepArgs& a, int x, int y) {
  return x >= a.bx0 && x < a.bx1 && y >= a.by0 && y < a.by1;
}

// Interior tile: plain pull streaming in every direction, no metadata.
template <int P>
__device__ __forceinline__ void interior_tile(const StepArgs& a, int tx, int ty) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const int64_t pl = a.plane;
  const int pitch = a.pitch;
  const int x = tx * kTileW + int(threadIdx.x);
#pragma unroll
  for (int r = 0; r < kTileH; ++r) {
    const int y = ty * kTileH + r;
    const int64_t o = int64_t(y) * pitch + x;
    C f[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      f[i] = S::unpack(src[i * pl + o - int64_t(kCy[i]) * pitch - kCx[i]], i);
    C g[kQ];
    collide<C>(f, C(a.omega), g);
#pragma unroll
    for (int i = 0; i < kQ; ++i) store_nt(dst + i * pl + o, S::pack(g[i], i));
  }
}

// Population of direction i arriving at fluid node (x, y), by its pull code.
template <int P>
__device__ __forceinline__ typename Storage<P>::C pull(const typename Storage<P>::T* __restrict__ src,
                                                       int64_t pl, int pitch, int nx, int ny,
                                                       const double* uin, double rho_w6,
                                                       uint32_t w, int x, int y, int i) {
  using S = Storage<P>;
  using C = typename S::C;
  const int o = kOpp[i];
  const int64_t own = int64_t(y) * pitch + x;
  switch (pull_code(w, i)) {
    case kStream:
      return S::unpack(src[i * pl + own - int64_t(kCy[i]) * pitch - kCx[i]], i);
    case kInlet:
      // Moving-wall bounce-back (Sec. II) with u_w = (u_in(y), 0):
      // f_i = f~_o + 2 w_i rho_w (c_i . u_w) / c_s^2.
      return S::unpack(src[o * pl + own], o) +
             C(rho_w6 * uin[y]) * (weight<C>(i) * C(kCx[i]));
    case kOutlet: {
      int sy = y - kCy[i];
      sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
      return S::unpack(src[i * pl + int64_t(sy) * pitch + (nx - 1)], i);
    }
    case kWrap: {
      int sx = x - kCx[i], sy = y - kCy[i];
      sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
      sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
      return S::unpack(src[i * pl + int64_t(sy) * pitch + sx], i);
    }
    default:  // kBody, kWall: half-way bounce-back
      return S::unpack(src[o * pl + own], o);
  }
}

// Sum 8 doubles over the block in a fixed order; thread k < 8 writes out[k].
__device__ __forceinline__ void block_sum8(double (&v)[8], double* out) {
  __shared__ double red[kThreads / 64][8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    double s = red[0][threadIdx.x];
#pragma unroll
    for (int wv = 1; wv < kThreads / 64; ++wv) s += red[wv][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// General tile: boundary rules from the pull codes, and the force sums.
template <int P, bool FORCES>
__device__ __forceinline__ void general_tile(const StepArgs& a, int tx, int ty, int slot) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const int64_t pl = a.plane;
  const int pitch = a.pitch;
  const int x = tx * kTileW + int(threadIdx.x);
  // FA(x,y), FB(x,y), J(x,y), Phi(x,y)
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = 0; r < kTileH; ++r) {
    const int y = ty * kTileH + r;
    if (x >= a.nx || y >= a.ny) continue;
    const uint32_t w = a.node[int64_t(y) * a.nx + x];
    if (w & kSolidBit) continue;
    const int64_t o = int64_t(y) * pitch + x;
    C f[kQ];
    f[0] = S::unpack(src[o], 0);
#pragma unroll
    for (int i = 1; i < kQ; ++i) f[i] = pull<P>(src, pl, pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, i);
    C g[kQ];
    collide<C>(f, C(a.omega), g);
    T s[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      s[i] = S::pack(g[i], i);
      store_nt(dst + i * pl + o, s[i]);
    }
    if (FORCES) {
      // Momentum exchange on the links of this node (Sec. III; Eq. rtt4): the
      // population leaving along c_i towards the body is f_i before collision (A) or
      // f~_i after it (B); the body returns f~_i (as stored) along -c_i.
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        if (pull_code(w, kOpp[i]) != kBody) continue;
        const double sv = double(S::unpack(s[i], i));
        const double fa = double(f[i]) + sv;
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
          jx += kCx[i] * double(f[i]);
          jy += kCy[i] * double(f[i]);
        }
        acc[4] += jx;
        acc[5] += jy;
#pragma unroll
        for (int i = 1; i < kQ; ++i)
          if (!in_box(a, x + kCx[i], y + kCy[i])) {
            const double sv = double(S::unpack(s[i], i));
            acc[6] -= kCx[i] * sv;
            acc[7] -= kCy[i] * sv;
          }
      } else {
#pragma unroll
        for (int i = 1; i < kQ; ++i)
          if (in_box(a, x + kCx[i], y + kCy[i])) {
            const double sv = double(S::unpack(s[i], i));
            acc[6] += kCx[i] * sv;
            acc[7] += kCy[i] * sv;
          }
      }
    }
  }
  if (FORCES) block_sum8(acc, a.part_out + int64_t(slot) * 8);
}

// Fixed-order reduction of [nslots][8] partials by one 256-thread block; returns the
// eight sums in threads 0..7.
__device__ __forceinline__ double reduce_partials8(const double* in, int nslots) {
  __shared__ double red[kThreads / 8][8];
  const int k = threadIdx.x & 7, grp = threadIdx.x >> 3;
  double s = 0.0;
  for (int j = grp; j < nslots; j += kThreads / 8) s += in[int64_t(j) * 8 + k];
  red[grp][k] = s;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < 8)
    for (int gI = 0; gI < kThreads / 8; ++gI) t += red[gI][threadIdx.x];
  return t;
}

template <int P, bool FORCES>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs a) {
  const int b = blockIdx.x;
  if (b >= a.ntiles) {
    // Reducer block: force row of the previous step.
    const double t = reduce_partials8(a.red_in, a.nslots);
    if (threadIdx.x < 8) {
      a.red_row[threadIdx.x] = t;
      if (a.red_prev_jnext && (threadIdx.x == 4 || threadIdx.x == 5))
        a.red_prev_jnext[threadIdx.x - 4] = t;
    }
    return;
  }
  const int tile = xcd_tile(b, a.ntiles);
  const int slot = a.tile_slot[tile];
  const int ty = tile / a.ntx, tx = tile - ty * a.ntx;
  if (slot < 0)
    interior_tile<P>(a, tx, ty);
  else
    general_tile<P, FORCES>(a, tx, ty, slot);
}

// J over the control volume of the populations one pull of src gives.
template <int P>
__global__ __launch_bounds__(kThreads) void box_momentum_kernel(BoxArgs a) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  const T* __restrict__ src = static_cast<const T*>(a.src);
  const int row = blockIdx.x / a.box_bx;
  const int x = a.bx0 + (blockIdx.x - row * a.box_bx) * kTileW + int(threadIdx.x);
  const int y = a.by0 + row;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (x < a.bx1) {
    const uint32_t w = a.node[int64_t(y) * a.nx + x];
    if (!(w & kSolidBit)) {
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const C fi = pull<P>(src, a.plane, a.pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, i);
        v[0] += kCx[i] * double(fi);
        v[1] += kCy[i] * double(fi);
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
    p[k] = S::pack(weight<typename S::C>(i), i);
  }
}

template <int P>
hipError_t step_dispatch(bool forces, const StepArgs& a, hipStream_t s) {
  const int grid = a.ntiles + (a.red_in ? 1 : 0);
  if (forces)
    hipLaunchKernelGGL((step_kernel<P, true>), dim3(grid), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((step_kernel<P, false>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int precision, bool forces, const StepArgs& a, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: return step_dispatch<LBM_FP64>(forces, a, s);
    case LBM_FP32: return step_dispatch<LBM_FP32>(forces, a, s);
    default: return step_dispatch<LBM_FP16DEV>(forces, a, s);
  }
}

hipError_t launch_box_momentum(int precision, const BoxArgs& a, int blocks, hipStream_t s) {
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(box_momentum_kernel<LBM_FP64>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(box_momentum_kernel<LBM_FP32>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL(box_momentum_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
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
    default:
      hipLaunchKernelGGL(fill_rest_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, plane);
  }
  return hipGetLastError();
}

}  // namespace lbm
