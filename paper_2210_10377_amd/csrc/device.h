// Device building blocks shared by the forward step and the adjoint kernels: storage
// formats, buffer addressing, the BGK and regularized collisions, the pull of one node with its boundary
// rules, and fixed-order wave / block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lbm.h"
#include "plan.h"

namespace lbm {
namespace dev {
constexpr int kThreads = kTileW;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <class C>
__device__ __forceinline__ constexpr C weight(int i) {
  return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

// w_i x with the weight carried to beyond binary32 precision.  The binary32 weights are
// 4, 1 and 1/4 times fl(1/9) = (1 + 7.45e-9)/9, so an equilibrium formed with them holds
// 1 + 7.45e-9 times the mass and momentum of its node, and every collision would add
// omega 7.45e-9 of both: a systematic drive that builds up to relative 1e-4 in the forces
// over 10^4 steps.  Adding the product with the binary32 remainder of the weight first
// leaves one rounding and no such bias.  Binary64 weights are used as they are.
// Binary32 remainder of the weight: w_i - fl(w_i).
__device__ __forceinline__ float weight_lo(int i) {
  constexpr float lo0 = float(4.0 / 9.0 - double(4.0f / 9.0f));
  constexpr float lo1 = float(1.0 / 9.0 - double(1.0f / 9.0f));
  constexpr float lo2 = float(1.0 / 36.0 - double(1.0f / 36.0f));
  return i == 0 ? lo0 : (i < 5 ? lo1 : lo2);
}
template <class C, bool EXACT = true>
__device__ __forceinline__ C wmul(int i, C x) {
  if constexpr (sizeof(C) == 8 || !EXACT)
    return weight<C>(i) * x;
  else
    return __builtin_fmaf(weight<float>(i), x, weight_lo(i) * x);
}

// Storage of a population and the arithmetic type it is computed in.  kDev: the
// arithmetic is in deviation form, h_i = f_i - w_i; kStoreF: the stored value is f_i
// itself (otherwise a deviation storage stores h_i); kSR: stores round stochastically.
template <int P>
struct Storage;

// kExactW: the equilibrium carries the binary32 weights' remainders (wmul); binary16
// storage rounds at 2^-11, far above the 2^-27 of the bare binary32 weights, and skips
// the two extra operations per weight.
template <>
struct Storage<LBM_FP64> {
  using T = double;
  using C = double;
  static constexpr bool kDev = false;
  static constexpr bool kExactW = true;
  static constexpr bool kStoreF = true;
  static constexpr bool kSR = false;
};

template <>
struct Storage<LBM_FP32> {
  using T = float;
  using C = float;
  static constexpr bool kDev = false;
  static constexpr bool kExactW = true;
  static constexpr bool kStoreF = true;
  static constexpr bool kSR = false;
};

template <>
struct Storage<LBM_FP32DEV> {
  using T = float;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kExactW = true;
  static constexpr bool kStoreF = false;
  static constexpr bool kSR = false;
};

template <>
struct Storage<LBM_FP16DEV> {
  using T = _Float16;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kExactW = false;
  static constexpr bool kStoreF = false;
  static constexpr bool kSR = false;
};

// Binary32 populations f_i, arithmetic in deviation form, stores rounded stochastically.
template <>
struct Storage<LBM_FP32SR> {
  using T = float;
  using C = float;
  static constexpr bool kDev = true;
  static constexpr bool kExactW = true;
  static constexpr bool kStoreF = true;
#ifdef LBM_SR_NEAREST
  static constexpr bool kSR = false;
#else
  static constexpr bool kSR = true;
#endif
};

// Stored value of direction i -> arithmetic value (f, or h for deviation arithmetic),
// and back (rounded to nearest; binary16: to nearest even).  When f_i itself is stored
// in binary32, the deviation is taken from the binary32 weight, h_i = f_i - fl(w_i):
// exact for f_i within a factor of two of fl(w_i) (Sterbenz), and so is the way back
// but for one rounding of f_i.  The remainders w_i - fl(w_i) = -eps w_i (one eps for
// all nine weights) then cancel in the equilibrium deviation: with s = sum h_i and the
// exact weights, w_i (s + rho poly_i) equals f^eq_i - fl(w_i) but for terms of order
// eps poly_i (below 1e-10).  Forming h_i - (w_i - fl(w_i)) in binary32 instead would
// drop the remainder wherever the spacing of h_i exceeds it, and bias every collision.
template <int P>
__device__ __forceinline__ typename Storage<P>::C unpack(typename Storage<P>::T v, int i) {
  using S = Storage<P>;
  if constexpr (S::kDev && S::kStoreF)
    return v - weight<float>(i);
  else
    return typename S::C(v);
}
template <int P>
__device__ __forceinline__ typename Storage<P>::T pack(typename Storage<P>::C v, int i) {
  using S = Storage<P>;
  if constexpr (S::kDev && S::kStoreF)
    return weight<float>(i) + v;
  else
    return typename S::T(v);
}

// Uniform 32-bit word of node (x, y) in one step, from the step's key (sr_step_key of
// the step number, on the host) and the node's index y nx + x (not its offset in the
// state buffer, so both layouts and every tile shape draw alike); direction i of the
// node takes the word + i * 0x9e3779b9 (each direction's word alone is uniform).
__device__ __forceinline__ uint32_t sr_node_word(uint32_t step_key, int nx, int x, int y) {
  return fmix32(step_key ^ (uint32_t(y) * uint32_t(nx) + uint32_t(x)));
}

// Stochastic rounding of f_i = fl(w_i) + h_i to binary32: the two neighbours
// y <= f_i <= y' (or y' <= f_i <= y) are taken with probabilities proportional to their
// closeness, so the expected stored value is f_i itself.  The error of the rounded sum is
// exact (TwoSum, Knuth), the draw the top 24 bits of the direction's word.  Round to
// nearest when kSR is off.
template <int P>
__device__ __forceinline__ typename Storage<P>::T pack_sr(typename Storage<P>::C v, int i,
                                                          uint32_t word) {
  using S = Storage<P>;
  if constexpr (S::kSR) {
    const float a = weight<float>(i);
    const float y = a + v;
    const float bb = y - a;
    const float e = (a - (y - bb)) + (v - bb);
    const uint32_t yb = __builtin_bit_cast(uint32_t, y);
    // Neighbour on the side of the error: one unit in the last place away from zero when
    // e and y share a sign, towards it otherwise.  A zero, infinite or NaN error fails the
    // comparison below, so y stays.
    const uint32_t nb = yb + 1u - (((__builtin_bit_cast(uint32_t, e) ^ yb) >> 30) & 2u);
    const float yn = __builtin_bit_cast(float, nb);
    const float gap = __builtin_fabsf(yn - y);
    const float u = float((word + uint32_t(i) * 0x9e3779b9u) >> 8) * 0x1p-24f;
    return (u * gap < __builtin_fabsf(e)) ? yn : y;
  } else {
    return pack<P>(v, i);
  }
}

// The population f_i in binary64 from an arithmetic value of direction i (f_i, or the
// deviation from the weight the storage uses).
template <int P>
__device__ __forceinline__ double pre_f64(typename Storage<P>::C v, int i) {
  using S = Storage<P>;
  if constexpr (!S::kDev)
    return double(v);
  else if constexpr (S::kStoreF)
    return double(weight<float>(i)) + double(v);
  else
    return weight<double>(i) + double(v);
}

// The population f_i in binary64 from a stored value of direction i.
template <int P>
__device__ __forceinline__ double to_f64(typename Storage<P>::T v, int i) {
  return (Storage<P>::kDev && !Storage<P>::kStoreF) ? weight<double>(i) + double(v) : double(v);
}

// Raw buffer access of one stored population (cache policy `aux`: 0 default, 2 nt).
template <class T>
struct RawBuf;
template <>
struct RawBuf<double> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, 2);
  }
};
template <>
struct RawBuf<float> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 2);
  }
};
template <>
struct RawBuf<_Float16> {
  static __device__ __forceinline__ _Float16 ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, _Float16 x) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 2);
  }
};

// The nine populations of one state buffer: population i of the node at element offset
// off = y * pitch + x sits at i * plane + off (row-interleaved or planar layout).
template <class T, bool BUF>
struct Planes;

template <class T>
struct Planes<T, true> {
  __amdgpu_buffer_rsrc_t r;
  uint32_t plane_bytes;
  __device__ __forceinline__ Planes(const void* base, int64_t plane, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000)),
        plane_bytes(uint32_t(plane * int64_t(sizeof(T)))) {}
  __device__ __forceinline__ T ld(int i, int32_t off) const {
    return RawBuf<T>::ld(r, uint32_t(off) * uint32_t(sizeof(T)), uint32_t(i) * plane_bytes);
  }
  // Plane index varying per lane.
  __device__ __forceinline__ T ld_lane(int i, int32_t off) const {
    return RawBuf<T>::ld(r, uint32_t(i) * plane_bytes + uint32_t(off) * uint32_t(sizeof(T)), 0u);
  }
  __device__ __forceinline__ void st(int i, int32_t off, T v) const {
    RawBuf<T>::st(r, uint32_t(off) * uint32_t(sizeof(T)), uint32_t(i) * plane_bytes, v);
  }
};

template <class T>
struct Planes<T, false> {
  T* p;
  int64_t plane;
  __device__ __forceinline__ Planes(const void* base, int64_t pl, uint32_t)
      : p(static_cast<T*>(const_cast<void*>(base))), plane(pl) {}
  __device__ __forceinline__ T ld(int i, int32_t off) const { return p[i * plane + off]; }
  __device__ __forceinline__ T ld_lane(int i, int32_t off) const { return p[i * plane + off]; }
  __device__ __forceinline__ void st(int i, int32_t off, T v) const {
    __builtin_nontemporal_store(v, p + i * plane + off);
  }
};

// Collision of one node; COLL selects the operator (LBM_COLL_*):
//   BGK (Eq. CollideAdv, first line, with 2 beta = omega) towards the second-order
//   equilibrium w_i rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2];
//   regularized (Latt & Chopard 2006): f~_i = f^eq_i + (1 - omega) (9/2) w_i
//   (c_i c_i - I/3) : Pi^neq, with Pi^neq = sum c c f - rho u u - rho I/3;
//   KBC (Karlin, Boesch & Chikatamarla 2014, with the same polynomial equilibrium):
//   d = f - f^eq is split into the shear part ds (+-N/4 on the axes, c_x c_y P/4 on the
//   diagonals, N = sum (c_x^2 - c_y^2) d, P = sum c_x c_y d) and dh = d - ds;
//   f~ = f - (omega/2)(2 ds + gamma dh), with the entropic stabilizer
//   gamma = 2/omega - (2 - 2/omega) <ds|dh>/<dh|dh>, <X|Y> = sum X Y / f^eq, and
//   gamma = 2 (BGK) when <dh|dh> is within the rounding noise of the arithmetic
//   (<= 2^-90 rho in binary64, 2^-40 rho in binary32).
// In deviation form (DEV) the inputs and outputs are h_i = f_i - w_i: rho - 1 = sum h_i,
// rho u = sum c_i h_i, f^eq_i - w_i = w_i [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 -
// 1.5 u^2)] and Pi^neq = sum c c h - rho u u - (rho - 1) I/3, so no quantity of order one
// is formed except the entropic weights f^eq_i.
template <class C, bool DEV, int COLL, bool EXACT = true>
__device__ __forceinline__ void collide(const C (&f)[kQ], C omega, C (&g)[kQ]) {
  const C s = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const C jx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const C jy = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const C rho = DEV ? C(1) + s : s;
  const C ir = C(1) / rho;
  const C ux = jx * ir, uy = jy * ir;
  const C usq = C(1.5) * (ux * ux + uy * uy);
  const C om = omega;
  C fe[kQ];  // f^eq (DEV: f^eq - w)
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const C cu = C(kCx[i]) * ux + C(kCy[i]) * uy;
    const C poly = C(3) * cu + C(4.5) * cu * cu - usq;
    fe[i] = DEV ? wmul<C, EXACT>(i, s + rho * poly) : wmul<C, EXACT>(i, rho * (C(1) + poly));
  }
  if constexpr (COLL == LBM_COLL_BGK) {
#pragma unroll
    for (int i = 0; i < kQ; ++i) g[i] = f[i] + om * (fe[i] - f[i]);
  } else if constexpr (COLL == LBM_COLL_REGULARIZED) {
    const C diag = (f[5] + f[6]) + (f[7] + f[8]);
    const C r3 = (DEV ? s : rho) * C(1.0 / 3.0);
    const C pxx = ((f[1] + f[3]) + diag) - rho * ux * ux - r3;
    const C pyy = ((f[2] + f[4]) + diag) - rho * uy * uy - r3;
    const C pxy = (f[5] + f[7]) - (f[6] + f[8]) - rho * ux * uy;
    const C k = (C(1) - om) * C(4.5);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const C q = C(kCx[i] * kCx[i] - 1.0 / 3.0) * pxx + C(2 * kCx[i] * kCy[i]) * pxy +
                  C(kCy[i] * kCy[i] - 1.0 / 3.0) * pyy;
      g[i] = fe[i] + k * weight<C>(i) * q;
    }
  } else {
    C d[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] = f[i] - fe[i];
    const C qn = C(0.25) * ((d[1] + d[3]) - (d[2] + d[4]));
    const C qp = C(0.25) * ((d[5] + d[7]) - (d[6] + d[8]));
    C ds[kQ];
    ds[0] = C(0);
#pragma unroll
    for (int i = 1; i < kQ; ++i) ds[i] = i < 5 ? (kCy[i] == 0 ? qn : -qn) : C(kCx[i] * kCy[i]) * qp;
    // Entropic weights 1/f^eq: exact division in binary64, the hardware reciprocal
    // (1 ulp) in binary32, where they only weigh the stabilizer.
    C sh = C(0), hh = C(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const C dh = d[i] - ds[i];
      const C fq = DEV ? weight<C>(i) + fe[i] : fe[i];
      C wi;
      if constexpr (sizeof(C) == 8)
        wi = C(1) / fq;
      else
        wi = __builtin_amdgcn_rcpf(fq);
      sh += ds[i] * dh * wi;
      hh += dh * dh * wi;
    }
    const C beta = C(0.5) * om;
    const C ib = C(1) / beta;
    const C thr = sizeof(C) == 8 ? C(0x1p-90) : C(0x1p-40);
    const C gamma = hh > thr * rho ? ib - (C(2) - ib) * sh / hh : C(2);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      g[i] = f[i] - beta * (C(2) * ds[i] + gamma * (d[i] - ds[i]));
  }
}

// Block index -> tile index.  Blocks are dealt round-robin over the 8 XCDs; this
// mapping hands each XCD runs of kGroup consecutive row-major tiles, so the cache
// lines shared by horizontally adjacent tiles (the +-1-shifted pulls) meet in one L2,
// while the XCDs together still sweep one region of memory at a time.  The tail that
// does not fill a whole round keeps the identity mapping.  The single-lattice step takes
// runs of 32 tiles at 4-byte storage and the same bytes per run at the others (16 tiles
// in FP64, 64 in FP16; measured best on the row-interleaved layout of a wide grid), as
// does the adjoint (keyed on its adjoint values); the batch (instances of 1-2 tiles per
// row) takes runs of 4.
#ifndef LBM_XCD_GROUP
#define LBM_XCD_GROUP 32
#endif
#ifndef LBM_XCD_GROUP_BATCH
#define LBM_XCD_GROUP_BATCH 4
#endif
constexpr int kStepGroup = LBM_XCD_GROUP, kBatchGroup = LBM_XCD_GROUP_BATCH;
template <int kGroup>
__device__ __forceinline__ int block_tile(int b, int n) {
  constexpr int kRound = 8 * kGroup;
  if (kGroup == 1 || b >= n / kRound * kRound) return b;
  const int xcd = b & 7, k = b >> 3;
  return ((k / kGroup) * 8 + xcd) * kGroup + (k % kGroup);
}

// Populations arriving at fluid node (x, y) (streaming of Eq. CollideAdv with the
// boundary rules), from the node's pull codes.  The source direction and offset of
// every direction are selected first and the nine loads issued together, so a node costs one
// memory latency whatever its boundary rules:
//   stream: S_i(x - c_i); body or wall: S_o(x) (half-way bounce-back, o = opposite);
//   inlet: S_o(x) + 2 w_i rho_w (c_i . u_w) / c_s^2 (moving-wall bounce-back, Sec. II);
//   outlet: S_i(nx-1, y - c_iy) (ghost column); wrap: S_i at the periodic image.
// Moving-wall term 2 w_i rho_w (c_i . u_w) / c_s^2 of a pull along c_i that bounces
// back from the body at the half-way point (x - c_i/2, y - c_i/2) (binary64).
__device__ __forceinline__ double body_wall_term(const BodyMotion& m, double rho_w6, int i,
                                                 int x, int y) {
  const double xw = x - 0.5 * kCx[i], yw = y - 0.5 * kCy[i];
  const double uwx = m.ux - m.omega * (yw - m.yc);
  const double uwy = m.uy + m.omega * (xw - m.xc);
  return rho_w6 * weight<double>(i) * (kCx[i] * uwx + kCy[i] * uwy);
}

template <int P, class A>
__device__ __forceinline__ void pull_all(const A& src, int pitch, int nx, int ny,
                                         const double* uin, double rho_w6, uint32_t w, int x,
                                         int y, typename Storage<P>::C (&f)[kQ],
                                         const BodyMotion* __restrict__ motion = nullptr) {
  using S = Storage<P>;
  using C = typename S::C;
  const int32_t own = y * pitch + x;
  int32_t off[kQ];
  int pl[kQ];
  off[0] = own;
  pl[0] = 0;
#pragma unroll
  for (int i = 1; i < kQ; ++i) {
    const uint32_t code = pull_code(w, i);
    int sx = x - kCx[i], sy = y - kCy[i];
    sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    const bool back = code == kBody || code == kWall || code == kInlet;
    const int32_t o_far = code == kOutlet ? sy * pitch + (nx - 1) : sy * pitch + sx;
    off[i] = back ? own : o_far;
    pl[i] = back ? kOpp[i] : i;
  }
  typename S::T v[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) v[i] = src.ld_lane(pl[i], off[i]);
  // The inlet term is additive, so it applies to f and to h = f - w alike (opposite
  // directions share a weight, so the value pulled from plane pl[i] unpacks with w_i);
  // it is formed in binary64 and rounded once.
  const double uw = rho_w6 * uin[y];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i] = unpack<P>(v[i], i);
    if (i > 0 && kCx[i] != 0 && pull_code(w, i) == kInlet)
      f[i] += C(uw * (weight<double>(i) * kCx[i]));
  }
  // A body in rigid motion: the moving-wall rule on its links (additive, as the inlet).
  if (motion) {
    const BodyMotion m = *motion;
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      if (pull_code(w, i) == kBody) f[i] += C(body_wall_term(m, rho_w6, i, x, y));
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

// Sum N doubles over the wave in a fixed (butterfly) order; lanes 0..N-1 store
// out[0..N-1].
template <int N>
__device__ __forceinline__ void wave_sum_store(double (&v)[N], double* out) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63;
  double mine = v[0];
#pragma unroll
  for (int k = 1; k < N; ++k) mine = lane == k ? v[k] : mine;
  if (lane < N) out[lane] = mine;
}

// Sum N doubles over the wave as wave_sum_store does and store them at out[at..at+N-1]
// of an M-double record whose other entries are written as zero.
template <int N, int M>
__device__ __forceinline__ void wave_sum_store_at(double (&v)[N], int at, double* out) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63;
  double mine = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) mine = lane == at + k ? v[k] : mine;
  if (lane < M) out[lane] = mine;
}

// Fixed-order reduction of [nslots][N] partials by one 256-thread block; returns the N
// sums in threads 0..N-1.  The first G*N threads (G = 256 / N groups) read element
// j*N + k (k = thread % N) of every G-th slot, so each keeps one component.
template <int N>
__device__ __forceinline__ double reduce_partials(const double* in, int nslots) {
  constexpr int kG = kThreads / N;  // slot groups
  __shared__ double red[kG][N];
  const int k = threadIdx.x % N, grp = threadIdx.x / N;
  if (grp < kG) {
    // Eight independent partial sums per lane keep eight loads in flight (this block
    // runs beside the step's tiles and must finish with them); they are combined in a
    // fixed order, so the result depends on nslots only.
    constexpr int kU = 8;
    double acc[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) acc[u] = 0.0;
    int j = grp;
    for (; j + (kU - 1) * kG < nslots; j += kU * kG) {
#pragma unroll
      for (int u = 0; u < kU; ++u) acc[u] += in[int64_t(j + u * kG) * N + k];
    }
    for (; j < nslots; j += kG) acc[0] += in[int64_t(j) * N + k];
    red[grp][k] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < N)
    for (int gI = 0; gI < kG; ++gI) t += red[gI][threadIdx.x];
  return t;
}

}  // namespace dev
}  // namespace lbm
