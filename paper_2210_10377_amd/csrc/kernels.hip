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

#include "kernels.h"
#include "plan.h"

namespace lbm {

namespace {

constexpr int kThreads = kTileW;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <class C>
__device__ __forceinline__ constexpr C weight(int i) {
  return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

// Storage of a population and the arithmetic type it is computed in.  Deviation
// storages keep h_i = f_i - w_i; their arithmetic stays in deviation form.
template <int P>
struct Storage;

template <>
struct Storage<LBM_FP64> {
  using T = double;
  using C = double;
  static constexpr bool kDev = false;
};

template <>
struct Storage<LBM_FP32> {
  using T = float;
  using C = float;
  static constexpr bool kDev = false;
};

template <>
struct Storage<LBM_FP32DEV> {
  using T = float;
  using C = float;
  static constexpr bool kDev = true;
};

template <>
struct Storage<LBM_FP16DEV> {
  using T = _Float16;
  using C = float;
  static constexpr bool kDev = true;
};

// Stored value -> arithmetic value (f, or h for deviation storages) and back (binary16:
// round to nearest even).
template <int P>
__device__ __forceinline__ typename Storage<P>::C unpack(typename Storage<P>::T v) {
  return typename Storage<P>::C(v);
}
template <int P>
__device__ __forceinline__ typename Storage<P>::T pack(typename Storage<P>::C v) {
  return typename Storage<P>::T(v);
}
// The population f_i in binary64 from a stored value of direction i.
template <int P>
__device__ __forceinline__ double to_f64(typename Storage<P>::T v, int i) {
  return Storage<P>::kDev ? weight<double>(i) + double(v) : double(v);
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

// The nine population planes of one state buffer.  Offsets are element offsets
// inside a plane (y * pitch + x); plane i starts i * plane elements into the buffer.
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

// BGK collision of one node (Eq. CollideAdv, first line, with 2 beta = omega) towards
// the second-order equilibrium w_i rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2].  In
// deviation form (DEV) the inputs and outputs are h_i = f_i - w_i: rho - 1 = sum h_i,
// rho u = sum c_i h_i, and f^eq_i - w_i = w_i [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 -
// 1.5 u^2)], so no quantity of order one is formed.
template <class C, bool DEV>
__device__ __forceinline__ void collide(const C (&f)[kQ], C omega, C (&g)[kQ]) {
  const C s = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const C jx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const C jy = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const C rho = DEV ? C(1) + s : s;
  const C ir = C(1) / rho;
  const C ux = jx * ir, uy = jy * ir;
  const C usq = C(1.5) * (ux * ux + uy * uy);
  const C om = omega;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const C cu = C(kCx[i]) * ux + C(kCy[i]) * uy;
    const C poly = C(3) * cu + C(4.5) * cu * cu - usq;
    const C feq = DEV ? weight<C>(i) * (s + rho * poly) : weight<C>(i) * rho * (C(1) + poly);
    g[i] = f[i] + om * (feq - f[i]);
  }
}

// Block index -> tile index.  Blocks are dealt round-robin over the 8 XCDs; this
// mapping hands each XCD runs of kGroup consecutive row-major tiles, so the cache
// lines shared by horizontally adjacent tiles (the +-1-shifted pulls) meet in one L2,
// while the XCDs together still sweep one region of memory at a time.  The tail that
// does not fill a whole round keeps the identity mapping.
#ifndef LBM_XCD_GROUP
#define LBM_XCD_GROUP 4
#endif
__device__ __forceinline__ int block_tile(int b, int n) {
  constexpr int kGroup = LBM_XCD_GROUP, kRound = 8 * kGroup;
  if (kGroup == 1 || b >= n / kRound * kRound) return b;
  const int xcd = b & 7, k = b >> 3;
  return ((k / kGroup) * 8 + xcd) * kGroup + (k % kGroup);
}

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

// Populations arriving at fluid node (x, y) (streaming of Eq. CollideAdv with the
// boundary rules), from the node's pull codes.  The source plane and offset of every
// direction are selected first and the nine loads issued together, so a node costs one
// memory latency whatever its boundary rules:
//   stream: S_i(x - c_i); body or wall: S_o(x) (half-way bounce-back, o = opposite);
//   inlet: S_o(x) + 2 w_i rho_w (c_i . u_w) / c_s^2 (moving-wall bounce-back, Sec. II);
//   outlet: S_i(nx-1, y - c_iy) (ghost column); wrap: S_i at the periodic image.
template <int P, class A>
__device__ __forceinline__ void pull_all(const A& src, int pitch, int nx, int ny,
                                         const double* uin, double rho_w6, uint32_t w, int x,
                                         int y, typename Storage<P>::C (&f)[kQ]) {
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
  // directions share a weight).
  const C uw = C(rho_w6 * uin[y]);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i] = unpack<P>(v[i]);
    if (i > 0 && kCx[i] != 0 && pull_code(w, i) == kInlet) f[i] += uw * (weight<C>(i) * C(kCx[i]));
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

// Sum 8 doubles over the wave in a fixed (butterfly) order; lanes 0..7 store out[0..7].
__device__ __forceinline__ void wave_sum8_store(double (&v)[8], double* out) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63;
  double mine = v[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) mine = lane == k ? v[k] : mine;
  if (lane < 8) out[lane] = mine;
}

// Fixed-order reduction of [nslots][8] partials by one 256-thread block; returns the
// eight sums in threads 0..7.
__device__ __forceinline__ double reduce_partials8(const double* in, int nslots) {
  __shared__ double red[kThreads / 8][8];
  constexpr int kG = kThreads / 8;  // slot groups
  const int k = threadIdx.x & 7, grp = threadIdx.x >> 3;
  // Four independent partial sums per lane keep four loads in flight; they are
  // combined in a fixed order, so the result depends on nslots only.
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = grp;
  for (; j + 3 * kG < nslots; j += 4 * kG) {
    s0 += in[int64_t(j) * 8 + k];
    s1 += in[int64_t(j + kG) * 8 + k];
    s2 += in[int64_t(j + 2 * kG) * 8 + k];
    s3 += in[int64_t(j + 3 * kG) * 8 + k];
  }
  for (; j < nslots; j += kG) s0 += in[int64_t(j) * 8 + k];
  const double s = (s0 + s1) + (s2 + s3);
  red[grp][k] = s;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < 8)
    for (int gI = 0; gI < kThreads / 8; ++gI) t += red[gI][threadIdx.x];
  return t;
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
