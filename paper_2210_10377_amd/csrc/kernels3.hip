// Kernels of the three-dimensional (D3Q27) path: the fused pull-stream + BGK step with
// the per-step forces (A, B, DRTT terms, SI), the control-volume momentum sweep, and the
// fixed-order reductions of the force partials into ring rows.
//
// One launch per step.  A block of 256 threads covers a tile of 256 nodes along x in one
// (y, z) row; each wave a 64-node strip whose class (strip table) picks its path:
//   plain / box-J: 27 loads at fixed offsets (no boundary within reach), collision,
//     27 non-temporal stores; box-J strips add the momentum of their pulled populations;
//   general: the node word and the coordinates select, per direction, plain streaming,
//     a periodic wrap, bounce-back (wall, body, outlet ghost of a solid node), the inlet
//     moving-wall rule or the outlet ghost copy; strips with force terms accumulate A, B,
//     J, Phi and SI in FP64 and reduce them over the wave into their slot.
// The first block of a launch reduces the previous step's slots, in a fixed order, into
// that step's ring row.  Blocks are mapped to tiles so that runs of kXcdRun (8)
// neighbouring tiles along x go to one XCD (their +-1-shifted pulls share cache lines in
// that L2).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "kernels3.h"
#include "lbm.h"
#include "plan3.h"

namespace lbm3 {
namespace {

constexpr int kThreads = kTileW;

template <int P>
struct St3;
// kDev: arithmetic in deviation form; kStoreF: the stored value is f_i itself (else a
// deviation storage stores h_i = f_i - w_i); kSR: stores round stochastically.
template <>
struct St3<LBM_FP64> {
  using T = double;
  using C = double;
  static constexpr bool kDev = false, kStoreF = true, kSR = false;
};
template <>
struct St3<LBM_FP32> {
  using T = float;
  using C = float;
  static constexpr bool kDev = false, kStoreF = true, kSR = false;
};
template <>
struct St3<LBM_FP32DEV> {
  using T = float;
  using C = float;
  static constexpr bool kDev = true, kStoreF = false, kSR = false;
};
template <>
struct St3<LBM_FP16DEV> {
  using T = _Float16;
  using C = float;
  static constexpr bool kDev = true, kStoreF = false, kSR = false;
};
// Binary32 populations, arithmetic in deviation form from the binary32 weights, stores
// rounded stochastically.
template <>
struct St3<LBM_FP32SR> {
  using T = float;
  using C = float;
  static constexpr bool kDev = true, kStoreF = true, kSR = true;
};

// Weights: (2/3, 1/6, 1/6) per axis.
template <class C>
__device__ __forceinline__ constexpr C w27(int i) {
  return (kCx[i] == 0 ? C(2) / C(3) : C(1) / C(6)) * (kCy[i] == 0 ? C(2) / C(3) : C(1) / C(6)) *
         (kCz[i] == 0 ? C(2) / C(3) : C(1) / C(6));
}

// w_i x with the weight carried beyond binary32 precision: the binary32 weights are not
// exact, and an equilibrium formed with them alone would hold slightly more (or less)
// mass and momentum than its node; every collision would add that bias (relative ~1e-8
// per step, ~1e-4 in the forces over 10^4 steps).  The product with the binary32
// remainder of the weight is added first, so one rounding remains and no bias.
template <class C>
__device__ __forceinline__ C wmul27(int i, C x) {
  if constexpr (sizeof(C) == 8) {
    return w27<C>(i) * x;
  } else {
    const float lo = float(w27<double>(i) - double(w27<float>(i)));
    return __builtin_fmaf(w27<float>(i), x, lo * x);
  }
}

// Stored value of direction i -> f_i in binary64.
template <int P>
__device__ __forceinline__ double f64(typename St3<P>::T v, int i) {
  return (St3<P>::kDev && !St3<P>::kStoreF) ? w27<double>(i) + double(v) : double(v);
}

// Stored value of direction i -> arithmetic value, and back (rounded to nearest).  With
// f_i stored in binary32 and deviation arithmetic, the deviation is taken from the
// binary32 weight, h_i = f_i - fl(w_i), exactly for f_i within a factor of two of
// fl(w_i).  The binary32 weights are fl(8/27) scaled by powers of 4, so each is
// (1 + eps) w_i with one eps; the equilibrium deviation w_i (sum h + rho poly_i) with the
// exact weights then equals f^eq_i - fl(w_i) but for terms of order eps poly_i.
template <int P>
__device__ __forceinline__ typename St3<P>::C unpack3(typename St3<P>::T v, int i) {
  using S = St3<P>;
  if constexpr (S::kDev && S::kStoreF)
    return v - w27<float>(i);
  else
    return typename S::C(v);
}
template <int P>
__device__ __forceinline__ typename St3<P>::T pack3(typename St3<P>::C v, int i) {
  using S = St3<P>;
  if constexpr (S::kDev && S::kStoreF)
    return w27<float>(i) + v;
  else
    return typename S::T(v);
}
// f_i in binary64 from an arithmetic value of direction i.
template <int P>
__device__ __forceinline__ double pre64(typename St3<P>::C v, int i) {
  using S = St3<P>;
  if constexpr (!S::kDev)
    return double(v);
  else if constexpr (S::kStoreF)
    return double(w27<float>(i)) + double(v);
  else
    return w27<double>(i) + double(v);
}

// Stochastic rounding of f_i = fl(w_i) + h_i to binary32 (as in two dimensions): the
// neighbour on the side of the exact TwoSum error is taken with probability |error| /
// spacing, from the top 24 bits of the node's word + i * 0x9e3779b9; the node's word is
// fmix32 of the step key and the node index.  Round to nearest when kSR is off.
template <int P>
__device__ __forceinline__ typename St3<P>::T pack3_sr(typename St3<P>::C v, int i,
                                                       uint32_t word) {
  using S = St3<P>;
  if constexpr (S::kSR) {
    const float a = w27<float>(i);
    const float y = a + v;
    const float bb = y - a;
    const float e = (a - (y - bb)) + (v - bb);
    const uint32_t yb = __builtin_bit_cast(uint32_t, y);
    const uint32_t nb = yb + 1u - (((__builtin_bit_cast(uint32_t, e) ^ yb) >> 30) & 2u);
    const float yn = __builtin_bit_cast(float, nb);
    const float gap = __builtin_fabsf(yn - y);
    const float u = float((word + uint32_t(i) * 0x9e3779b9u) >> 8) * 0x1p-24f;
    return (u * gap < __builtin_fabsf(e)) ? yn : y;
  } else {
    return pack3<P>(v, i);
  }
}
__device__ __forceinline__ uint32_t sr_word3(uint32_t step_key, int64_t node) {
  return lbm::fmix32(step_key ^ uint32_t(node));
}

template <class T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Collision of one node, in place, f or deviations h = f - w: BGK (Eq. CollideAdv), or
// with COLL = LBM_COLL_REGULARIZED the non-equilibrium part replaced by its projection
// w_i / (2 theta0^2) Q_i : Pi^neq on the second-order Hermite polynomials
// (Q_i = c_i c_i - theta0 I) and relaxed: f~ = f^eq + (1 - omega) f^(1).
template <class C, bool DEV, int COLL>
__device__ __forceinline__ void collide27(C (&f)[kQ], C omega) {
  C r = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    r += f[i];
    if (kCx[i]) jx += kCx[i] > 0 ? f[i] : -f[i];
    if (kCy[i]) jy += kCy[i] > 0 ? f[i] : -f[i];
    if (kCz[i]) jz += kCz[i] > 0 ? f[i] : -f[i];
  }
  const C rho = DEV ? C(1) + r : r;
  const C inv = C(1) / rho;
  const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
  if (COLL == LBM_COLL_REGULARIZED) {
    C pxx = C(0), pyy = C(0), pzz = C(0), pxy = C(0), pxz = C(0), pyz = C(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const C cu = C(kCx[i]) * ux + C(kCy[i]) * uy + C(kCz[i]) * uz;
      const C poly = C(3) * cu + C(4.5) * cu * cu - usq;
      const C feq = DEV ? wmul27<C>(i, r + rho * poly) : wmul27<C>(i, rho * (C(1) + poly));
      const C d = f[i] - feq;
      if (kCx[i]) pxx += d;
      if (kCy[i]) pyy += d;
      if (kCz[i]) pzz += d;
      if (kCx[i] * kCy[i]) pxy += kCx[i] * kCy[i] > 0 ? d : -d;
      if (kCx[i] * kCz[i]) pxz += kCx[i] * kCz[i] > 0 ? d : -d;
      if (kCy[i] * kCz[i]) pyz += kCy[i] * kCz[i] > 0 ? d : -d;
      f[i] = feq;
    }
    const C tr = (pxx + pyy + pzz) / C(3);
    const C k1 = (C(1) - omega) * C(4.5);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const C q = C(kCx[i] * kCx[i]) * pxx + C(kCy[i] * kCy[i]) * pyy +
                  C(kCz[i] * kCz[i]) * pzz +
                  C(2) * (C(kCx[i] * kCy[i]) * pxy + C(kCx[i] * kCz[i]) * pxz +
                          C(kCy[i] * kCz[i]) * pyz) - tr;
      f[i] += k1 * w27<C>(i) * q;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const C cu = C(kCx[i]) * ux + C(kCy[i]) * uy + C(kCz[i]) * uz;
    const C poly = C(3) * cu + C(4.5) * cu * cu - usq;
    const C feq = DEV ? wmul27<C>(i, r + rho * poly) : wmul27<C>(i, rho * (C(1) + poly));
    f[i] += omega * (feq - f[i]);
  }
}

__device__ __forceinline__ int wrapc(int s, int n) { return s < 0 ? s + n : (s >= n ? s - n : s); }

__device__ __forceinline__ bool in_box(const Geom3& g, int x, int y, int z) {
  return (g.whole[0] || (x >= g.box[0] && x < g.box[1])) &&
         (g.whole[1] || (y >= g.box[2] && y < g.box[3])) &&
         (g.whole[2] || (z >= g.box[4] && z < g.box[5]));
}

// Source of the pull of direction i at fluid node (x, y, z) with node word w: the
// element offset of the source node ((z ny + y) rstride + x), and whether direction
// opp(i) of the node itself is read (bounce-back: wall, body, outlet ghost of a solid node; the inlet's
// moving-wall rule).  *inl: the inlet term applies; *body: a force-bearing body link in
// direction opp(i).
__device__ __forceinline__ int32_t pull_offset(const Geom3& g, int x, int y, int z, uint32_t w,
                                               int i, int32_t self, bool* bb, bool* inl,
                                               bool* body) {
  int sx = x - kCx[i], sy = y - kCy[i], sz = z - kCz[i];
  if (g.bc_x == LBM_BCX_PERIODIC) sx = wrapc(sx, g.nx);
  if (g.bc_y == LBM_BCY_PERIODIC) sy = wrapc(sy, g.ny);
  if (g.bc_z == LBM_BCY_PERIODIC) sz = wrapc(sz, g.nz);
  *inl = false;
  *body = false;
  *bb = true;
  if (sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) return self;  // wall
  if ((w >> i) & 1u) {
    *body = sx >= 0 && sx < g.nx;
    return self;
  }
  if (sx < 0) {
    *inl = true;
    return self;
  }
  *bb = false;
  const int cx = sx >= g.nx ? g.nx - 1 : sx;  // the outlet ghost copies plane nx-1
  return (sz * g.ny + sy) * g.rstride + cx;
}

// Moving-wall term of the population pulled in direction i across a body link at node
// (x, y, z): 2 rho_w w_i (c_i . u_w) / theta0 with u_w the rigid-body velocity at the
// half-way point x - c_i / 2.
__device__ __forceinline__ double body_wall_term3(const Geom3& g, int i, int x, int y, int z) {
  const double r0 = x - 0.5 * kCx[i] - g.mc[0], r1 = y - 0.5 * kCy[i] - g.mc[1],
               r2 = z - 0.5 * kCz[i] - g.mc[2];
  const double u0 = g.mu[0] + g.mw[1] * r2 - g.mw[2] * r1;
  const double u1 = g.mu[1] + g.mw[2] * r0 - g.mw[0] * r2;
  const double u2 = g.mu[2] + g.mw[0] * r1 - g.mw[1] * r0;
  return g.rho_w6 * w27<double>(i) * (kCx[i] * u0 + kCy[i] * u1 + kCz[i] * u2);
}

// Pull of all 27 populations of a fluid node through the boundary rules; *links: bit d
// set for a body link in direction d.  MOV: the body links carry the moving-wall term.
template <int P, bool MOV>
__device__ __forceinline__ void pull27(const Geom3& g, const typename St3<P>::T* __restrict__ src,
                                       int x, int y, int z, uint32_t w, int32_t self,
                                       typename St3<P>::C (&f)[kQ], uint32_t* links) {
  using C = typename St3<P>::C;
  uint32_t inlm = 0, lk = 0;
  f[0] = unpack3<P>(src[self], 0);
#pragma unroll
  for (int i = 1; i < kQ; ++i) {
    bool bb, inl, body;
    const int32_t off = pull_offset(g, x, y, z, w, i, self, &bb, &inl, &body);
    f[i] = unpack3<P>(src[int64_t(bb ? opp(i) : i) * g.dstride + off], i);  // w_opp(i) = w_i
    if (inl) inlm |= 1u << i;
    if (body) lk |= 1u << opp(i);
  }
  if (MOV && lk) {
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      if ((lk >> opp(i)) & 1u) f[i] += C(body_wall_term3(g, i, x, y, z));
  }
  if (inlm) {
    const double u = g.rho_w6 * g.uin[z * g.ny + y];
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      if (kCx[i] && ((inlm >> i) & 1u)) f[i] += C(u * (w27<double>(i) * kCx[i]));
  }
  *links = lk;
}

// Sum N doubles over the wave (butterfly, fixed order); lanes 0..N-1 store them.
template <int N>
__device__ __forceinline__ void wave_store(double (&v)[N], double* out) {
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

// Sum N doubles over the block in a fixed order; thread k < N gets total k in out[k].
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* out) {
  __shared__ double red[kThreads / 64][N];
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x < N) {
    double s = red[0][threadIdx.x];
#pragma unroll
    for (int wv = 1; wv < kThreads / 64; ++wv) s += red[wv][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Previous step's partials -> ring row (15 values), its J -> J(t+1) of the row before;
// with jpart, the J of the next pull -> this row's J(t+1).  Thread t sums component
// t % 16 of slots t / 16, t / 16 + 16, ... (coalesced, one accumulator), then the 16
// partial sums of each component are added in a fixed order.
__device__ void reduce_row(const double* __restrict__ in, int nslots, int njslots, double* row,
                           double* prev_jnext, const double* __restrict__ jpart, int njblocks) {
  __shared__ double red[16][16];
  const int t = threadIdx.x, c = t & 15, g = t >> 4;
  double acc = 0.0;
  // Eight loads in flight, added in slot order.
  if (c < kPart)
    for (int s0 = g; s0 < nslots; s0 += 16 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int s = s0 + 16 * u;
        v[u] = s < nslots ? in[int64_t(s) * kPart + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
  if (c >= 6 && c < 9) {
    const double* jin = in + int64_t(nslots) * kPart;
    for (int s0 = g; s0 < njslots; s0 += 16 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int s = s0 + 16 * u;
        v[u] = s < njslots ? jin[int64_t(s) * 3 + (c - 6)] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
  }
  red[g][c] = acc;
  __syncthreads();
  if (t < kPart) {
    double v = 0.0;
    for (int k = 0; k < 16; ++k) v += red[k][t];
    row[t] = v;
    if (prev_jnext && t >= 6 && t < 9) prev_jnext[t - 6] = v;
  }
  if (jpart) {
    __syncthreads();
    double j = 0.0;
    if (c < 3)
      for (int b = g; b < njblocks; b += 16) j += jpart[int64_t(b) * 3 + c];
    red[g][c] = j;
    __syncthreads();
    if (t < 3) {
      double v = 0.0;
      for (int k = 0; k < 16; ++k) v += red[k][t];
      row[kPart + t] = v;
    }
  }
}

// Tile of block b: runs of kXcdRun consecutive tiles per XCD (blocks go to the 8 XCDs
// round-robin).
#ifndef LBM3_XCD_RUN
#define LBM3_XCD_RUN 8
#endif
constexpr int64_t kXcdRun = LBM3_XCD_RUN;
__device__ __forceinline__ int64_t tile_of(int64_t b) {
  const int64_t xcd = b & 7, k = b >> 3;
  return ((k / kXcdRun) * 8 + xcd) * kXcdRun + (k % kXcdRun);
}

// General path of one strip: the boundary-aware pull of every node, collision, store,
// and with FTERMS the force terms reduced over the wave into the strip's slot.
template <int P, bool FTERMS, int COLL, bool MOV>
__device__ __forceinline__ void general_strip(const Step3Args& a, uint32_t e, int64_t row, int x,
                                              int y, int z, int lane) {
  using S = St3<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Geom3& g = a.g;
  const int64_t self = row * g.rstride + x;
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const C omega = C(a.omega);
  C f[kQ];
  const bool valid = x < g.nx;
  const uint32_t w = valid ? g.word[row * g.nx + x] : kSolid;
  const bool fluid = !(w & kSolid);
  constexpr bool fterms = FTERMS;
  // Force terms go through two fixed-order wave reductions (before and after the
  // collision), so that few of them are live across it.  Pre: A's lost momentum (0-2),
  // J (3-5), SI (6-8).  Post: A's returned momentum (0-2), B (3-5), Phi (6-8).
  double pre[9], post[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) pre[k] = post[k] = 0.0;
  uint32_t lk = 0;
  bool inV = false;
  if (fluid) {
    pull27<P, MOV>(g, src, x, y, z, w, int32_t(self), f, &lk);
    if (fterms) {
      inV = g.has_box && in_box(g, x, y, z);
      if (inV)
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
          const double v = pre64<P>(f[i], i);
          if (kCx[i]) pre[3] += kCx[i] * v;
          if (kCy[i]) pre[4] += kCy[i] * v;
          if (kCz[i]) pre[5] += kCz[i] * v;
        }
      if (lk) {
#pragma unroll
        for (int d = 1; d < kQ; ++d)
          if ((lk >> d) & 1u) {
            const double v = pre64<P>(f[d], d);
            pre[0] += kCx[d] * v;
            pre[1] += kCy[d] * v;
            pre[2] += kCz[d] * v;
          }
        // SI over the axis links of this node: (sigma - p I) . sum n, n = -c_d.
        if (lk & 0x7eu) {
          double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
          for (int i = 0; i < kQ; ++i) {
            const double v = pre64<P>(f[i], i);
            rho += v;
            jx += kCx[i] * v;
            jy += kCy[i] * v;
            jz += kCz[i] * v;
          }
          const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
          const double usq = ux * ux + uy * uy + uz * uz;
          double pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
          for (int i = 0; i < kQ; ++i) {
            const double v = pre64<P>(f[i], i);
            const double cu = kCx[i] * ux + kCy[i] * uy + kCz[i] * uz;
            const double neq =
                v - w27<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            pxx += kCx[i] * kCx[i] * neq;
            pyy += kCy[i] * kCy[i] * neq;
            pzz += kCz[i] * kCz[i] * neq;
            pxy += kCx[i] * kCy[i] * neq;
            pxz += kCx[i] * kCz[i] * neq;
            pyz += kCy[i] * kCz[i] * neq;
          }
          const double k = -(1.0 - 0.5 * a.omega), p = rho / 3.0;
          double nx = 0.0, ny = 0.0, nz = 0.0;
#pragma unroll
          for (int d = 1; d <= 6; ++d)
            if ((lk >> d) & 1u) {
              nx -= kCx[d];
              ny -= kCy[d];
              nz -= kCz[d];
            }
          pre[6] += (k * pxx - p) * nx + k * pxy * ny + k * pxz * nz;
          pre[7] += k * pxy * nx + (k * pyy - p) * ny + k * pyz * nz;
          pre[8] += k * pxz * nx + k * pyz * ny + (k * pzz - p) * nz;
        }
      }
    }
  }
  // Lane k of the wave keeps total k of the pre-collision terms.
  double mine_pre = 0.0;
  if (fterms) {
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) pre[k] += __shfl_xor(pre[k], o, 64);
#pragma unroll
    for (int k = 0; k < 9; ++k) mine_pre = lane == k ? pre[k] : mine_pre;
  }
  if (fluid) {
    collide27<C, S::kDev, COLL>(f, omega);
    const uint32_t word = S::kSR ? sr_word3(a.step_key, row * g.nx + x) : 0u;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const T q = pack3_sr<P>(f[i], i, word);
      st_nt(dst + int64_t(i) * g.dstride + self, q);
      f[i] = unpack3<P>(q, i);  // forces read the populations as stored
    }
    if (fterms) {
      if (lk) {
        // The population returned along link d at t+1 is f~_d plus, for a moving body,
        // the moving-wall term of the pull of opp(d) (half-way point x + c_d / 2).
#pragma unroll
        for (int d = 1; d < kQ; ++d)
          if ((lk >> d) & 1u) {
            const double v = pre64<P>(f[d], d);
            const double back = MOV ? v + body_wall_term3(g, opp(d), x, y, z) : v;
            post[0] += kCx[d] * back;
            post[1] += kCy[d] * back;
            post[2] += kCz[d] * back;
            post[3] += kCx[d] * (v + back);
            post[4] += kCy[d] * (v + back);
            post[5] += kCz[d] * (v + back);
          }
      }
      if (g.has_box) {
        // Surface flux: populations leaving V (node inside) or entering it (outside).
        bool near = true;
        if (!g.whole[0]) near = near && x >= g.box[0] - 1 && x <= g.box[1];
        if (!g.whole[1]) near = near && y >= g.box[2] - 1 && y <= g.box[3];
        if (!g.whole[2]) near = near && z >= g.box[4] - 1 && z <= g.box[5];
        if (near) {
#pragma unroll
          for (int d = 1; d < kQ; ++d) {
            int tx2 = x + kCx[d], ty2 = y + kCy[d], tz2 = z + kCz[d];
            if (g.bc_x == LBM_BCX_PERIODIC) tx2 = wrapc(tx2, g.nx);
            if (g.bc_y == LBM_BCY_PERIODIC) ty2 = wrapc(ty2, g.ny);
            if (g.bc_z == LBM_BCY_PERIODIC) tz2 = wrapc(tz2, g.nz);
            if (in_box(g, tx2, ty2, tz2) != inV) {
              const double v = (pre64<P>(f[d], d)) *
                               (inV ? -1.0 : 1.0);
              post[6] += kCx[d] * v;
              post[7] += kCy[d] * v;
              post[8] += kCz[d] * v;
            }
          }
        }
      }
    }
  }
  if (fterms) {
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) post[k] += __shfl_xor(post[k], o, 64);
    double mine_post = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) mine_post = lane == k ? post[k] : mine_post;
    // Slot layout FA(3) FB(3) J(3) Phi(3) SI(3): lanes 0-2 A = pre + post, 3-5 B,
    // 6-8 J, 9-11 Phi, 12-14 SI.
    const double apre = __shfl(mine_pre, lane % 3, 64);       // A lost (lanes 0-2)
    const double jv = __shfl(mine_pre, 3 + lane % 3, 64);     // J
    const double si = __shfl(mine_pre, 6 + lane % 3, 64);     // SI
    const double apost = __shfl(mine_post, lane % 3, 64);     // A returned
    const double bv = __shfl(mine_post, 3 + lane % 3, 64);    // B
    const double ph = __shfl(mine_post, 6 + lane % 3, 64);    // Phi
    double v = 0.0;
    if (lane < 3) v = apre + apost;
    else if (lane < 6) v = bv;
    else if (lane < 9) v = jv;
    else if (lane < 12) v = ph;
    else v = si;
    if (lane < kPart) a.part_out[int64_t(strip_slot(e)) * kPart + lane] = v;
  }
}

template <int P, bool FORCES, int COLL, bool MOV>
__global__ __launch_bounds__(kThreads) void step3_kernel(Step3Args a) {
  using S = St3<P>;
  using T = typename S::T;
  using C = typename S::C;
  // With a reducer, blocks 0-7 (one per XCD) come first: block 0 reduces while the
  // tiles stream, and the tile blocks keep their XCD alignment.
  int64_t b = blockIdx.x;
  if (a.red_in) {
    if (b == 0)
      reduce_row(a.red_in, a.nslots, a.njslots, a.red_row, a.red_prev_jnext, nullptr, 0);
    if (b < 8) return;
    b -= 8;
  }
  const int64_t tile = tile_of(b);
  if (tile >= a.ntiles) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t e = a.strip[tile * kStrips + wave];
  if (e == kStripEmpty) return;
  const Geom3& g = a.g;
  const int tx = int(tile % a.ntx);
  const int64_t row = tile / a.ntx;
  const int y = int(row % g.ny), z = int(row / g.ny);
  const int x = tx * kTileW + wave * kStripW + lane;
  const int64_t self = row * g.rstride + x;
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const uint32_t cls = strip_class(e);
  const C omega = C(a.omega);
  C f[kQ];

  if (cls == kPlain || cls == kBoxJ) {
    // No boundary within reach: every source is the neighbour itself.
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      f[i] = unpack3<P>(src[int64_t(i) * g.dstride + self -
                             (int64_t(kCz[i]) * g.ny + kCy[i]) * g.rstride - kCx[i]], i);
    if (FORCES && cls == kBoxJ) {
      double j[3] = {0.0, 0.0, 0.0};
      if (P == LBM_FP16DEV) {
        // sum c_i w_i = 0, so the node's momentum is that of its deviations; binary16
        // deviations are summed in binary32 (the rounding stays far below theirs),
        // and the nodes in FP64.
        float jf[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
          if (kCx[i]) jf[0] += kCx[i] > 0 ? float(f[i]) : -float(f[i]);
          if (kCy[i]) jf[1] += kCy[i] > 0 ? float(f[i]) : -float(f[i]);
          if (kCz[i]) jf[2] += kCz[i] > 0 ? float(f[i]) : -float(f[i]);
        }
        j[0] = jf[0];
        j[1] = jf[1];
        j[2] = jf[2];
      } else {
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
          const double v = pre64<P>(f[i], i);
          if (kCx[i]) j[0] += kCx[i] * v;
          if (kCy[i]) j[1] += kCy[i] * v;
          if (kCz[i]) j[2] += kCz[i] * v;
        }
      }
      wave_store<3>(j, a.part_out + int64_t(a.nslots) * kPart + int64_t(strip_slot(e)) * 3);
    }
    collide27<C, S::kDev, COLL>(f, omega);
    const uint32_t word = S::kSR ? sr_word3(a.step_key, row * g.nx + x) : 0u;
#pragma unroll
    for (int i = 0; i < kQ; ++i) st_nt(dst + int64_t(i) * g.dstride + self, pack3_sr<P>(f[i], i, word));
    return;
  }
  // Strips with force terms run in force3_kernel when forces are evaluated; they hold
  // every body link, so the edge strips left here need no moving-wall term then.
  if (FORCES && cls == kForce) return;
  general_strip<P, false, COLL, FORCES ? false : MOV>(a, e, row, x, y, z, lane);
}

// The strips with force terms (one wave per slot, in slot order): the general path
// with A, B, J, Phi and SI.
template <int P, int COLL, bool MOV>
__global__ __launch_bounds__(kThreads) void force3_kernel(Step3Args a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t slot = int64_t(blockIdx.x) * kStrips + wave;
  if (slot >= a.nslots) return;
  const uint32_t si = a.fstrips[slot];
  const uint32_t e = a.strip[si];
  const int64_t tile = si / kStrips;
  const int tx = int(tile % a.ntx);
  const int64_t row = tile / a.ntx;
  const int y = int(row % a.g.ny), z = int(row / a.g.ny);
  const int x = tx * kTileW + int(si % kStrips) * kStripW + lane;
  general_strip<P, true, COLL, MOV>(a, e, row, x, y, z, lane);
}

// J of the pull of the state src over V, per block of 256 nodes along x in a box row.
template <int P, bool MOV>
__global__ __launch_bounds__(kThreads) void box3_kernel(Box3Args a) {
  using S = St3<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Geom3& g = a.g;
  const int bw = g.box[1] - g.box[0];
  const int nbx = (bw + kThreads - 1) / kThreads;
  const int64_t r = blockIdx.x / nbx;
  const int bx = int(blockIdx.x % nbx);
  const int by = g.box[3] - g.box[2];
  const int y = g.box[2] + int(r % by), z = g.box[4] + int(r / by);
  const int x = g.box[0] + bx * kThreads + threadIdx.x;
  double j[3] = {0.0, 0.0, 0.0};
  if (x < g.box[1]) {
    const int64_t row = int64_t(z) * g.ny + y;
    const uint32_t w = g.word[row * g.nx + x];
    if (!(w & kSolid)) {
      C f[kQ];
      uint32_t lk;
      pull27<P, MOV>(g, static_cast<const T*>(a.src), x, y, z, w, int32_t(row * g.rstride + x), f,
                     &lk);
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const double v = pre64<P>(f[i], i);
        if (kCx[i]) j[0] += kCx[i] * v;
        if (kCy[i]) j[1] += kCy[i] * v;
        if (kCz[i]) j[2] += kCz[i] * v;
      }
    }
  }
  __shared__ double out[3];
  block_sum<3>(j, out);
  if (threadIdx.x < 3) a.jpart[int64_t(blockIdx.x) * 3 + threadIdx.x] = out[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void final3_kernel(Final3Args a) {
  reduce_row(a.red_in, a.nslots, a.njslots, a.row, a.prev_jnext, a.jpart, a.njblocks);
}

// Mask change: one thread per listed node.  A covered node contributes its momentum; an
// uncovered one is refilled with f^eq(rho, u_w) (rho the mean density of its lattice
// neighbours fluid in both masks, periodic axes wrapping, rho_w when none; u_w the
// rigid-body velocity at the node) and contributes minus what it now stores.  Refills
// read valid neighbours only, so no thread reads what another writes.
template <int P>
__global__ __launch_bounds__(kThreads) void remask3_kernel(Remask3Args a) {
  using S = St3<P>;
  using T = typename S::T;
  using C = typename S::C;
  const Geom3& g = a.g;
  T* st = static_cast<T*>(a.state);
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < a.n;
       k += int64_t(gridDim.x) * kThreads) {
    const uint32_t e = uint32_t(a.list[k]);
    const int32_t node = int32_t(e & 0x7fffffffu);
    const int x = node % g.nx, y = (node / g.nx) % g.ny, z = node / (g.nx * g.ny);
    const int64_t at = (int64_t(z) * g.ny + y) * g.rstride + x;
    if (!(e >> 31)) {
      for (int i = 0; i < kQ; ++i) {
        const double f = f64<P>(st[i * g.dstride + at], i);
        v[0] += kCx[i] * f;
        v[1] += kCy[i] * f;
        v[2] += kCz[i] * f;
      }
      continue;
    }
    double rsum = 0.0;
    int cnt = 0;
    for (int i = 1; i < kQ; ++i) {
      int ax = x + kCx[i], ay = y + kCy[i], az = z + kCz[i];
      if (g.bc_x == LBM_BCX_PERIODIC) ax = wrapc(ax, g.nx);
      if (g.bc_y == LBM_BCY_PERIODIC) ay = wrapc(ay, g.ny);
      if (g.bc_z == LBM_BCY_PERIODIC) az = wrapc(az, g.nz);
      if (ax < 0 || ax >= g.nx || ay < 0 || ay >= g.ny || az < 0 || az >= g.nz) continue;
      if (!a.valid[(int64_t(az) * g.ny + ay) * g.nx + ax]) continue;
      const int64_t nb = (int64_t(az) * g.ny + ay) * g.rstride + ax;
      double r = 0.0;
      for (int j = 0; j < kQ; ++j) r += f64<P>(st[j * g.dstride + nb], j);
      rsum += r;
      ++cnt;
    }
    const double rho = cnt > 0 ? rsum / double(cnt) : a.rho_w;
    const double r0 = x - g.mc[0], r1 = y - g.mc[1], r2 = z - g.mc[2];
    const double u0 = g.mu[0] + g.mw[1] * r2 - g.mw[2] * r1;
    const double u1 = g.mu[1] + g.mw[2] * r0 - g.mw[0] * r2;
    const double u2 = g.mu[2] + g.mw[0] * r1 - g.mw[1] * r0;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    for (int i = 0; i < kQ; ++i) {
      const double cu = kCx[i] * u0 + kCy[i] * u1 + kCz[i] * u2;
      const double feq = w27<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      const T q = S::kStoreF ? T(feq) : T(C(feq - w27<double>(i)));
      st[i * g.dstride + at] = q;
      const double f = f64<P>(q, i);
      v[0] -= kCx[i] * f;
      v[1] -= kCy[i] * f;
      v[2] -= kCz[i] * f;
    }
  }
  __shared__ double out[3];
  block_sum<3>(v, out);
  if (threadIdx.x < 3) a.block_out[3 * int64_t(blockIdx.x) + threadIdx.x] = out[threadIdx.x];
}

// Sum of the per-block momenta in a fixed order (one block).
__global__ __launch_bounds__(kThreads) void remask3_sum_kernel(const double* block_out, int nb,
                                                               double* res) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kThreads)
    for (int k = 0; k < 3; ++k) v[k] += block_out[3 * int64_t(b) + k];
  __shared__ double out[3];
  block_sum<3>(v, out);
  if (threadIdx.x < 3) res[threadIdx.x] = out[threadIdx.x];
}

template <int P>
__global__ __launch_bounds__(kThreads) void fill_rest3_kernel(void* buf, int64_t n,
                                                                int64_t dstride) {
  using S = St3<P>;
  using T = typename S::T;
  T* p = static_cast<T*>(buf);
  // Both layouts repeat the 27 directions every 27 * dstride elements.
  const int64_t period = dstride * kQ;
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * kThreads) {
    const int i = int((k % period) / dstride);
    // The stochastically rounded storage's rest state is its reference weights.
    p[k] = (S::kDev && !S::kStoreF) ? T(0)
                                    : (S::kDev ? T(w27<float>(i)) : T(w27<double>(i)));
  }
}

template <int P, int COLL, bool MOV>
hipError_t step_pcm(bool forces, const Step3Args& a, hipStream_t s) {
  const int64_t tiles = (a.ntiles + 8 * kXcdRun - 1) / (8 * kXcdRun) * (8 * kXcdRun);
  const dim3 grid(unsigned(tiles + (a.red_in ? 8 : 0)));
  if (forces) {
    hipLaunchKernelGGL((step3_kernel<P, true, COLL, MOV>), grid, dim3(kThreads), 0, s, a);
    if (a.nslots > 0) {
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      const unsigned fblocks = unsigned((a.nslots + kStrips - 1) / kStrips);
      hipLaunchKernelGGL((force3_kernel<P, COLL, MOV>), dim3(fblocks), dim3(kThreads), 0, s, a);
    }
  } else {
    hipLaunchKernelGGL((step3_kernel<P, false, COLL, MOV>), grid, dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

// Bodies in motion take their own instantiation, so the resting case keeps its
// registers.
template <int P, int COLL>
hipError_t step_pc(bool forces, const Step3Args& a, hipStream_t s) {
  return a.g.moving ? step_pcm<P, COLL, true>(forces, a, s)
                    : step_pcm<P, COLL, false>(forces, a, s);
}

template <int P>
hipError_t step_p(bool forces, const Step3Args& a, hipStream_t s) {
  return a.collision == LBM_COLL_REGULARIZED ? step_pc<P, LBM_COLL_REGULARIZED>(forces, a, s)
                                             : step_pc<P, LBM_COLL_BGK>(forces, a, s);
}

}  // namespace

hipError_t launch_step3(int precision, bool forces, const Step3Args& a, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: return step_p<LBM_FP64>(forces, a, s);
    case LBM_FP32: return step_p<LBM_FP32>(forces, a, s);
    case LBM_FP32DEV: return step_p<LBM_FP32DEV>(forces, a, s);
    case LBM_FP32SR: return step_p<LBM_FP32SR>(forces, a, s);
    case LBM_FP16DEV: return step_p<LBM_FP16DEV>(forces, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
void box_p(const Box3Args& a, int blocks, hipStream_t s) {
  if (a.g.moving)
    hipLaunchKernelGGL((box3_kernel<P, true>), dim3(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((box3_kernel<P, false>), dim3(blocks), dim3(kThreads), 0, s, a);
}

hipError_t launch_box3(int precision, const Box3Args& a, int blocks, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: box_p<LBM_FP64>(a, blocks, s); break;
    case LBM_FP32: box_p<LBM_FP32>(a, blocks, s); break;
    case LBM_FP32DEV: box_p<LBM_FP32DEV>(a, blocks, s); break;
    case LBM_FP32SR: box_p<LBM_FP32SR>(a, blocks, s); break;
    case LBM_FP16DEV: box_p<LBM_FP16DEV>(a, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_final3(const Final3Args& a, hipStream_t s) {
  hipLaunchKernelGGL(final3_kernel, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_remask3(int precision, const Remask3Args& a, int blocks, double* out,
                          hipStream_t s) {
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(remask3_kernel<LBM_FP64>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(remask3_kernel<LBM_FP32>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32DEV:
      hipLaunchKernelGGL(remask3_kernel<LBM_FP32DEV>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP32SR:
      hipLaunchKernelGGL(remask3_kernel<LBM_FP32SR>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    case LBM_FP16DEV:
      hipLaunchKernelGGL(remask3_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(remask3_sum_kernel, dim3(1), dim3(kThreads), 0, s,
                     static_cast<const double*>(a.block_out), blocks, out);
  return hipGetLastError();
}

hipError_t launch_fill_rest3(int precision, void* buf, int64_t n, int64_t dstride, hipStream_t s) {
  const int blocks = 2048;
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(fill_rest3_kernel<LBM_FP64>, dim3(blocks), dim3(kThreads), 0, s, buf, n,
                         dstride);
      break;
    case LBM_FP32:
      hipLaunchKernelGGL(fill_rest3_kernel<LBM_FP32>, dim3(blocks), dim3(kThreads), 0, s, buf, n,
                         dstride);
      break;
    case LBM_FP32DEV:
      hipLaunchKernelGGL(fill_rest3_kernel<LBM_FP32DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, n,
                         dstride);
      break;
    case LBM_FP32SR:
      hipLaunchKernelGGL(fill_rest3_kernel<LBM_FP32SR>, dim3(blocks), dim3(kThreads), 0, s, buf, n,
                         dstride);
      break;
    case LBM_FP16DEV:
      hipLaunchKernelGGL(fill_rest3_kernel<LBM_FP16DEV>, dim3(blocks), dim3(kThreads), 0, s, buf, n,
                         dstride);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbm3
