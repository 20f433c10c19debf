// Reverse-mode (adjoint) kernel of the collide-stream-bounce-back step, for gradients of
// a time-averaged momentum-exchange force with respect to the inlet velocity profile
// and the relaxation time.
//
// Forward map of one step (Kaushal, Succi & Ansumali, arXiv:2210.10377, Eq. CollideAdv
// with the bounce-back rules of Sec. II): f(t) = P(S(t-1); u_in) (pull: streaming,
// half-way bounce-back, moving-wall inlet, outlet copy) and S(t) = C(f(t); omega) (BGK).
// The objective J = sum_t g_t(S(t)) is linear in the stored state: g_t = (1/T) sum over
// links of 2 c_i . (wx, wy) S_i(x, t) for t in the averaging window (algorithm B, the
// bounce-back force of Sec. IV).  With lambda(t) = dJ/dS(t) and mu(t) = dJ/df(t):
//   mu(t)       = C'(f(t))^T lambda(t)
//   lambda(t-1) = dg_{t-1}/dS(t-1) + P^T mu(t)
//   dJ/domega   = sum_t lambda(t) . (f^eq(f(t)) - f(t))
//   dJ/du_in(y) = sum_t sum_{inlet pulls i at (0, y)} mu_i(t) 2 rho_w w_i c_ix / c_s^2
// One launch handles one reverse step t: it gathers lambda(t) from mu(t+1) (the
// transpose of the pull: the node that pulled S_k(s) returns its adjoint to s), pulls
// f(t) from the stored S(t-1), applies the collision's vector-Jacobian product and
// stores mu(t).  Collision Jacobian (rho = sum f, j = sum c f, u = j / rho):
//   dC_i/df_k = (1 - omega) delta_ik + omega (dfeq_i/drho + dfeq_i/dj . c_k),
//   dfeq_i/drho = w_i [1 - 4.5 (c_i.u)^2 + 1.5 u^2],
//   dfeq_i/dj   = w_i [3 c_i + 9 (c_i.u) c_i - 3 u].
#include <hip/hip_runtime.h>

#include "adjoint.h"
#include "device.h"
#include "plan.h"

namespace lbm {

namespace {

using namespace dev;

// Adjoint code of node s, direction k (see build_adjoint_codes).
__device__ __forceinline__ uint32_t adj_code(uint32_t word, int k) {
  return (word >> (3 * (k - 1))) & 7u;
}

// Collision vector-Jacobian product at one node: mu = C'(f)^T lambda, and the node's
// contribution lambda . (f^eq - f) to dJ/domega.  f is f (or h = f - w for deviation
// storages, whose Jacobian is the same function of rho and u).
template <class C, bool DEV>
__device__ __forceinline__ C collide_vjp(const C (&f)[kQ], const C (&lam)[kQ], C omega,
                                         C (&mu)[kQ]) {
  const C s = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const C jx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
  const C jy = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
  const C rho = DEV ? C(1) + s : s;
  const C ir = C(1) / rho;
  const C ux = jx * ir, uy = jy * ir;
  const C usq = ux * ux + uy * uy;
  C a = 0, bx = 0, by = 0, dom = 0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const C cu = C(kCx[i]) * ux + C(kCy[i]) * uy;
    const C wl = weight<C>(i) * lam[i];
    a += wl * (C(1) - C(4.5) * cu * cu + C(1.5) * usq);
    bx += wl * (C(3) * C(kCx[i]) + C(9) * cu * C(kCx[i]) - C(3) * ux);
    by += wl * (C(3) * C(kCy[i]) + C(9) * cu * C(kCy[i]) - C(3) * uy);
    const C poly = C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq;
    const C feq = DEV ? weight<C>(i) * (s + rho * poly) : weight<C>(i) * rho * (C(1) + poly);
    dom += lam[i] * (feq - f[i]);
  }
#pragma unroll
  for (int k = 0; k < kQ; ++k)
    mu[k] = (C(1) - omega) * lam[k] + omega * (a + bx * C(kCx[k]) + by * C(kCy[k]));
  return dom;
}

template <int P, bool BUF>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(AdjArgs a) {
  using S = Storage<P>;
  using T = typename S::T;
  using C = typename S::C;
  // Tiles reach the XCDs in runs of the single-lattice step's length (the same bytes per
  // run: 32 tiles at 4-byte adjoint values, 16 at 8-byte).
  constexpr int kGroup = kStepGroup * 4 / int(sizeof(C));
  const int tile = block_tile<kGroup>(blockIdx.x, a.ntiles);
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  // The wave's strip (the step kernel's tiles): 64 nodes of row y0 from x0.
  int x0 = 0, y0 = 0;
  strip_origin(tile, wave, a.ntx, a.tile_rows, x0, y0);
  const Planes<T, BUF> st(a.state, a.plane, a.state_bytes);
  const Planes<C, BUF> min(a.mu_in, a.plane, a.mu_bytes);
  const Planes<C, BUF> mout(a.mu_out, a.plane, a.mu_bytes);
  const int pitch = a.pitch;
  const int x = x0 + (int(threadIdx.x) & 63);
  const C om = C(a.omega);
  // The running sums of the earlier launches, read before the gathers so that their
  // latency overlaps them (each slot belongs to this wave alone).
  const int64_t dslot = int64_t(tile) * kStrips + wave;
  const double dom_prev = a.domega[dslot];
  const double duin_prev = x0 == 0 && y0 < a.ny ? a.duin[y0] : 0.0;
  double dom_acc = 0.0;
  if (y0 >= a.ny) {
    // a narrow tile's strip below the last row: nothing to do
  } else if (strip_is_plain(a.nx, a.ny, a.gx0, a.gx1, a.gy0, a.gy1, x0, y0) &&
             strip_is_interior(a.nx, a.ny, x0, y0)) {
    // Every neighbour is fluid and streams: lambda_k(s) = mu_k(s + c_k),
    // f_i(s) = S_i(s - c_i).
    {
      const int32_t o = y0 * pitch + x;
      C lam[kQ], f[kQ];
#pragma unroll
      for (int k = 0; k < kQ; ++k) lam[k] = min.ld(k, o + kCy[k] * pitch + kCx[k]);
#pragma unroll
      for (int i = 0; i < kQ; ++i) f[i] = unpack<P>(st.ld(i, o - kCy[i] * pitch - kCx[i]), i);
      C mu[kQ];
      dom_acc += double(collide_vjp<C, S::kDev>(f, lam, om, mu));
#pragma unroll
      for (int k = 0; k < kQ; ++k) mout.st(k, o, mu[k]);
    }
  } else {
    do {
      const int y = y0;
      if (x >= a.nx) break;
      const int32_t o = y * pitch + x;
      // Every adjoint value the transposed pull may gather is read unconditionally (all
      // in bounds) and the codes select among them afterwards: no gather waits for the
      // adjoint code word.
      const uint32_t w = a.node[int64_t(y) * a.nx + x];
      const uint32_t aw = a.adj[int64_t(y) * a.nx + x];
      C lown[kQ], lfar[kQ], lout[kQ];
#pragma unroll
      for (int k = 0; k < kQ; ++k) lown[k] = min.ld(k, o);
#pragma unroll
      for (int k = 1; k < kQ; ++k) {
        // The reader s + c_k (periodic images included) ...
        int dx = x + kCx[k], dy = y + kCy[k];
        dx = dx < 0 ? dx + a.nx : (dx >= a.nx ? dx - a.nx : dx);
        dy = dy < 0 ? dy + a.ny : (dy >= a.ny ? dy - a.ny : dy);
        lfar[k] = min.ld(k, dy * pitch + dx);
        // ... and the outlet node (nx - 1, s_y + c_ky), which copies S_k(s) for the
        // directions entering the outlet column from outside (c_kx < 0).
        lout[k] = kCx[k] < 0 ? min.ld(k, dy * pitch + (a.nx - 1)) : C(0);
      }
      if (w & kSolidBit) break;
      // The pull of f(t) from S(t-1) (its addresses need the node word only) goes out
      // before the adjoint code word is used.
      C f[kQ];
      pull_all<P>(st, pitch, a.nx, a.ny, a.uin, a.rho_w6, w, x, y, f);
      C lam[kQ];
      lam[0] = lown[0];
#pragma unroll
      for (int k = 1; k < kQ; ++k) {
        const uint32_t ac = adj_code(aw, k);
        C l = 0;
        // streaming or a periodic wrap (one reader at most)
        if (ac & (kAdjStream | kAdjWrap)) l += lfar[k];
        if (kCx[k] < 0 && (ac & kAdjOutlet)) l += lout[k];
        // Bounce-back at s: the pull of the opposite direction returns S_k(s).
        const uint32_t oc = pull_code(w, kOpp[k]);
        if (oc == kBody || oc == kWall || oc == kInlet) l += lown[kOpp[k]];
        // The objective reads S_k(s) on the link (s, k) of the body.
        if (oc == kBody) l += C(a.gx * kCx[k] + a.gy * kCy[k]);
        lam[k] = l;
      }
      C mu[kQ];
      dom_acc += double(collide_vjp<C, S::kDev>(f, lam, om, mu));
#pragma unroll
      for (int k = 0; k < kQ; ++k) mout.st(k, o, mu[k]);
      // Inlet pulls add 2 rho_w w_i c_ix u_in(y) / c_s^2 to f_i(0, y).
      if (x == 0) {
        double g = 0.0;
#pragma unroll
        for (int i = 1; i < kQ; ++i)
          if (kCx[i] != 0 && pull_code(w, i) == kInlet)
            g += double(mu[i]) * a.rho_w6 * weight<double>(i) * kCx[i];
        a.duin[y] = duin_prev + g;
      }
    } while (false);
  }
  // dJ/domega: one running sum per wave, updated in launch order (deterministic).
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) dom_acc += __shfl_xor(dom_acc, off, 64);
  if ((threadIdx.x & 63) == 0) a.domega[dslot] = dom_prev + dom_acc;
}

template <class C>
__global__ __launch_bounds__(kThreads) void zero_kernel(C* p, int64_t n) {
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * kThreads)
    p[k] = C(0);
}

template <int P>
hipError_t adjoint_dispatch(const AdjArgs& a, hipStream_t s) {
  if (a.state_bytes && a.mu_bytes)
    hipLaunchKernelGGL((adjoint_kernel<P, true>), dim3(a.ntiles), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((adjoint_kernel<P, false>), dim3(a.ntiles), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint(int precision, const AdjArgs& a, hipStream_t s) {
  switch (precision) {
    case LBM_FP64: return adjoint_dispatch<LBM_FP64>(a, s);
    case LBM_FP32: return adjoint_dispatch<LBM_FP32>(a, s);
    case LBM_FP32DEV: return adjoint_dispatch<LBM_FP32DEV>(a, s);
    case LBM_FP32SR: return adjoint_dispatch<LBM_FP32SR>(a, s);
    case LBM_FP16DEV: return adjoint_dispatch<LBM_FP16DEV>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel<double>, dim3(1024), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel<float>, dim3(1024), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace lbm
