// TEST INFRASTRUCTURE ONLY -- the oracle.
//
// A plain, slow reference of the D2Q9 lattice Boltzmann time step with half-way
// bounce-back and the per-step flow-force estimators of Kaushal, Succi & Ansumali,
// "Flow force calculation in Lattice Boltzmann Method" (arXiv:2210.10377): momentum
// exchange under algorithm A and algorithm B (Sec. IV, Eq. rtt4/rtt5), the discrete
// Reynolds-transport-theorem control-volume force DRTT (Sec. IV, second Eq. rtt7;
// Appendix), and stress integration over the staircase surface (Sec. III,
// Eq. stress_int).
//
// Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark load
// this library.  The product (the HIP library) never links, calls or reads it, and the
// two share no code, tables or constants.
//
// Everything is written as loops over nodes (y, x) and directions i in the order the
// paper's Appendix gives for one time step.  No blocking, no fusion, no reordering.
// The scalar type is a template parameter, so the same code runs in
// std::complex<double> for complex-step derivatives.  Build with
//   g++ -O2 -ffp-contract=off -shared -fPIC
//
// Readings of passages where the paper is silent or ambiguous:
//  * node (x, y) sits at the point (x, y); directions are numbered
//      0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1);
//  * tau is the lattice relaxation time tau_lb = tau_paper + 1/2, so that the factor
//    2*beta = 2/(2*tau_paper + 1) of Eq. CollideAdv equals omega = 1/tau_lb;
//  * the stored state is the post-collision field; one step pulls it (streaming with
//    the boundary rules), records J over the control volume from the pulled,
//    pre-collision populations (Appendix: "before collide"), collides, and evaluates
//    the forces;
//  * pull rules, first match wins: periodic wrap > no-slip wall > inlet > outlet >
//    body bounce-back > plain streaming;
//  * the inlet is the moving-wall bounce-back of Sec. II at x = -1/2 with wall
//    velocity (u_in(y), 0) and wall density rho_w; a body in rigid motion takes the same
//    rule at the half-way point of each link, with the same rho_w;
//  * the outlet copies the post-collision populations of column nx-1 into a ghost
//    column nx (zero gradient);
//  * algorithm A uses the pre-collision outgoing population f_i(x,t) in the lost
//    momentum, algorithm B the post-collision one (Eq. rtt4); both use the populations
//    returned by the boundary at t+1 for the gained momentum (Eq. rtt3);
//  * a population crosses a surface when its streaming link crosses it (the normal
//    tests "c.n > 0" / "c.n <= 0" of Eq. rtt3-rtt7 read as link crossings);
//  * the control volume V is the set of fluid nodes in the half-open box
//    [x0, x1) x [y0, y1);
//  * stress integration: the body surface is the staircase of unit faces crossed by
//    the axis links; the traction of a face is evaluated at the link's fluid node from
//    its pre-collision populations; the deviatoric stress is
//    -(1 - beta) sum f^neq c c, the sign that gives the viscous stress 2 rho nu S of
//    the continuum limit (the printed formula is read with that sign).

#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// Threads of the row loops (1: serial).  The node loops over rows are independent.
// Every sum over nodes is formed from per-row lists of its terms that are added
// afterwards, one term at a time in the serial (y, x, i) order, so every result is
// bitwise the same for any thread count.
int g_threads = 1;

// Terms of K sums, row by row: rows may be filled in parallel; fold() adds them to
// acc[0..K-1] in row order and, within a row, in the order they were pushed.
template <class T, int K>
struct RowTerms {
  std::vector<std::vector<std::array<T, K>>> rows;
  explicit RowTerms(int ny) : rows(size_t(ny)) {}
  void push(int y, const std::array<T, K>& t) { rows[size_t(y)].push_back(t); }
  void fold(T* acc) const {
    for (const auto& r : rows)
      for (const auto& t : r)
        for (int k = 0; k < K; ++k) acc[k] += t[k];
  }
};

// ---------------------------------------------------------------------------------
// Lattice: D2Q9 velocity set and weights (Sec. II, Table I), theta0 = 1/3.
// ---------------------------------------------------------------------------------
const int NQ = 9;
const int CX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double W[NQ] = {16.0 / 36.0, 4.0 / 36.0, 4.0 / 36.0, 4.0 / 36.0, 4.0 / 36.0,
                      1.0 / 36.0,  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const double THETA0 = 1.0 / 3.0;

// Direction opposite to i (Sec. II, bounce-back), found once by search over the table.
int search_opposite(int i) {
  for (int k = 0; k < NQ; ++k)
    if (CX[k] == -CX[i] && CY[k] == -CY[i]) return k;
  return -1;
}
struct OppTable {
  int o[NQ];
  OppTable() {
    for (int i = 0; i < NQ; ++i) o[i] = search_opposite(i);
  }
};
const OppTable OPP;
int opposite(int i) { return OPP.o[i]; }

enum { BCX_INLET_OUTLET = 0, BCX_PERIODIC = 1 };
enum { BCY_WALL = 0, BCY_PERIODIC = 1 };

// Second-order equilibrium (Sec. II):
//   f_i^eq = w_i rho [1 + (u.c_i)/theta0 + ((u.c_i)^2 - theta0 u^2) / (2 theta0^2)].
template <class T>
T equilibrium(int i, T rho, T ux, T uy) {
  T cu = double(CX[i]) * ux + double(CY[i]) * uy;
  T usq = ux * ux + uy * uy;
  return W[i] * rho *
         (1.0 + cu / THETA0 + (cu * cu - THETA0 * usq) / (2.0 * THETA0 * THETA0));
}

// One node of the BGK collision, Eq. CollideAdv (first line):
//   f~_i = f_i + 2 beta (f_i^eq(rho, u) - f_i),  rho = sum f_i, rho u = sum c_i f_i
// (Sec. II, moments).  2 beta is passed as omega.  When a body force g is given (test
// fixtures only; the paper has none) the Guo, Zheng & Shi (2002) forcing is added:
//   u = (sum c_i f_i + g/2) / rho,  extra term (1 - omega/2) w_i [3(c_i - u) + 9 (c_i.u) c_i].g
template <class T>
void collide_node(const T* f, T omega, double gx, double gy, T* out) {
  T rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    jx += double(CX[i]) * f[i];
    jy += double(CY[i]) * f[i];
  }
  T ux = (jx + 0.5 * gx) / rho;
  T uy = (jy + 0.5 * gy) / rho;
  for (int i = 0; i < NQ; ++i) {
    out[i] = f[i] + omega * (equilibrium<T>(i, rho, ux, uy) - f[i]);
    if (gx != 0.0 || gy != 0.0) {
      T cu = double(CX[i]) * ux + double(CY[i]) * uy;
      T fx = 3.0 * (double(CX[i]) - ux) + 9.0 * cu * double(CX[i]);
      T fy = 3.0 * (double(CY[i]) - uy) + 9.0 * cu * double(CY[i]);
      out[i] += (1.0 - 0.5 * omega) * W[i] * (fx * gx + fy * gy);
    }
  }
}

// Regularized collision (Latt & Chopard, Math. Comput. Simul. 72 (2006) 165): the
// stated variant for relaxation times close to 1/2, where BGK loses stability.  It is
// not in the paper.  The non-equilibrium part of f is replaced by its projection on the
// second-order Hermite subspace before relaxing:
//   Pi^neq = sum_i c_i c_i (f_i - f_i^eq),
//   f_i^(1) = w_i / (2 theta0^2) (c_i c_i - theta0 I) : Pi^neq,
//   f~_i = f_i^eq + (1 - 2 beta) f_i^(1).
// Mass and momentum are conserved as in BGK (f^(1) has neither).
template <class T>
void collide_node_regularized(const T* f, T omega, T* out) {
  T rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    jx += double(CX[i]) * f[i];
    jy += double(CY[i]) * f[i];
  }
  T ux = jx / rho;
  T uy = jy / rho;
  T feq[NQ];
  T pxx = 0.0, pxy = 0.0, pyy = 0.0;
  for (int i = 0; i < NQ; ++i) {
    feq[i] = equilibrium<T>(i, rho, ux, uy);
    T neq = f[i] - feq[i];
    pxx += double(CX[i] * CX[i]) * neq;
    pxy += double(CX[i] * CY[i]) * neq;
    pyy += double(CY[i] * CY[i]) * neq;
  }
  for (int i = 0; i < NQ; ++i) {
    T q = (double(CX[i] * CX[i]) - THETA0) * pxx + 2.0 * double(CX[i] * CY[i]) * pxy +
          (double(CY[i] * CY[i]) - THETA0) * pyy;
    T f1 = W[i] / (2.0 * THETA0 * THETA0) * q;
    out[i] = feq[i] + (1.0 - omega) * f1;
  }
}

// Entropic multi-relaxation collision of Karlin, Boesch & Chikatamarla (Phys. Rev. E 90
// (2014) 031302(R)), the "KBC" model, written here with the paper's second-order
// polynomial equilibrium.  It is not in the paper.  The non-equilibrium part
// d = f - f^eq (no mass, no momentum) is split into a shear part ds, built from the
// deviatoric normal stress N = sum (c_x^2 - c_y^2) d and the shear stress
// P = sum c_x c_y d of d alone:
//   ds = 0 (rest),  +N/4 (c = (+-1, 0)),  -N/4 (c = (0, +-1)),  c_x c_y P / 4 (diagonals),
// and the remainder dh = d - ds (trace, third and fourth moments).  Then
//   f~ = f - beta (2 ds + gamma dh),  beta = omega / 2,
// with gamma the entropic stabilizer that minimizes the quadratic entropy
// <f~ - f^eq | f~ - f^eq>, <X|Y> = sum X_i Y_i / f^eq_i:
//   gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>.
// When dh is within a few hundred rounding units of the populations
// (<dh|dh> <= 2^-90 rho, against about 2^-106 rho for one unit in binary64), its
// direction is rounding noise and gamma = 2 (BGK) is used.
// The shear stress relaxes exactly as in BGK (same viscosity); mass and momentum are
// conserved.
template <class T>
void collide_node_kbc(const T* f, T omega, T* out) {
  T rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    jx += double(CX[i]) * f[i];
    jy += double(CY[i]) * f[i];
  }
  T ux = jx / rho;
  T uy = jy / rho;
  T feq[NQ], d[NQ], ds[NQ], dh[NQ];
  T dN = 0.0, dP = 0.0;
  for (int i = 0; i < NQ; ++i) {
    feq[i] = equilibrium<T>(i, rho, ux, uy);
    d[i] = f[i] - feq[i];
    dN += double(CX[i] * CX[i] - CY[i] * CY[i]) * d[i];
    dP += double(CX[i] * CY[i]) * d[i];
  }
  for (int i = 0; i < NQ; ++i) {
    if (CX[i] == 0 && CY[i] == 0)
      ds[i] = 0.0;
    else if (CY[i] == 0)
      ds[i] = 0.25 * dN;
    else if (CX[i] == 0)
      ds[i] = -0.25 * dN;
    else
      ds[i] = 0.25 * double(CX[i] * CY[i]) * dP;
    dh[i] = d[i] - ds[i];
  }
  T sh = 0.0, hh = 0.0;
  for (int i = 0; i < NQ; ++i) {
    sh += ds[i] * dh[i] / feq[i];
    hh += dh[i] * dh[i] / feq[i];
  }
  T beta = 0.5 * omega;
  T gamma = 2.0;
  if (std::real(hh) > std::ldexp(1.0, -90) * std::real(rho))
    gamma = 1.0 / beta - (2.0 - 1.0 / beta) * sh / hh;
  for (int i = 0; i < NQ; ++i) out[i] = f[i] - beta * (2.0 * ds[i] + gamma * dh[i]);
}

enum { COLLISION_BGK = 0, COLLISION_REGULARIZED = 1, COLLISION_KBC = 2 };

struct Config {
  int32_t nx, ny, bc_x, bc_y;
  int32_t box[4];  // x0, x1, y0, y1; x0 < 0 means no control volume
  double rho_w;    // inlet wall density
  double gx, gy;   // body force (test fixtures only; BGK only)
  int32_t collision;  // COLLISION_BGK, COLLISION_REGULARIZED or COLLISION_KBC
  // Rigid motion of the body (all zero: at rest): translation velocity, rotation rate
  // about the z axis, and the centre of rotation.
  double body_u[2];
  double body_omega;
  double body_c[2];
};

// Per-step record: FA(2), FB(2), J(2), Phi(2), SI(2), Jpost(2).
const int NREC = 12;
// Estimators reported per step: A, B, DRTT, SI, DRTT with the post-collision box
// momentum; two components each.
const int NSCHEME = 5;

template <class T>
struct Sim {
  Config cfg;
  std::vector<uint8_t> solid;  // [ny][nx]
  std::vector<T> uin;          // [ny]
  T omega;
  std::vector<T> S;   // post-collision state of the last step, [9][ny][nx]
  std::vector<T> f;   // pulled (pre-collision) populations of the last step
  std::vector<T> Sn;  // scratch for the next state
  std::vector<T> rec;  // [t][NREC]
  // Records whose J(t+1) was fixed when the geometry changed after them: the record
  // index and the control-volume momentum of the pull that followed under the old mask.
  std::vector<size_t> jfix_t;
  std::vector<T> jfix;  // [k][2]

  int nx() const { return cfg.nx; }
  int ny() const { return cfg.ny; }
  size_t idx(int i, int x, int y) const {
    return (size_t(i) * cfg.ny + size_t(y)) * cfg.nx + size_t(x);
  }
  bool is_solid(int x, int y) const { return solid[size_t(y) * cfg.nx + x] != 0; }
  bool in_box(int x, int y) const {
    return cfg.box[0] >= 0 && x >= cfg.box[0] && x < cfg.box[1] && y >= cfg.box[2] &&
           y < cfg.box[3];
  }
  // V: the fluid nodes inside the control-volume box.
  bool in_V(int x, int y) const { return in_box(x, y) && !is_solid(x, y); }

  // Population arriving at fluid node (x, y) in direction i, pulled from state St
  // (streaming, Eq. CollideAdv second line) with the boundary rules in the order
  // periodic > wall > inlet > outlet > body > stream.
  T pull(const std::vector<T>& St, int x, int y, int i) const {
    const int o = opposite(i);
    int sx = x - CX[i], sy = y - CY[i];
    if (cfg.bc_x == BCX_PERIODIC) sx = (sx + cfg.nx) % cfg.nx;
    if (cfg.bc_y == BCY_PERIODIC) sy = (sy + cfg.ny) % cfg.ny;
    // No-slip wall half-way between rows -1|0 and ny-1|ny: stationary-wall
    // bounce-back (Sec. II).
    if (cfg.bc_y == BCY_WALL && (sy < 0 || sy >= cfg.ny)) return St[idx(o, x, y)];
    // Inlet at x = -1/2: moving-wall bounce-back (Sec. II) with u_w = (u_in(y), 0).
    // The population leaving towards the wall is o; the one returned is i:
    //   f~_i(x, t+1) = f~_o(x, t) - 2 w_o rho_w (c_o . u_w) / c_s^2,  c_s^2 = theta0.
    if (cfg.bc_x == BCX_INLET_OUTLET && sx < 0) {
      T cu = double(CX[o]) * uin[y];
      return St[idx(o, x, y)] - 2.0 * W[o] * cfg.rho_w * cu / THETA0;
    }
    // Outlet at x = nx - 1/2: ghost column nx holds a copy of column nx-1.
    if (cfg.bc_x == BCX_INLET_OUTLET && sx >= cfg.nx) {
      if (is_solid(cfg.nx - 1, sy)) return St[idx(o, x, y)];
      return St[idx(i, cfg.nx - 1, sy)];
    }
    // Body: half-way bounce-back (Sec. II).  A body in rigid motion moves the wall
    // point half-way along the link, x - c_i/2, with u_w = U + Omega e_z x (x_w - x_c),
    // and the moving-wall rule applies as at the inlet (zero term at rest).
    if (is_solid(sx, sy)) {
      const double xw = x - 0.5 * CX[i], yw = y - 0.5 * CY[i];
      const double uwx = cfg.body_u[0] - cfg.body_omega * (yw - cfg.body_c[1]);
      const double uwy = cfg.body_u[1] + cfg.body_omega * (xw - cfg.body_c[0]);
      const double cu = double(CX[o]) * uwx + double(CY[o]) * uwy;
      return St[idx(o, x, y)] - 2.0 * W[o] * cfg.rho_w * cu / THETA0;
    }
    return St[idx(i, sx, sy)];
  }

  // Fluid node (x, y) and direction i form a fluid-solid link when x + c_i is a body
  // node (Sec. III, momentum exchange; Fig. 1 caption: boundary point half-way along
  // the link).  Periodic axes wrap; leaving the domain along a bounded axis is not a
  // body link (walls, inlet and outlet are not part of the body).
  bool is_link(int x, int y, int i) const {
    if (i == 0 || is_solid(x, y)) return false;
    int tx = x + CX[i], ty = y + CY[i];
    if (cfg.bc_x == BCX_PERIODIC) tx = (tx + cfg.nx) % cfg.nx;
    if (cfg.bc_y == BCY_PERIODIC) ty = (ty + cfg.ny) % cfg.ny;
    if (tx < 0 || tx >= cfg.nx || ty < 0 || ty >= cfg.ny) return false;
    return is_solid(tx, ty);
  }

  // Control-volume momentum J^Omega (Eq. rtt1) of a population field.
  void box_momentum(const std::vector<T>& g, T* J) const {
    J[0] = 0.0;
    J[1] = 0.0;
    RowTerms<T, 2> terms(cfg.ny);
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int y = 0; y < cfg.ny; ++y)
      for (int x = 0; x < cfg.nx; ++x) {
        if (!in_V(x, y)) continue;
        for (int i = 0; i < NQ; ++i)
          terms.push(y, {double(CX[i]) * g[idx(i, x, y)], double(CY[i]) * g[idx(i, x, y)]});
      }
    terms.fold(J);
  }

  void stream_all(const std::vector<T>& St, std::vector<T>& out) const {
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int y = 0; y < cfg.ny; ++y)
      for (int x = 0; x < cfg.nx; ++x) {
        if (is_solid(x, y)) continue;
        for (int i = 0; i < NQ; ++i) out[idx(i, x, y)] = pull(St, x, y, i);
      }
  }

  // One time step (Appendix order): J(t) before collision, collide, boundary flux
  // through the control-volume surface, advection with bounce-back, MEA forces.
  void step() {
    const int nx = cfg.nx, ny = cfg.ny;
    // Streaming of the previous post-collision state gives f(., t).
    stream_all(S, f);
    // Control-volume momentum before collision (Appendix).
    T J[2];
    box_momentum(f, J);
    // Collision of the entire fluid domain (Eq. CollideAdv, first line).
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        if (is_solid(x, y)) {  // body nodes keep what they hold; it is never read
          for (int i = 0; i < NQ; ++i) Sn[idx(i, x, y)] = S[idx(i, x, y)];
          continue;
        }
        T fin[NQ], fout[NQ];
        for (int i = 0; i < NQ; ++i) fin[i] = f[idx(i, x, y)];
        if (cfg.collision == COLLISION_REGULARIZED)
          collide_node_regularized<T>(fin, omega, fout);
        else if (cfg.collision == COLLISION_KBC)
          collide_node_kbc<T>(fin, omega, fout);
        else
          collide_node<T>(fin, omega, cfg.gx, cfg.gy, fout);
        for (int i = 0; i < NQ; ++i) Sn[idx(i, x, y)] = fout[i];
      }
    // Control-volume momentum after collision, of the populations as stored (the
    // momentum J(t) of Eq. rtt1 sampled on the other side of the collision).
    T Jpost[2];
    box_momentum(Sn, Jpost);
    // Momentum exchange on every fluid-solid link (Sec. III; Eq. rtt4, rtt5):
    // lost momentum c_i f_i (A: pre-collision) or c_i f~_i (B: post-collision) plus
    // the momentum -c_o f_o(x, t+1) = c_i f_o(x, t+1) returned by the boundary.
    // Terms [FAx, FAy, FBx, FBy] per link.
    T F4[4] = {0.0, 0.0, 0.0, 0.0};
    RowTerms<T, 4> mea(ny);
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int i = 1; i < NQ; ++i) {
          if (!is_link(x, y, i)) continue;
          const int o = opposite(i);
          T back = pull(Sn, x, y, o);  // f_o(x, t+1)
          mea.push(y, {double(CX[i]) * (f[idx(i, x, y)] + back),
                       double(CY[i]) * (f[idx(i, x, y)] + back),
                       double(CX[i]) * (Sn[idx(i, x, y)] + back),
                       double(CY[i]) * (Sn[idx(i, x, y)] + back)});
        }
    mea.fold(F4);
    const T FA[2] = {F4[0], F4[1]}, FB[2] = {F4[2], F4[3]};
    // DRTT surface terms on the outer surface of the control volume (second Eq. rtt7):
    //  + populations f~_i(x - c_i, t) entering a node x of V from outside V,
    //  - populations f~_i(x, t) leaving a node x of V for a node outside V.
    // (A leaving population is added negated: a - b is a + (-b) in IEEE arithmetic.)
    T Phi[2] = {0.0, 0.0};
    if (cfg.box[0] >= 0) {
      RowTerms<T, 2> flux(ny);
#pragma omp parallel for schedule(static) num_threads(g_threads)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          if (!in_V(x, y)) continue;
          for (int i = 1; i < NQ; ++i) {
            int ux = x - CX[i], uy = y - CY[i];  // upstream node
            if (!in_box(ux, uy))
              flux.push(y, {double(CX[i]) * Sn[idx(i, ux, uy)], double(CY[i]) * Sn[idx(i, ux, uy)]});
            int dx = x + CX[i], dy = y + CY[i];  // downstream node
            if (!in_box(dx, dy))
              flux.push(y, {-(double(CX[i]) * Sn[idx(i, x, y)]), -(double(CY[i]) * Sn[idx(i, x, y)])});
          }
        }
      flux.fold(Phi);
    }
    // Stress integration (Sec. III, Eq. stress_int) over the staircase surface of the
    // body: every axis link (x, i) (i = 1..4, x fluid, x + c_i solid) is a unit face
    // whose normal out of the body is n = -c_i; the traction there is
    // (-p I + sigma) . n with p = rho theta0 and the deviatoric stress taken as the
    // second moment of the non-equilibrium populations (the passage following Eq.
    // stress_int), sigma = -(1 - beta) sum_k (f_k - f_k^eq) c_k c_k, 2 beta = omega,
    // all from the pre-collision populations f(x, t) of the fluid node of the link
    // (f^eq of the collision; the theta0 delta / D term vanishes since sum f^neq = 0).
    T SI[2] = {0.0, 0.0};
    RowTerms<T, 2> traction(ny);
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int i = 1; i <= 4; ++i) {
          if (!is_link(x, y, i)) continue;
          T fin[NQ];
          for (int k = 0; k < NQ; ++k) fin[k] = f[idx(k, x, y)];
          T rho = 0.0, jx = 0.0, jy = 0.0;
          for (int k = 0; k < NQ; ++k) {
            rho += fin[k];
            jx += double(CX[k]) * fin[k];
            jy += double(CY[k]) * fin[k];
          }
          T ux = (jx + 0.5 * cfg.gx) / rho;
          T uy = (jy + 0.5 * cfg.gy) / rho;
          T pxx = 0.0, pxy = 0.0, pyy = 0.0;
          for (int k = 0; k < NQ; ++k) {
            T neq = fin[k] - equilibrium<T>(k, rho, ux, uy);
            pxx += double(CX[k] * CX[k]) * neq;
            pxy += double(CX[k] * CY[k]) * neq;
            pyy += double(CY[k] * CY[k]) * neq;
          }
          T visc = -(1.0 - 0.5 * omega);
          T sxx = visc * pxx, sxy = visc * pxy, syy = visc * pyy;
          T p = rho * THETA0;
          double nxv = -CX[i], nyv = -CY[i];
          traction.push(y, {(sxx - p) * nxv + sxy * nyv, sxy * nxv + (syy - p) * nyv});
        }
    traction.fold(SI);
    S.swap(Sn);
    const T r[NREC] = {FA[0], FA[1], FB[0], FB[1], J[0], J[1],
                       Phi[0], Phi[1], SI[0], SI[1], Jpost[0], Jpost[1]};
    rec.insert(rec.end(), r, r + NREC);
  }

  // Forces of every recorded step: [t][scheme A, B, DRTT, SI, DRTT-post][x, y].
  // DRTT (second Eq. rtt7): F(t) = J(t) - J(t+1) + Phi(t), both J before collision
  // (Appendix); the J of the step after the last recorded one is the control-volume
  // momentum of the populations the next pull would give.  DRTT-post takes J(t) after
  // the collision instead: F(t) = J^post(t) - J(t+1) + Phi(t), the momentum balance of
  // the box over the streaming half of the step alone.  A collision that conserves
  // momentum makes the two equal.
  void forces(T* out) const {
    const size_t n = rec.size() / NREC;
    T Jlast[2] = {0.0, 0.0};
    if (cfg.box[0] >= 0 && n > 0) {
      std::vector<T> g(S.size(), T(0.0));
      stream_all(S, g);
      box_momentum(g, Jlast);
    }
    for (size_t t = 0; t < n; ++t) {
      const T* r = &rec[NREC * t];
      T* o = out + 2 * NSCHEME * t;
      o[0] = r[0];
      o[1] = r[1];
      o[2] = r[2];
      o[3] = r[3];
      if (cfg.box[0] >= 0) {
        T jx1 = (t + 1 < n) ? rec[NREC * (t + 1) + 4] : Jlast[0];
        T jy1 = (t + 1 < n) ? rec[NREC * (t + 1) + 5] : Jlast[1];
        for (size_t k = 0; k < jfix_t.size(); ++k)
          if (jfix_t[k] == t) {
            jx1 = jfix[2 * k];
            jy1 = jfix[2 * k + 1];
          }
        o[4] = r[4] - jx1 + r[6];
        o[5] = r[5] - jy1 + r[7];
        o[8] = r[10] - jx1 + r[6];
        o[9] = r[11] - jy1 + r[7];
      } else {
        o[4] = NAN;
        o[5] = NAN;
        o[8] = NAN;
        o[9] = NAN;
      }
      o[6] = r[8];
      o[7] = r[9];
    }
  }
};

// Admissible control volume: the box lies at least one node inside the domain on
// every side, and every body node lies strictly inside it with a fluid ring between
// the body and the box surface (so every fluid-solid link is inside V and no
// population crossing the box surface comes from a boundary rule).
bool box_admissible(const Config& c, const uint8_t* mask) {
  if (c.box[0] < 0) return true;
  const int x0 = c.box[0], x1 = c.box[1], y0 = c.box[2], y1 = c.box[3];
  if (x0 < 1 || y0 < 1 || x1 > c.nx - 1 || y1 > c.ny - 1 || x1 - x0 < 3 || y1 - y0 < 3)
    return false;
  for (int y = 0; y < c.ny; ++y)
    for (int x = 0; x < c.nx; ++x)
      if (mask[size_t(y) * c.nx + x] &&
          !(x >= x0 + 1 && x < x1 - 1 && y >= y0 + 1 && y < y1 - 1))
        return false;
  return true;
}

bool config_valid(const Config& c, const uint8_t* mask) {
  if (c.nx < 2 || c.ny < 2) return false;
  if (c.bc_x != BCX_INLET_OUTLET && c.bc_x != BCX_PERIODIC) return false;
  if (c.bc_y != BCY_WALL && c.bc_y != BCY_PERIODIC) return false;
  if (c.collision != COLLISION_BGK && c.collision != COLLISION_REGULARIZED &&
      c.collision != COLLISION_KBC)
    return false;
  if (c.collision != COLLISION_BGK && (c.gx != 0.0 || c.gy != 0.0)) return false;
  for (size_t k = 0; k < size_t(c.nx) * c.ny; ++k)
    if (mask[k] > 1) return false;
  return box_admissible(c, mask);
}

template <class T>
Sim<T>* make_sim(const Config* c, const uint8_t* mask, T omega) {
  if (!config_valid(*c, mask)) return nullptr;
  Sim<T>* s = new Sim<T>();
  s->cfg = *c;
  const size_t n = size_t(c->nx) * c->ny;
  s->solid.assign(mask, mask + n);
  s->uin.assign(c->ny, T(0.0));
  s->omega = omega;
  s->S.assign(NQ * n, T(0.0));
  // Start from rest: every node holds the zero-velocity equilibrium w_i at rho = 1.
  for (int i = 0; i < NQ; ++i)
    for (size_t k = 0; k < n; ++k) s->S[size_t(i) * n + k] = W[i];
  s->f = s->S;
  s->Sn = s->S;
  return s;
}

// A body that moves through the grid: replace the mask (and optionally the control
// volume) between two steps.  Every recorded step keeps the geometry it was taken with:
// the J(t+1) of the last recorded step is fixed now, from the pull of the present state
// under the old mask and box, so the momentum that changes hands with the nodes the body
// covers or uncovers enters no estimator.  Nodes the body uncovers (solid before, fluid
// now) are refilled with the equilibrium at the local wall velocity u_w (the rigid-body
// velocity at the node) and the mean density of their lattice neighbours that are fluid
// in both masks (rho_w when there is none); a neighbour across a periodic edge wraps, one
// outside a non-periodic edge does not count.  impulse = momentum of the covered nodes
// minus that of the refilled ones, i.e. what the fluid hands to the body in the change.
// Returns -1 (nothing changed) when the mask or box is not admissible.
template <class T>
int set_mask(Sim<T>& s, const uint8_t* mask, const int32_t* box, T* impulse) {
  Config c = s.cfg;
  if (box) {
    if ((box[0] >= 0) != (c.box[0] >= 0)) return -1;  // a control volume stays one
    for (int k = 0; k < 4; ++k) c.box[k] = box[k];
  }
  if (!config_valid(c, mask)) return -1;
  const int nx = c.nx, ny = c.ny;
  const size_t n = size_t(nx) * ny;
  const size_t nrec = s.rec.size() / NREC;
  if (s.cfg.box[0] >= 0 && nrec > 0) {
    std::vector<T> g(s.S.size(), T(0.0));
    s.stream_all(s.S, g);
    T J[2];
    s.box_momentum(g, J);
    s.jfix_t.push_back(nrec - 1);
    s.jfix.push_back(J[0]);
    s.jfix.push_back(J[1]);
  }
  const std::vector<uint8_t> old = s.solid;
  auto fluid_both = [&](int x, int y) {
    const size_t k = size_t(y) * nx + x;
    return old[k] == 0 && mask[k] == 0;
  };
  T P[2] = {0.0, 0.0};
  std::vector<T> fresh(NQ * n, T(0.0));
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const size_t k = size_t(y) * nx + x;
      if (old[k] == 0 && mask[k] != 0) {  // covered: its momentum goes to the body
        for (int i = 0; i < NQ; ++i) {
          P[0] += double(CX[i]) * s.S[s.idx(i, x, y)];
          P[1] += double(CY[i]) * s.S[s.idx(i, x, y)];
        }
      } else if (old[k] != 0 && mask[k] == 0) {  // uncovered: refill
        T rsum = 0.0;
        int cnt = 0;
        for (int i = 1; i < NQ; ++i) {
          int ax = x + CX[i], ay = y + CY[i];
          if (c.bc_x == BCX_PERIODIC) ax = (ax + nx) % nx;
          if (c.bc_y == BCY_PERIODIC) ay = (ay + ny) % ny;
          if (ax < 0 || ax >= nx || ay < 0 || ay >= ny || !fluid_both(ax, ay)) continue;
          T r = 0.0;
          for (int j = 0; j < NQ; ++j) r += s.S[s.idx(j, ax, ay)];
          rsum += r;
          ++cnt;
        }
        const T rho = cnt > 0 ? rsum / double(cnt) : T(c.rho_w);
        const T ux = c.body_u[0] - c.body_omega * (double(y) - c.body_c[1]);
        const T uy = c.body_u[1] + c.body_omega * (double(x) - c.body_c[0]);
        for (int i = 0; i < NQ; ++i) fresh[s.idx(i, x, y)] = equilibrium<T>(i, rho, ux, uy);
      }
    }
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const size_t k = size_t(y) * nx + x;
      if (old[k] != 0 && mask[k] == 0)
        for (int i = 0; i < NQ; ++i) {
          s.S[s.idx(i, x, y)] = fresh[s.idx(i, x, y)];
          P[0] -= double(CX[i]) * fresh[s.idx(i, x, y)];
          P[1] -= double(CY[i]) * fresh[s.idx(i, x, y)];
        }
    }
  s.solid.assign(mask, mask + n);
  s.cfg = c;
  if (impulse) {
    impulse[0] = P[0];
    impulse[1] = P[1];
  }
  return 0;
}

}  // namespace

extern "C" {

typedef Config orc_cfg;

// Threads of the oracle's row loops (values below 1 mean 1); results do not depend on
// it.  Returns the previous value.
int32_t orc_set_threads(int32_t n) {
  const int32_t old = g_threads;
  g_threads = n < 1 ? 1 : n;
  return old;
}

// Lattice tables of the oracle (for pins against the paper's Table I).
void orc_lattice(int32_t* cx, int32_t* cy, int32_t* opp, double* w, double* theta0) {
  for (int i = 0; i < NQ; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    opp[i] = opposite(i);
    w[i] = W[i];
  }
  *theta0 = THETA0;
}

void orc_equilibrium(double rho, double ux, double uy, double* feq) {
  for (int i = 0; i < NQ; ++i) feq[i] = equilibrium<double>(i, rho, ux, uy);
}

void orc_collide_node(const double* f, double omega, double gx, double gy, double* out) {
  collide_node<double>(f, omega, gx, gy, out);
}

void orc_collide_node_regularized(const double* f, double omega, double* out) {
  collide_node_regularized<double>(f, omega, out);
}

void orc_collide_node_kbc(const double* f, double omega, double* out) {
  collide_node_kbc<double>(f, omega, out);
}

int orc_box_admissible(const orc_cfg* c, const uint8_t* mask) {
  return box_admissible(*c, mask) ? 1 : 0;
}

// Canonical list of fluid-solid links: pairs (y*nx + x, i), sorted by node index then
// direction.  Returns the number of links (or -1 on an invalid configuration); writes
// at most cap pairs.
int64_t orc_links(const orc_cfg* c, const uint8_t* mask, int32_t* out, int64_t cap) {
  Sim<double>* s = make_sim<double>(c, mask, 1.0);
  if (!s) return -1;
  int64_t n = 0;
  for (int y = 0; y < c->ny; ++y)
    for (int x = 0; x < c->nx; ++x)
      for (int i = 1; i < NQ; ++i)
        if (s->is_link(x, y, i)) {
          if (n < cap) {
            out[2 * n] = int32_t(y * c->nx + x);
            out[2 * n + 1] = i;
          }
          ++n;
        }
  delete s;
  return n;
}

void* orc_create(const orc_cfg* c, const uint8_t* mask, double omega, const double* uin) {
  Sim<double>* s = make_sim<double>(c, mask, omega);
  if (!s) return nullptr;
  if (uin)
    for (int y = 0; y < c->ny; ++y) s->uin[y] = uin[y];
  return s;
}

void orc_destroy(void* h) { delete static_cast<Sim<double>*>(h); }

void orc_set_state(void* h, const double* S) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  std::memcpy(s->S.data(), S, s->S.size() * sizeof(double));
}

void orc_get_state(void* h, double* S) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  std::memcpy(S, s->S.data(), s->S.size() * sizeof(double));
}

// Pre-collision populations f(., t) of the last step (pulled state).
void orc_get_pre(void* h, double* f) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  std::memcpy(f, s->f.data(), s->f.size() * sizeof(double));
}

void orc_step(void* h, int32_t n) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  for (int32_t k = 0; k < n; ++k) s->step();
}

int64_t orc_nrec(void* h) { return int64_t(static_cast<Sim<double>*>(h)->rec.size() / NREC); }

// Raw per-step records [t][FAx, FAy, FBx, FBy, Jx, Jy, Phix, Phiy, SIx, SIy, Jpostx,
// Jposty].
void orc_records(void* h, double* out) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  std::memcpy(out, s->rec.data(), s->rec.size() * sizeof(double));
}

// Forces [t][A, B, DRTT, SI, DRTT-post][x, y] of all recorded steps.
void orc_forces(void* h, double* out) { static_cast<Sim<double>*>(h)->forces(out); }

void orc_clear_records(void* h) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  s->rec.clear();
  s->jfix_t.clear();
  s->jfix.clear();
}

// Replace the body mask, and the control volume when box is non-null (see set_mask).
int orc_set_mask(void* h, const uint8_t* mask, const int32_t* box, double* impulse) {
  return set_mask(*static_cast<Sim<double>*>(h), mask, box, impulse);
}

// Replace the rigid-body motion (translation, rotation rate, centre of rotation).
void orc_set_body_motion(void* h, double ux, double uy, double omega, double xc, double yc) {
  Config& c = static_cast<Sim<double>*>(h)->cfg;
  c.body_u[0] = ux;
  c.body_u[1] = uy;
  c.body_omega = omega;
  c.body_c[0] = xc;
  c.body_c[1] = yc;
}

// Time-averaged momentum-exchange force of algorithm B,
//   J = (1/T) sum_{t=t0}^{t0+T-1} (wx F_Bx(t) + wy F_By(t)),
// of a run of nsteps steps from rest, in complex arithmetic: with omega and u_in given
// a small imaginary part h v, Im J / h is the directional derivative of J (complex
// step).  Every operation of the step is analytic, so no cancellation enters.
int orc_objective_cs(const orc_cfg* c, const uint8_t* mask, double om_re, double om_im,
                     const double* uin_re, const double* uin_im, int32_t nsteps, int32_t t0,
                     int32_t T, double wx, double wy, double* out) {
  typedef std::complex<double> Z;
  Sim<Z>* s = make_sim<Z>(c, mask, Z(om_re, om_im));
  if (!s) return -1;
  for (int y = 0; y < c->ny; ++y)
    s->uin[y] = Z(uin_re ? uin_re[y] : 0.0, uin_im ? uin_im[y] : 0.0);
  for (int32_t k = 0; k < nsteps; ++k) s->step();
  Z J = 0.0;
  for (int32_t t = t0; t < t0 + T; ++t)
    J += wx * s->rec[NREC * size_t(t) + 2] + wy * s->rec[NREC * size_t(t) + 3];
  J /= double(T);
  out[0] = J.real();
  out[1] = J.imag();
  delete s;
  return 0;
}

// Pressure coefficient at the boundary fluid nodes (Sec. V, the C_p equation: computed
// over the boundary fluid nodes, no extrapolation): C_p = (p - p_inf) / (rho_ref U^2 / 2)
// with p = rho theta0 (rho = sum_i f_i of the stored state) and p_inf the pressure at the
// far-upstream reference node (x_inf, y_inf), or rho_ref theta0 when x_inf < 0.  A
// boundary fluid node is a fluid node with at least one fluid-solid link.  Nodes in
// row-major order; writes at most cap (node index y*nx + x, C_p) pairs and returns their
// number, or -1 when the reference node is outside the grid or solid.
int64_t orc_boundary_cp(void* h, int32_t x_inf, int32_t y_inf, double rho_ref, double u_ref,
                        int32_t* nodes, double* cp, int64_t cap) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  auto density = [&](int x, int y) {
    double rho = 0.0;
    for (int i = 0; i < NQ; ++i) rho += s->S[s->idx(i, x, y)];
    return rho;
  };
  double p_inf = rho_ref * THETA0;
  if (x_inf >= 0) {
    if (x_inf >= nx || y_inf < 0 || y_inf >= ny || s->is_solid(x_inf, y_inf)) return -1;
    p_inf = density(x_inf, y_inf) * THETA0;
  }
  const double q = 0.5 * rho_ref * u_ref * u_ref;
  int64_t n = 0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      bool boundary = false;
      for (int i = 1; i < NQ; ++i) boundary = boundary || s->is_link(x, y, i);
      if (!boundary) continue;
      if (n < cap) {
        nodes[n] = int32_t(y * nx + x);
        cp[n] = (density(x, y) * THETA0 - p_inf) / q;
      }
      ++n;
    }
  return n;
}

// Control-volume momentum of an arbitrary population field g (Eq. rtt1).
void orc_momentum_of(void* h, const double* g, double* J) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  std::vector<double> v(g, g + s->S.size());
  s->box_momentum(v, J);
}

}  // extern "C"
