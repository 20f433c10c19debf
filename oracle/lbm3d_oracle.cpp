// TEST INFRASTRUCTURE ONLY -- the three-dimensional oracle.
//
// A plain, slow reference of the D3Q27 lattice Boltzmann time step with half-way
// bounce-back and the per-step flow-force estimators of Kaushal, Succi & Ansumali,
// "Flow force calculation in Lattice Boltzmann Method" (arXiv:2210.10377), carried to
// three dimensions: momentum exchange under algorithms A and B (Sec. IV, Eq. rtt4/rtt5),
// the control-volume force DRTT (second Eq. rtt7; the Appendix's steps with a box in
// x, y and z), and stress integration over the staircase surface (Sec. III,
// Eq. stress_int).  The paper's own 3-D runs use the RD3Q41 model, whose equilibrium
// needs a constant defined only in a cited work; this oracle uses the standard cubic
// D3Q27 set (theta0 = 1/3) with the same second-order equilibrium, collision,
// boundary rules and estimators.
//
// Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark load
// this library.  The product (the HIP library) never links, calls or reads it, and the
// two share no code, tables or constants.
//
// Loops over nodes (z, y, x) and directions in the Appendix's order for one step: pull
// with the boundary rules, box momentum before collision, collide, momentum exchange on
// every link, box surface flux, stress integral.  No blocking, fusion or reordering.
// Build with  g++ -O2 -ffp-contract=off -shared -fPIC
//
// Readings (as for the two-dimensional oracle, one more axis):
//  * node (x, y, z) sits at the point (x, y, z); the directions are numbered
//      0 rest; 1..6 faces +x -x +y -y +z -z; 7..18 edges (xy, xz, yz planes, each as
//      ++ -- +- -+); 19..26 corners +++ --- ++- --+ +-+ -+- -++ +--;
//  * tau is tau_lb, omega = 1/tau_lb = 2 beta of Eq. CollideAdv;
//  * the stored state is post-collision; a step pulls it with the boundary rules,
//    records J over the control volume from the pulled populations, collides and
//    evaluates the forces;
//  * pull rules, first match wins: periodic wrap (any axis) > no-slip walls (y, then z)
//    > inlet (x = -1/2, moving-wall bounce-back with u_w = (u_in(y, z), 0, 0) and wall
//    density rho_w) > outlet (ghost plane x = nx holds plane nx-1) > body bounce-back >
//    plain streaming;
//  * A uses the pre-collision outgoing population, B the post-collision one, both with
//    the population the boundary returns at t+1;
//  * the control volume V is the set of fluid nodes of [x0,x1) x [y0,y1) x [z0,z1);
//    along a periodic axis the box may span the whole axis (then it has no surface
//    there and neighbours wrap into it), which lets a body spanning a periodic
//    direction (an airfoil of infinite span) have a control volume;
//  * collision: BGK (Eq. CollideAdv) or the regularized variant (not in the paper);
//  * a body in rigid motion (not in the paper's runs) takes the moving-wall rule of
//    Sec. II on its links, with the rigid-body velocity at each link's half-way point;
//  * stress integration: unit faces crossed by the six axis links; traction
//    (-p I + sigma) . n, n = -c_i, at the link's fluid node from its pre-collision
//    populations, p = rho theta0, sigma = -(1 - omega/2) sum f^neq c c.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

const int NQ = 27;
const int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                    0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
const int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0,
                    1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
const int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1,
                    1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
const double THETA0 = 1.0 / 3.0;

// Weights of the tensor-product D3Q27 set: (2/3, 1/6, 1/6) per axis, so a velocity
// with k non-zero components has weight (2/3)^(3-k) (1/6)^k.
double weight(int i) {
  double w = 1.0;
  const int c[3] = {CX[i], CY[i], CZ[i]};
  for (int a = 0; a < 3; ++a) w *= (c[a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
  return w;
}

int opposite(int i) {
  for (int k = 0; k < NQ; ++k)
    if (CX[k] == -CX[i] && CY[k] == -CY[i] && CZ[k] == -CZ[i]) return k;
  return -1;
}

enum { BCX_INLET_OUTLET = 0, BCX_PERIODIC = 1 };
enum { BC_WALL = 0, BC_PERIODIC = 1 };

// Second-order equilibrium (Sec. II) with theta0 = 1/3.
double equilibrium(int i, double rho, double ux, double uy, double uz) {
  const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
  const double usq = ux * ux + uy * uy + uz * uz;
  return weight(i) * rho *
         (1.0 + cu / THETA0 + (cu * cu - THETA0 * usq) / (2.0 * THETA0 * THETA0));
}

// BGK collision of one node (Eq. CollideAdv, first line); a body force g (test
// fixtures only) by Guo, Zheng & Shi (2002), as in the two-dimensional oracle.
void collide_node(const double* f, double omega, const double* g, double* out) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    j[0] += CX[i] * f[i];
    j[1] += CY[i] * f[i];
    j[2] += CZ[i] * f[i];
  }
  const double u[3] = {(j[0] + 0.5 * g[0]) / rho, (j[1] + 0.5 * g[1]) / rho,
                       (j[2] + 0.5 * g[2]) / rho};
  const bool forced = g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0;
  for (int i = 0; i < NQ; ++i) {
    out[i] = f[i] + omega * (equilibrium(i, rho, u[0], u[1], u[2]) - f[i]);
    if (forced) {
      const int c[3] = {CX[i], CY[i], CZ[i]};
      const double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += (3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]) * g[a];
      out[i] += (1.0 - 0.5 * omega) * weight(i) * s;
    }
  }
}

// Regularized BGK (Latt & Chopard 2006; not in the paper), as in the two-dimensional
// oracle: the non-equilibrium part is replaced by its projection on the second-order
// Hermite polynomials, f^(1)_i = w_i / (2 theta0^2) Q_i : Pi^neq with
// Q_i = c_i c_i - theta0 I and Pi^neq = sum_k (f_k - f_k^eq) c_k c_k, and relaxed:
// f~_i = f^eq_i + (1 - omega) f^(1)_i.
void collide_node_regularized(const double* f, double omega, double* out) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    j[0] += CX[i] * f[i];
    j[1] += CY[i] * f[i];
    j[2] += CZ[i] * f[i];
  }
  const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double feq[NQ], Pi[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int i = 0; i < NQ; ++i) {
    feq[i] = equilibrium(i, rho, u[0], u[1], u[2]);
    const int c[3] = {CX[i], CY[i], CZ[i]};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Pi[a][b] += double(c[a] * c[b]) * (f[i] - feq[i]);
  }
  for (int i = 0; i < NQ; ++i) {
    const int c[3] = {CX[i], CY[i], CZ[i]};
    double q = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) q += (double(c[a] * c[b]) - (a == b ? THETA0 : 0.0)) * Pi[a][b];
    out[i] = feq[i] + (1.0 - omega) * weight(i) / (2.0 * THETA0 * THETA0) * q;
  }
}

enum { COLLISION_BGK = 0, COLLISION_REGULARIZED = 1 };

struct Config3 {
  int32_t nx, ny, nz, bc_x, bc_y, bc_z;
  int32_t box[6];  // x0, x1, y0, y1, z0, z1; x0 < 0: no control volume
  double rho_w;
  double g[3];     // body force (test fixtures only; BGK only)
  int32_t collision;  // COLLISION_BGK or COLLISION_REGULARIZED
  // Rigid motion of the body (all zero: at rest): translation velocity, angular
  // velocity and the centre of rotation.
  double body_u[3];
  double body_omega[3];
  double body_c[3];
};

// Per-step record: FA(3), FB(3), J(3), Phi(3), SI(3).
const int NREC = 15;

struct Sim3 {
  Config3 cfg;
  std::vector<uint8_t> solid;  // [nz][ny][nx]
  std::vector<double> uin;     // [nz][ny]
  double omega = 1.0;
  std::vector<double> S, f, Sn;  // [27][nz][ny][nx]
  std::vector<double> rec;
  // Records whose J(t+1) was fixed when the geometry changed after them (set_mask): the
  // record index and the box momentum of the pull that followed under the old mask.
  std::vector<size_t> jfix_t;
  std::vector<double> jfix;  // [k][3]

  size_t nodes() const { return size_t(cfg.nx) * cfg.ny * cfg.nz; }
  size_t node(int x, int y, int z) const {
    return (size_t(z) * cfg.ny + size_t(y)) * cfg.nx + size_t(x);
  }
  size_t idx(int i, int x, int y, int z) const { return size_t(i) * nodes() + node(x, y, z); }
  bool is_solid(int x, int y, int z) const { return solid[node(x, y, z)] != 0; }
  bool in_box(int x, int y, int z) const {
    const int32_t* b = cfg.box;
    return b[0] >= 0 && x >= b[0] && x < b[1] && y >= b[2] && y < b[3] && z >= b[4] &&
           z < b[5];
  }
  bool in_V(int x, int y, int z) const { return in_box(x, y, z) && !is_solid(x, y, z); }
  // The node x + d, wrapped along periodic axes (may lie outside a bounded axis).
  void shifted(int x, int y, int z, int dx, int dy, int dz, int* o) const {
    o[0] = x + dx;
    o[1] = y + dy;
    o[2] = z + dz;
    if (cfg.bc_x == BCX_PERIODIC) o[0] = (o[0] + cfg.nx) % cfg.nx;
    if (cfg.bc_y == BC_PERIODIC) o[1] = (o[1] + cfg.ny) % cfg.ny;
    if (cfg.bc_z == BC_PERIODIC) o[2] = (o[2] + cfg.nz) % cfg.nz;
  }

  // Population arriving at fluid node (x, y, z) in direction i, pulled from St.
  double pull(const std::vector<double>& St, int x, int y, int z, int i) const {
    const int o = opposite(i);
    int sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
    if (cfg.bc_x == BCX_PERIODIC) sx = (sx + cfg.nx) % cfg.nx;
    if (cfg.bc_y == BC_PERIODIC) sy = (sy + cfg.ny) % cfg.ny;
    if (cfg.bc_z == BC_PERIODIC) sz = (sz + cfg.nz) % cfg.nz;
    if (cfg.bc_y == BC_WALL && (sy < 0 || sy >= cfg.ny)) return St[idx(o, x, y, z)];
    if (cfg.bc_z == BC_WALL && (sz < 0 || sz >= cfg.nz)) return St[idx(o, x, y, z)];
    if (cfg.bc_x == BCX_INLET_OUTLET && sx < 0) {
      const double cu = CX[o] * uin[size_t(z) * cfg.ny + y];
      return St[idx(o, x, y, z)] - 2.0 * weight(o) * cfg.rho_w * cu / THETA0;
    }
    if (cfg.bc_x == BCX_INLET_OUTLET && sx >= cfg.nx) {
      if (is_solid(cfg.nx - 1, sy, sz)) return St[idx(o, x, y, z)];
      return St[idx(i, cfg.nx - 1, sy, sz)];
    }
    // Body: half-way bounce-back; a body in rigid motion moves the wall point half-way
    // along the link, x_w = x - c_i/2, with u_w = U + Omega x (x_w - x_c), and the
    // moving-wall rule of Sec. II applies as at the inlet (zero term at rest).
    if (is_solid(sx, sy, sz)) {
      const double r[3] = {x - 0.5 * CX[i] - cfg.body_c[0], y - 0.5 * CY[i] - cfg.body_c[1],
                           z - 0.5 * CZ[i] - cfg.body_c[2]};
      const double* W = cfg.body_omega;
      const double uw[3] = {cfg.body_u[0] + W[1] * r[2] - W[2] * r[1],
                            cfg.body_u[1] + W[2] * r[0] - W[0] * r[2],
                            cfg.body_u[2] + W[0] * r[1] - W[1] * r[0]};
      const double cu = CX[o] * uw[0] + CY[o] * uw[1] + CZ[o] * uw[2];
      return St[idx(o, x, y, z)] - 2.0 * weight(o) * cfg.rho_w * cu / THETA0;
    }
    return St[idx(i, sx, sy, sz)];
  }

  // Fluid node x and direction i form a body link when x + c_i (wrapped along periodic
  // axes) is a body node inside the domain.
  bool is_link(int x, int y, int z, int i) const {
    if (i == 0 || is_solid(x, y, z)) return false;
    int tx = x + CX[i], ty = y + CY[i], tz = z + CZ[i];
    if (cfg.bc_x == BCX_PERIODIC) tx = (tx + cfg.nx) % cfg.nx;
    if (cfg.bc_y == BC_PERIODIC) ty = (ty + cfg.ny) % cfg.ny;
    if (cfg.bc_z == BC_PERIODIC) tz = (tz + cfg.nz) % cfg.nz;
    if (tx < 0 || tx >= cfg.nx || ty < 0 || ty >= cfg.ny || tz < 0 || tz >= cfg.nz)
      return false;
    return is_solid(tx, ty, tz);
  }

  void box_momentum(const std::vector<double>& g, double* J) const {
    J[0] = J[1] = J[2] = 0.0;
    for (int z = 0; z < cfg.nz; ++z)
      for (int y = 0; y < cfg.ny; ++y)
        for (int x = 0; x < cfg.nx; ++x) {
          if (!in_V(x, y, z)) continue;
          for (int i = 0; i < NQ; ++i) {
            J[0] += CX[i] * g[idx(i, x, y, z)];
            J[1] += CY[i] * g[idx(i, x, y, z)];
            J[2] += CZ[i] * g[idx(i, x, y, z)];
          }
        }
  }

  void stream_all(const std::vector<double>& St, std::vector<double>& out) const {
    for (int z = 0; z < cfg.nz; ++z)
      for (int y = 0; y < cfg.ny; ++y)
        for (int x = 0; x < cfg.nx; ++x) {
          if (is_solid(x, y, z)) continue;
          for (int i = 0; i < NQ; ++i) out[idx(i, x, y, z)] = pull(St, x, y, z, i);
        }
  }

  void step() {
    const int nx = cfg.nx, ny = cfg.ny, nz = cfg.nz;
    stream_all(S, f);
    double J[3];
    box_momentum(f, J);
    Sn = S;
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          if (is_solid(x, y, z)) continue;
          double fin[NQ], fout[NQ];
          for (int i = 0; i < NQ; ++i) fin[i] = f[idx(i, x, y, z)];
          if (cfg.collision == COLLISION_REGULARIZED)
            collide_node_regularized(fin, omega, fout);
          else
            collide_node(fin, omega, cfg.g, fout);
          for (int i = 0; i < NQ; ++i) Sn[idx(i, x, y, z)] = fout[i];
        }
    // Momentum exchange on every link: c_i (f_i + f_o(x, t+1)) (A) and
    // c_i (f~_i + f_o(x, t+1)) (B), with f_o(x, t+1) pulled from the new state.
    double FA[3] = {0.0, 0.0, 0.0}, FB[3] = {0.0, 0.0, 0.0};
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
          for (int i = 1; i < NQ; ++i) {
            if (!is_link(x, y, z, i)) continue;
            const double back = pull(Sn, x, y, z, opposite(i));
            const double c[3] = {double(CX[i]), double(CY[i]), double(CZ[i])};
            for (int a = 0; a < 3; ++a) {
              FA[a] += c[a] * (f[idx(i, x, y, z)] + back);
              FB[a] += c[a] * (Sn[idx(i, x, y, z)] + back);
            }
          }
    // DRTT surface terms (second Eq. rtt7): populations entering V across the box
    // surface, minus those leaving it.
    double Phi[3] = {0.0, 0.0, 0.0};
    if (cfg.box[0] >= 0) {
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
          for (int x = 0; x < nx; ++x) {
            if (!in_V(x, y, z)) continue;
            for (int i = 1; i < NQ; ++i) {
              const double c[3] = {double(CX[i]), double(CY[i]), double(CZ[i])};
              int u[3], d[3];
              shifted(x, y, z, -CX[i], -CY[i], -CZ[i], u);
              if (!in_box(u[0], u[1], u[2]))
                for (int a = 0; a < 3; ++a) Phi[a] += c[a] * Sn[idx(i, u[0], u[1], u[2])];
              shifted(x, y, z, CX[i], CY[i], CZ[i], d);
              if (!in_box(d[0], d[1], d[2]))
                for (int a = 0; a < 3; ++a) Phi[a] -= c[a] * Sn[idx(i, x, y, z)];
            }
          }
    }
    // Stress integration over the axis links (faces 1..6).
    double SI[3] = {0.0, 0.0, 0.0};
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
          for (int i = 1; i <= 6; ++i) {
            if (!is_link(x, y, z, i)) continue;
            double fin[NQ];
            for (int k = 0; k < NQ; ++k) fin[k] = f[idx(k, x, y, z)];
            double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < NQ; ++k) {
              rho += fin[k];
              j[0] += CX[k] * fin[k];
              j[1] += CY[k] * fin[k];
              j[2] += CZ[k] * fin[k];
            }
            const double u[3] = {(j[0] + 0.5 * cfg.g[0]) / rho, (j[1] + 0.5 * cfg.g[1]) / rho,
                                 (j[2] + 0.5 * cfg.g[2]) / rho};
            double Pi[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
            for (int k = 0; k < NQ; ++k) {
              const double neq = fin[k] - equilibrium(k, rho, u[0], u[1], u[2]);
              const int c[3] = {CX[k], CY[k], CZ[k]};
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Pi[a][b] += double(c[a] * c[b]) * neq;
            }
            const double visc = -(1.0 - 0.5 * omega), p = rho * THETA0;
            const double n[3] = {-double(CX[i]), -double(CY[i]), -double(CZ[i])};
            for (int a = 0; a < 3; ++a) {
              double t = -p * n[a];
              for (int b = 0; b < 3; ++b) t += visc * Pi[a][b] * n[b];
              SI[a] += t;
            }
          }
    S.swap(Sn);
    const double r[NREC] = {FA[0], FA[1], FA[2], FB[0], FB[1], FB[2], J[0], J[1], J[2],
                            Phi[0], Phi[1], Phi[2], SI[0], SI[1], SI[2]};
    rec.insert(rec.end(), r, r + NREC);
  }

  // Forces [t][A, B, DRTT, SI][x, y, z]; DRTT F(t) = J(t) - J(t+1) + Phi(t), the J
  // after the last recorded step from the pull of the present state.
  void forces(double* out) const {
    const size_t n = rec.size() / NREC;
    double Jlast[3] = {0.0, 0.0, 0.0};
    if (cfg.box[0] >= 0 && n > 0) {
      std::vector<double> g(S.size(), 0.0);
      stream_all(S, g);
      box_momentum(g, Jlast);
    }
    for (size_t t = 0; t < n; ++t) {
      const double* r = &rec[NREC * t];
      double* o = out + 12 * t;
      for (int a = 0; a < 3; ++a) {
        o[a] = r[a];
        o[3 + a] = r[3 + a];
        double j1 = (t + 1 < n) ? rec[NREC * (t + 1) + 6 + a] : Jlast[a];
        for (size_t k = 0; k < jfix_t.size(); ++k)
          if (jfix_t[k] == t) j1 = jfix[3 * k + a];
        o[6 + a] = cfg.box[0] >= 0 ? r[6 + a] - j1 + r[9 + a] : NAN;
        o[9 + a] = r[12 + a];
      }
    }
  }
};

// Admissible control volume, axis by axis: a periodic axis may be spanned whole;
// otherwise the box lies one node inside the domain and every body node lies strictly
// inside it with a fluid layer (so every body link is inside V and no population
// crossing the surface comes from a boundary rule).
bool box_admissible(const Config3& c, const uint8_t* mask) {
  if (c.box[0] < 0) return true;
  const int n[3] = {c.nx, c.ny, c.nz};
  const bool per[3] = {c.bc_x == BCX_PERIODIC, c.bc_y == BC_PERIODIC, c.bc_z == BC_PERIODIC};
  bool whole[3];
  for (int a = 0; a < 3; ++a) {
    const int b0 = c.box[2 * a], b1 = c.box[2 * a + 1];
    whole[a] = per[a] && b0 == 0 && b1 == n[a];
    if (!whole[a] && (b0 < 1 || b1 > n[a] - 1 || b1 - b0 < 3)) return false;
  }
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        if (!mask[(size_t(z) * c.ny + y) * c.nx + x]) continue;
        const int p[3] = {x, y, z};
        for (int a = 0; a < 3; ++a)
          if (!whole[a] && !(p[a] >= c.box[2 * a] + 1 && p[a] < c.box[2 * a + 1] - 1))
            return false;
      }
  return true;
}

bool config_valid(const Config3& c, const uint8_t* mask) {
  if (c.nx < 2 || c.ny < 2 || c.nz < 2) return false;
  if (c.bc_x != BCX_INLET_OUTLET && c.bc_x != BCX_PERIODIC) return false;
  if (c.bc_y != BC_WALL && c.bc_y != BC_PERIODIC) return false;
  if (c.bc_z != BC_WALL && c.bc_z != BC_PERIODIC) return false;
  if (c.collision != COLLISION_BGK && c.collision != COLLISION_REGULARIZED) return false;
  if (c.collision != COLLISION_BGK && (c.g[0] != 0.0 || c.g[1] != 0.0 || c.g[2] != 0.0))
    return false;
  for (size_t k = 0; k < size_t(c.nx) * c.ny * c.nz; ++k)
    if (mask[k] > 1) return false;
  return box_admissible(c, mask);
}

// A body that moves through the grid: replace the mask (and optionally the control
// volume) between two steps, as in the two-dimensional oracle.  Every recorded step
// keeps its geometry (the J(t+1) of the last recorded step is fixed now, under the old
// mask and box); uncovered nodes get the equilibrium at the rigid-body velocity at the
// node and the mean density of their lattice neighbours that are fluid in both masks
// (rho_w when there is none; periodic axes wrap, other edges do not count); impulse =
// momentum of the covered nodes minus that of the refilled ones.  -1 (nothing changed)
// for an inadmissible mask or box, or a box added or removed.
int set_mask(Sim3& s, const uint8_t* mask, const int32_t* box, double* impulse) {
  Config3 c = s.cfg;
  if (box) {
    if ((box[0] >= 0) != (c.box[0] >= 0)) return -1;
    for (int k = 0; k < 6; ++k) c.box[k] = box[k];
  }
  if (!config_valid(c, mask)) return -1;
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const size_t n = s.nodes();
  const size_t nrec = s.rec.size() / NREC;
  if (s.cfg.box[0] >= 0 && nrec > 0) {
    std::vector<double> g(s.S.size(), 0.0);
    s.stream_all(s.S, g);
    double J[3];
    s.box_momentum(g, J);
    s.jfix_t.push_back(nrec - 1);
    for (int a = 0; a < 3; ++a) s.jfix.push_back(J[a]);
  }
  const std::vector<uint8_t> old = s.solid;
  double P[3] = {0.0, 0.0, 0.0};
  std::vector<double> fresh(NQ * n, 0.0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t k = s.node(x, y, z);
        if (old[k] == 0 && mask[k] != 0) {  // covered
          for (int i = 0; i < NQ; ++i) {
            P[0] += CX[i] * s.S[s.idx(i, x, y, z)];
            P[1] += CY[i] * s.S[s.idx(i, x, y, z)];
            P[2] += CZ[i] * s.S[s.idx(i, x, y, z)];
          }
        } else if (old[k] != 0 && mask[k] == 0) {  // uncovered
          double rsum = 0.0;
          int cnt = 0;
          for (int i = 1; i < NQ; ++i) {
            int a[3];
            s.shifted(x, y, z, CX[i], CY[i], CZ[i], a);
            if (a[0] < 0 || a[0] >= nx || a[1] < 0 || a[1] >= ny || a[2] < 0 || a[2] >= nz)
              continue;
            const size_t ka = s.node(a[0], a[1], a[2]);
            if (old[ka] != 0 || mask[ka] != 0) continue;
            double r = 0.0;
            for (int j = 0; j < NQ; ++j) r += s.S[s.idx(j, a[0], a[1], a[2])];
            rsum += r;
            ++cnt;
          }
          const double rho = cnt > 0 ? rsum / cnt : c.rho_w;
          const double rr[3] = {x - c.body_c[0], y - c.body_c[1], z - c.body_c[2]};
          const double* W = c.body_omega;
          const double u[3] = {c.body_u[0] + W[1] * rr[2] - W[2] * rr[1],
                               c.body_u[1] + W[2] * rr[0] - W[0] * rr[2],
                               c.body_u[2] + W[0] * rr[1] - W[1] * rr[0]};
          for (int i = 0; i < NQ; ++i) fresh[s.idx(i, x, y, z)] = equilibrium(i, rho, u[0], u[1], u[2]);
        }
      }
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t k = s.node(x, y, z);
        if (!(old[k] != 0 && mask[k] == 0)) continue;
        for (int i = 0; i < NQ; ++i) {
          const double v = fresh[s.idx(i, x, y, z)];
          s.S[s.idx(i, x, y, z)] = v;
          P[0] -= CX[i] * v;
          P[1] -= CY[i] * v;
          P[2] -= CZ[i] * v;
        }
      }
  s.solid.assign(mask, mask + n);
  s.cfg = c;
  if (impulse)
    for (int a = 0; a < 3; ++a) impulse[a] = P[a];
  return 0;
}

}  // namespace

extern "C" {

typedef Config3 orc3_cfg;

void orc3_lattice(int32_t* cx, int32_t* cy, int32_t* cz, int32_t* opp, double* w) {
  for (int i = 0; i < NQ; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    cz[i] = CZ[i];
    opp[i] = opposite(i);
    w[i] = weight(i);
  }
}

void orc3_equilibrium(double rho, double ux, double uy, double uz, double* feq) {
  for (int i = 0; i < NQ; ++i) feq[i] = equilibrium(i, rho, ux, uy, uz);
}

void orc3_collide_node(const double* f, double omega, double gx, double gy, double gz,
                       double* out) {
  const double g[3] = {gx, gy, gz};
  collide_node(f, omega, g, out);
}

void orc3_collide_node_regularized(const double* f, double omega, double* out) {
  collide_node_regularized(f, omega, out);
}

int orc3_box_admissible(const orc3_cfg* c, const uint8_t* mask) {
  return box_admissible(*c, mask) ? 1 : 0;
}

// Body links (node index (z*ny + y)*nx + x, direction) in (z, y, x, i) order; returns
// their number (at most cap are written).
int64_t orc3_links(const orc3_cfg* c, const uint8_t* mask, int64_t* out, int64_t cap) {
  Sim3 s;
  s.cfg = *c;
  s.solid.assign(mask, mask + size_t(c->nx) * c->ny * c->nz);
  int64_t n = 0;
  for (int z = 0; z < c->nz; ++z)
    for (int y = 0; y < c->ny; ++y)
      for (int x = 0; x < c->nx; ++x)
        for (int i = 1; i < NQ; ++i)
          if (s.is_link(x, y, z, i)) {
            if (n < cap) {
              out[2 * n] = int64_t(s.node(x, y, z));
              out[2 * n + 1] = i;
            }
            ++n;
          }
  return n;
}

void* orc3_create(const orc3_cfg* c, const uint8_t* mask, double omega, const double* uin) {
  if (!config_valid(*c, mask)) return nullptr;
  Sim3* s = new Sim3();
  s->cfg = *c;
  const size_t n = size_t(c->nx) * c->ny * c->nz;
  s->solid.assign(mask, mask + n);
  s->uin.assign(size_t(c->ny) * c->nz, 0.0);
  if (uin)
    for (size_t k = 0; k < s->uin.size(); ++k) s->uin[k] = uin[k];
  s->omega = omega;
  s->S.assign(NQ * n, 0.0);
  for (int i = 0; i < NQ; ++i)
    for (size_t k = 0; k < n; ++k) s->S[size_t(i) * n + k] = weight(i);
  s->f = s->S;
  s->Sn = s->S;
  return s;
}

void orc3_destroy(void* h) { delete static_cast<Sim3*>(h); }

int orc3_set_mask(void* h, const uint8_t* mask, const int32_t* box, double* impulse) {
  return set_mask(*static_cast<Sim3*>(h), mask, box, impulse);
}

void orc3_set_body_motion(void* h, const double* u, const double* w, const double* c) {
  Config3& cfg = static_cast<Sim3*>(h)->cfg;
  for (int a = 0; a < 3; ++a) {
    cfg.body_u[a] = u[a];
    cfg.body_omega[a] = w[a];
    cfg.body_c[a] = c[a];
  }
}

void orc3_set_state(void* h, const double* S) {
  Sim3* s = static_cast<Sim3*>(h);
  std::memcpy(s->S.data(), S, s->S.size() * sizeof(double));
}

void orc3_get_state(void* h, double* S) {
  Sim3* s = static_cast<Sim3*>(h);
  std::memcpy(S, s->S.data(), s->S.size() * sizeof(double));
}

void orc3_get_pre(void* h, double* f) {
  Sim3* s = static_cast<Sim3*>(h);
  std::memcpy(f, s->f.data(), s->f.size() * sizeof(double));
}

void orc3_step(void* h, int32_t n) {
  Sim3* s = static_cast<Sim3*>(h);
  for (int32_t k = 0; k < n; ++k) s->step();
}

int64_t orc3_nrec(void* h) { return int64_t(static_cast<Sim3*>(h)->rec.size() / NREC); }

void orc3_records(void* h, double* out) {
  Sim3* s = static_cast<Sim3*>(h);
  std::memcpy(out, s->rec.data(), s->rec.size() * sizeof(double));
}

void orc3_forces(void* h, double* out) { static_cast<Sim3*>(h)->forces(out); }

void orc3_momentum_of(void* h, const double* g, double* J) {
  Sim3* s = static_cast<Sim3*>(h);
  std::vector<double> v(g, g + s->S.size());
  s->box_momentum(v, J);
}

}  // extern "C"
