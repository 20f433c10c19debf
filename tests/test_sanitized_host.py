"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (g++, CPU only):
the library's planning (plan.cpp, plan3.cpp, including the incremental re-planning of
a mask change, checked against a fresh plan of the new mask) and both oracles
(lbm_oracle.cpp, lbm3d_oracle.cpp: steps, forces, mask changes, the boundary pressure
coefficient, complex-step objective).  Any invalid access, leak or undefined operation
aborts the driver."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2210_10377_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]

PLAN_DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>
#include "plan.h"
#include "plan3.h"

static int fail(const char* what, int seed) { std::printf("mismatch %s seed %d\n", what, seed); return 1; }

static bool same2(const lbm::Plan& a, const lbm::Plan& b) {
  return a.node == b.node && a.links == b.links && a.strip_slot == b.strip_slot &&
         a.gx0 == b.gx0 && a.gx1 == b.gx1 && a.gy0 == b.gy0 && a.gy1 == b.gy1 &&
         a.nslots == b.nslots && a.njslots == b.njslots && a.ngeneral == b.ngeneral &&
         a.n_fluid == b.n_fluid && a.n_box == b.n_box && a.tile_rows == b.tile_rows;
}

static void blob(std::vector<uint8_t>& m, int nx, int ny, std::mt19937& r, int x0, int x1, int y0, int y1) {
  std::uniform_int_distribution<int> ux(x0, x1), uy(y0, y1), us(0, 3);
  const int cx = ux(r), cy = uy(r), s = us(r);
  for (int y = cy - s; y <= cy + s; ++y)
    for (int x = cx - s; x <= cx + s; ++x)
      if (x >= x0 && x <= x1 && y >= y0 && y <= y1) m[size_t(y) * nx + x] = 1;
}

int main() {
  // Two dimensions: random grids, boundaries, bodies inside a box, tile shapes; a chain
  // of mask changes re-planned incrementally and compared with fresh plans.
  for (int seed = 0; seed < 60; ++seed) {
    std::mt19937 r(seed);
    const int nx = 12 + int(r() % 300), ny = 12 + int(r() % 60);
    lbm_grid g{};
    g.nx = nx; g.ny = ny; g.bc_x = int(r() % 2); g.bc_y = int(r() % 2);
    g.precision = LBM_FP32; g.max_record = 4; g.rho_ref = g.u_ref = g.l_ref = 1.0;
    g.tile = int(r() % 3);
    const bool box = r() % 2;
    const int bx0 = 2, bx1 = nx - 2, by0 = 2, by1 = ny - 2;
    g.box[0] = box ? bx0 : -1; g.box[1] = bx1; g.box[2] = by0; g.box[3] = by1;
    std::vector<uint8_t> m(size_t(nx) * ny, 0);
    for (int k = 0; k < 3; ++k) blob(m, nx, ny, r, bx0 + 2, bx1 - 3, by0 + 2, by1 - 3);
    lbm::Plan p;
    std::string err;
    if (lbm::build_plan(g, m.data(), p, err) != LBM_OK) return fail(err.c_str(), seed);
    for (int change = 0; change < 6; ++change) {
      std::vector<uint8_t> m2 = m;
      for (auto& v : m2) v = 0;
      for (int k = 0; k < 3; ++k) blob(m2, nx, ny, r, bx0 + 2, bx1 - 3, by0 + 2, by1 - 3);
      if (change == 5) m2[0] = 1;  // a solid node outside the box: refused when boxed
      std::vector<int32_t> changed;
      for (size_t k = 0; k < m.size(); ++k)
        if ((m[k] != 0) != (m2[k] != 0)) changed.push_back(int32_t(k));
      lbm::Plan np, fresh;
      lbm::PlanDelta d;
      const std::vector<uint32_t> before = p.node;
      const int rc = lbm::replan(g, m2.data(), changed, p, np, d, err);
      const int rf = lbm::build_plan(g, m2.data(), fresh, err);
      if ((rc == LBM_OK) != (rf == LBM_OK)) return fail("replan status", seed);
      if (rc != LBM_OK) {
        if (p.node != before) return fail("refused replan changed the plan", seed);
        continue;
      }
      if (!same2(np, fresh)) return fail("replan vs fresh 2-D", seed);
      p = std::move(np);
      m = m2;
    }
  }
  // Three dimensions: the same for D3Q27 plans.
  for (int seed = 0; seed < 30; ++seed) {
    std::mt19937 r(1000 + seed);
    const int nx = 10 + int(r() % 40), ny = 10 + int(r() % 12), nz = 10 + int(r() % 10);
    lbm3d_grid g{};
    g.nx = nx; g.ny = ny; g.nz = nz; g.bc_x = int(r() % 2); g.bc_y = int(r() % 2); g.bc_z = int(r() % 2);
    g.precision = LBM_FP32; g.max_record = 4;
    const bool box = r() % 2;
    g.box[0] = box ? 2 : -1; g.box[1] = nx - 2; g.box[2] = 2; g.box[3] = ny - 2; g.box[4] = 2; g.box[5] = nz - 2;
    auto make = [&](std::mt19937& q) {
      std::vector<uint8_t> m(size_t(nx) * ny * nz, 0);
      std::uniform_int_distribution<int> ux(4, nx - 5), uy(4, ny - 5), uz(4, nz - 5);
      for (int k = 0; k < 2; ++k) {
        const int cx = ux(q), cy = uy(q), cz = uz(q);
        for (int z = cz - 1; z <= cz + 1; ++z)
          for (int y = cy - 1; y <= cy + 1; ++y)
            for (int x = cx - 1; x <= cx + 1; ++x) m[(size_t(z) * ny + y) * nx + x] = 1;
      }
      return m;
    };
    std::vector<uint8_t> m = make(r);
    lbm3::Plan3 p;
    std::string err;
    if (lbm3::build_plan3(g, m.data(), p, err) != LBM_OK) return fail(err.c_str(), seed);
    for (int change = 0; change < 4; ++change) {
      std::vector<uint8_t> m2 = make(r);
      std::vector<int32_t> changed;
      for (size_t k = 0; k < m.size(); ++k)
        if ((m[k] != 0) != (m2[k] != 0)) changed.push_back(int32_t(k));
      lbm3::Plan3 np, fresh;
      lbm3::Plan3Delta d;
      const int rc = lbm3::replan3(g, m2.data(), changed, p, np, d, err);
      const int rf = lbm3::build_plan3(g, m2.data(), fresh, err);
      if ((rc == LBM_OK) != (rf == LBM_OK)) return fail("replan3 status", seed);
      if (rc != LBM_OK) continue;
      std::vector<int64_t> la, lb;
      lbm3::plan3_links(np, la);
      lbm3::plan3_links(fresh, lb);
      if (np.word != fresh.word || np.strip != fresh.strip || np.fstrips != fresh.fstrips ||
          la != lb || np.nslots != fresh.nslots || np.njslots != fresh.njslots)
        return fail("replan3 vs fresh", seed);
      p = std::move(np);
      m = m2;
    }
  }
  std::printf("ok\n");
  return 0;
}
'''

ORACLE_DRIVER = r'''
#include <complex>
#include <cstdint>
#include <cstdio>
#include <vector>
extern "C" {
struct Cfg { int32_t nx, ny, bc_x, bc_y; int32_t box[4]; double rho_w, gx, gy; int32_t collision;
             double body_u[2]; double body_omega; double body_c[2]; };
void* orc_create(const Cfg*, const uint8_t*, double, const double*);
void orc_destroy(void*);
void orc_step(void*, int32_t);
int64_t orc_nrec(void*);
void orc_forces(void*, double*);
int orc_set_mask(void*, const uint8_t*, const int32_t*, double*);
int64_t orc_boundary_cp(void*, int32_t, int32_t, double, double, int32_t*, double*, int64_t);
int orc_objective_cs(const Cfg*, const uint8_t*, double, double, const double*, const double*,
                     int32_t, int32_t, int32_t, double, double, double*);
int32_t orc_set_threads(int32_t);
}
static std::vector<uint8_t> disk(int nx, int ny, int cx, int cy, int r) {
  std::vector<uint8_t> m(size_t(nx) * ny, 0);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) m[size_t(y) * nx + x] = (x - cx) * (x - cx) + (y - cy) * (y - cy) <= r * r;
  return m;
}
int main() {
  const int nx = 60, ny = 30;
  for (int coll = 0; coll < 3; ++coll)
    for (int threads : {1, 3}) {
      orc_set_threads(threads);
      Cfg c{nx, ny, 0, 0, {8, 40, 4, 26}, 1.0, 0.0, 0.0, coll, {0, 0}, 0.0, {0, 0}};
      std::vector<uint8_t> m = disk(nx, ny, 20, 15, 4);
      std::vector<double> uin(ny, 0.04);
      void* h = orc_create(&c, m.data(), 1.0 / 0.7, uin.data());
      if (!h) return 1;
      orc_step(h, 20);
      std::vector<double> F(size_t(orc_nrec(h)) * 10);
      orc_forces(h, F.data());
      std::vector<uint8_t> m2 = disk(nx, ny, 22, 15, 4);
      double imp[2];
      if (orc_set_mask(h, m2.data(), nullptr, imp) != 0) return 2;
      orc_step(h, 5);
      std::vector<int32_t> nodes(400);
      std::vector<double> cp(400);
      if (orc_boundary_cp(h, 2, 15, 1.0, 0.04, nodes.data(), cp.data(), 400) <= 0) return 3;
      orc_destroy(h);
    }
  Cfg c{40, 20, 0, 0, {-1, -1, -1, -1}, 1.0, 0.0, 0.0, 0, {0, 0}, 0.0, {0, 0}};
  std::vector<uint8_t> m = disk(40, 20, 12, 10, 3);
  std::vector<double> ure(20, 0.03), uim(20, 1e-30);
  double out[2];
  if (orc_objective_cs(&c, m.data(), 1.0 / 0.8, 0.0, ure.data(), uim.data(), 30, 10, 20, 1.0, 0.0, out) != 0) return 4;
  std::printf("ok\n");
  return 0;
}
'''

ORACLE3_DRIVER = r'''
#include <cstdint>
#include <cstdio>
#include <vector>
extern "C" {
struct Cfg3 { int32_t nx, ny, nz, bc_x, bc_y, bc_z; int32_t box[6]; double rho_w; double g[3];
              int32_t collision; double body_u[3]; double body_omega[3]; double body_c[3]; };
void* orc3_create(const Cfg3*, const uint8_t*, double, const double*);
void orc3_destroy(void*);
void orc3_step(void*, int32_t);
int64_t orc3_nrec(void*);
void orc3_forces(void*, double*);
int orc3_set_mask(void*, const uint8_t*, const int32_t*, double*);
}
int main() {
  const int nx = 24, ny = 12, nz = 10;
  for (int coll = 0; coll < 2; ++coll) {
    Cfg3 c{nx, ny, nz, 0, 0, 1, {4, 16, 2, 10, 0, nz}, 1.0, {0, 0, 0}, coll, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    std::vector<uint8_t> m(size_t(nx) * ny * nz, 0), m2;
    for (int z = 0; z < nz; ++z)
      for (int y = 5; y <= 6; ++y)
        for (int x = 8; x <= 9; ++x) m[(size_t(z) * ny + y) * nx + x] = 1;
    m2 = m;
    for (int z = 0; z < nz; ++z) m2[(size_t(z) * ny + 5) * nx + 10] = 1;
    std::vector<double> uin(size_t(ny) * nz, 0.03);
    void* h = orc3_create(&c, m.data(), 1.0 / 0.75, uin.data());
    if (!h) return 1;
    orc3_step(h, 6);
    double imp[3];
    if (orc3_set_mask(h, m2.data(), nullptr, imp) != 0) return 2;
    orc3_step(h, 3);
    std::vector<double> F(size_t(orc3_nrec(h)) * 12);
    orc3_forces(h, F.data());
    orc3_destroy(h);
  }
  std::printf("ok\n");
  return 0;
}
'''


def _build_and_run(tmp_path, name, driver, sources, extra=()):
    src = tmp_path / f"{name}.cpp"
    src.write_text(driver)
    exe = tmp_path / name
    cmd = ["g++", "-std=c++17", "-O1", "-g", *SAN, *extra, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, str(src), *sources, "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0 and "ok" in out.stdout, (out.stdout[-2000:], out.stderr[-4000:])


def test_planning_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "plan_driver", PLAN_DRIVER,
                   [os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "plan3.cpp")])


def test_oracles_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "oracle_driver", ORACLE_DRIVER,
                   [os.path.join(ROOT, "oracle", "lbm_oracle.cpp")], extra=["-fopenmp"])
    _build_and_run(tmp_path, "oracle3_driver", ORACLE3_DRIVER,
                   [os.path.join(ROOT, "oracle", "lbm3d_oracle.cpp")])
