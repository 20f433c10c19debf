"""Pins of the three-dimensional oracle (D3Q27) against what the mathematics fixes:
exact weights and lattice isotropy, equilibrium moments, collision invariants, brute-force
streaming, the exact reduction to the (separately pinned) two-dimensional oracle for
span-invariant flows, Newton's law for the fluid, DRTT = MEA-B around a sphere, the
exact Poiseuille profile between walls in z, and symmetry."""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import d3q27 as D
from oracle import BCX_INLET_OUTLET, BCX_PERIODIC, BCY_PERIODIC, BCY_WALL, OracleSim
from workloads import d3


@pytest.fixture(scope="module")
def lat():
    return D.lattice()


def test_velocity_set_and_exact_weights(lat):
    """The 27 velocities are {-1, 0, 1}^3, each once, numbered as the population
    arrays are laid out; the weights by shell are 8/27, 2/27, 1/54, 1/216 exactly;
    opposite pairs are consecutive (2k-1, 2k)."""
    cx, cy, cz, opp, w = lat
    vel = set(zip(cx.tolist(), cy.tolist(), cz.tolist()))
    assert len(vel) == 27 and vel == {(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1)
                                      for c in (-1, 0, 1)}
    assert (cx[0], cy[0], cz[0]) == (0, 0, 0)
    faces = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    assert list(zip(cx[1:7], cy[1:7], cz[1:7])) == faces
    shell = {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54), 3: Fraction(1, 216)}
    for i in range(27):
        k = abs(cx[i]) + abs(cy[i]) + abs(cz[i])
        assert w[i] == float(shell[k])
        assert (cx[opp[i]], cy[opp[i]], cz[opp[i]]) == (-cx[i], -cy[i], -cz[i])
        if i:
            assert opp[i] == (i + 1 if i % 2 else i - 1)
    assert sum(Fraction(w[i]).limit_denominator(1000) for i in range(27)) == 1


def test_lattice_isotropy_to_fourth_order(lat):
    """sum w = 1, sum w c_a c_b = theta0 delta_ab, odd moments vanish, and
    sum w c_a c_b c_c c_d = theta0^2 (delta delta + delta delta + delta delta)."""
    cx, cy, cz, _, w = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    th = 1.0 / 3.0
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia->a", w, C), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, C, C), th * d, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, C, C, C), 0, atol=1e-16)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, C, C, C, C)
    iso = th * th * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                     + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(M4, iso, atol=1e-16)


def test_equilibrium_moments(lat):
    cx, cy, cz, _, w = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    rho, u = 1.07, np.array([0.03, -0.05, 0.02])
    feq = D.equilibrium(rho, *u)
    assert abs(feq.sum() - rho) < 1e-15
    np.testing.assert_allclose(C.T @ feq, rho * u, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", feq, C, C),
                               rho * np.outer(u, u) + rho / 3 * np.eye(3), atol=1e-15)
    np.testing.assert_allclose(D.equilibrium(1.0, 0, 0, 0), w, atol=0)


def test_collision_invariants_and_relaxation(lat):
    cx, cy, cz, _, w = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    f = d3.near_rest_state3(1, 1, 1, seed=3, amp=0.2)[:, 0, 0, 0]
    for om in (0.6, 1.0, 1.7):
        out = D.collide_node(f, om)
        assert abs(out.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ out, C.T @ f, atol=1e-16)
    rho = f.sum()
    u = C.T @ f / rho
    np.testing.assert_allclose(D.collide_node(f, 1.0), D.equilibrium(rho, *u), atol=1e-16)
    g = np.array([1e-4, -2e-4, 3e-4])
    np.testing.assert_allclose(C.T @ D.collide_node(f, 0.8, g), C.T @ f + g, atol=1e-16)


def test_pure_streaming_of_single_populations(lat):
    """omega = 0 on a fully periodic 7x6x5 lattice: one marked population per direction
    moves by c_i per step and wraps."""
    cx, cy, cz, _, _ = lat
    nx, ny, nz = 7, 6, 5
    S = np.ones((27, nz, ny, nx))      # a background keeps rho > 0 at every node
    x0, y0, z0 = 3, 2, 1
    S[:, z0, y0, x0] = 2.0
    s = D.OracleSim3(np.zeros((nz, ny, nx), np.uint8), omega=0.0, bc_x=BCX_PERIODIC,
                     bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC)
    s.set_state(S)
    s.step(3)
    T = s.state()
    for i in range(27):
        x, y, z = (x0 + 3 * cx[i]) % nx, (y0 + 3 * cy[i]) % ny, (z0 + 3 * cz[i]) % nz
        assert T[i, z, y, x] == 2.0 and T[i].sum() == nx * ny * nz + 1


def test_body_bounce_back_and_links_brute_force(lat):
    """A single solid node in a periodic lattice: 26 links, one from each neighbour
    towards it, and the population sent at it comes back reversed after one step."""
    cx, cy, cz, opp, _ = lat
    nx, ny, nz = 6, 6, 6
    m = np.zeros((nz, ny, nx), np.uint8)
    m[3, 3, 3] = 1
    L = D.links(m, bc_x=BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC)
    expect = sorted(((((3 - cz[i]) * ny + 3 - cy[i]) * nx + 3 - cx[i]), i) for i in range(1, 27))
    assert sorted(map(tuple, L.tolist())) == expect
    S = np.ones((27, nz, ny, nx))
    i = 19
    S[i, 3 - cz[i], 3 - cy[i], 3 - cx[i]] = 2.0
    s = D.OracleSim3(m, omega=0.0, bc_x=BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC)
    s.set_state(S)
    s.step(1)
    assert s.pre()[opp[i], 3 - cz[i], 3 - cy[i], 3 - cx[i]] == 2.0


def _marginal(S3, lat):
    """Sum over c_z of a [27, ...] field, in the two-dimensional direction order."""
    cx, cy, cz, _, _ = lat
    order2 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    out = np.zeros((9,) + S3.shape[1:])
    for i in range(27):
        out[order2.index((cx[i], cy[i]))] += S3[i]
    return out


@pytest.mark.parametrize("collision", ["bgk", "regularized"])
@pytest.mark.parametrize("bcx", [BCX_INLET_OUTLET, BCX_PERIODIC])
def test_span_invariant_flow_reduces_to_the_two_dimensional_oracle(lat, bcx, collision):
    """An extruded body in a lattice periodic across the span, started from a
    span-invariant state: the z-marginal of the D3Q27 state equals the D2Q9 oracle's
    state, and the x, y forces of every estimator equal nz times the two-dimensional ones
    (DRTT with a box spanning the whole span), the z forces vanish."""
    cx, cy, cz, _, _ = lat
    nx, ny, nz = 60, 26, 4
    m2 = workloads.cylinder_mask(nx, ny, 20, 12.5, 5)
    box2 = (10, 31, 4, 22)
    uin = None if bcx == BCX_PERIODIC else np.linspace(0.5, 1.0, ny) * 0.04
    S2 = workloads.near_rest_state(nx, ny, seed=9, amp=0.05)
    # a span-invariant 3-D state whose marginal is S2: split each 2-D population over
    # c_z in fixed proportions
    frac = {0: 2 / 3, 1: 1 / 6, -1: 1 / 6}
    order2 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    S3 = np.zeros((27, nz, ny, nx))
    for i in range(27):
        S3[i] = frac[cz[i]] * S2[order2.index((cx[i], cy[i]))][None]
    o2 = OracleSim(m2, tau=0.7, uin=uin, bc_x=bcx, bc_y=BCY_WALL, box=box2,
                   collision=collision)
    o2.set_state(S2)
    o3 = D.OracleSim3(d3.extrude(m2, nz), tau=0.7,
                      uin=None if uin is None else np.broadcast_to(uin, (nz, ny)),
                      bc_x=bcx, bc_y=D.BC_WALL, bc_z=D.BC_PERIODIC,
                      box=box2 + (0, nz), collision=collision)
    o3.set_state(S3)
    o2.step(25)
    o3.step(25)
    np.testing.assert_allclose(_marginal(o3.state(), lat)[:, 0], o2.state(), rtol=0, atol=1e-14)
    F2, F3 = o2.forces(), o3.forces()
    scale = np.abs(F2).max()
    np.testing.assert_allclose(F3[:, :, :2], nz * F2[:, :4], rtol=0, atol=1e-12 * nz * scale)
    assert np.abs(F3[:, :, 2]).max() <= 1e-13 * nz * scale


def test_newtons_law_for_the_fluid_pins_mea_b(lat):
    """Fully periodic lattice with a sphere and a uniform body force g: the total fluid
    momentum (pre-collision) obeys P(t+1) = P(t) + N g - F_B(t) at every step."""
    cx, cy, cz, _, _ = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    nx, ny, nz = 20, 18, 16
    m = d3.sphere_mask(nx, ny, nz, 9.5, 8.7, 7.9, 4.2)
    g = np.array([2e-5, -1e-5, 5e-6])
    s = D.OracleSim3(m, tau=0.8, bc_x=BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC,
                     g=g)
    s.set_state(d3.near_rest_state3(nx, ny, nz, seed=2, amp=0.02))
    fl = m == 0
    N = fl.sum()
    P = []
    for _ in range(12):
        s.step(1)
        P.append(np.einsum("ia,i...->a...", C, s.pre())[:, fl].sum(1))
    FB = s.forces()[:, 1]
    for t in range(11):
        np.testing.assert_allclose(P[t + 1], P[t] + N * g - FB[t], rtol=0, atol=1e-12)
    assert np.abs(FB).max() > 1e-4


def test_drtt_equals_mea_b_around_a_sphere_for_two_boxes(lat):
    """Inlet/outlet duct with walls in y and z and a sphere: DRTT equals MEA-B at every
    step for two different admissible boxes; A differs from B."""
    w = d3.sphere_channel_64x32x32()
    Fs, Js = [], []
    for box in (w.box, (10, 40, 5, 27, 4, 28)):
        s = D.OracleSim3(w.mask, tau=w.tau, uin=w.uin, box=box)
        s.step(60)
        Fs.append(s.forces())
        Js.append(np.abs(s.records()[:, 6:9]).max())
    # DRTT is a difference of box momenta of order |J| (~1e4 nodes): rounding 1e-13 |J|
    for F, J in zip(Fs, Js):
        scale = np.abs(F[:, 1]).max()
        assert scale > 0
        assert np.abs(F[:, 2] - F[:, 1]).max() <= 1e-12 * J
        assert np.abs(F[:, 0] - F[:, 1]).max() > 1e-3 * scale
    np.testing.assert_allclose(Fs[0][:, 2], Fs[1][:, 2], rtol=0, atol=1e-12 * max(Js))


def test_symmetric_sphere_has_no_side_forces():
    """A sphere centred in a square duct (mirror-symmetric in y and z) with a uniform
    inlet: lift and side force vanish for every estimator, drag is positive."""
    nx, ny, nz = 48, 24, 24
    m = d3.sphere_mask(nx, ny, nz, 16, 11.5, 11.5, 4.5)
    s = D.OracleSim3(m, tau=0.7, uin=np.full((nz, ny), 0.04), box=d3.default_box3(m, 3))
    s.step(150)
    F = s.forces()
    drag = np.abs(F[:, :, 0]).max()
    assert np.abs(F[:, :, 1:]).max() <= 1e-12 * drag
    assert np.all(F[-20:, 1, 0] > 0)


def test_poiseuille_between_walls_in_z_is_exact_at_the_magic_tau():
    """Plane Poiseuille flow driven by g along x between no-slip walls at z = -1/2 and
    nz - 1/2 (periodic x and y): at (tau - 1/2)^2 = 3/16 half-way bounce-back gives the
    parabola u(z) = g/(2 nu) (z + 1/2)(nz - 1/2 - z) exactly at steady state."""
    nx, ny, nz = 4, 3, 12
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    g = 1e-6
    s = D.OracleSim3(np.zeros((nz, ny, nx), np.uint8), tau=tau, bc_x=BCX_PERIODIC,
                     bc_y=D.BC_PERIODIC, bc_z=D.BC_WALL, g=(g, 0.0, 0.0))
    s.step(6000)
    S = s.pre()          # velocity from the pre-collision populations (Guo forcing)
    cx, _, _, _, _ = D.lattice()
    rho = S.sum(0)
    u = (np.tensordot(cx.astype(float), S, 1) + 0.5 * g) / rho
    z = np.arange(nz)
    exact = g / (2 * nu) * (z + 0.5) * (nz - 0.5 - z)
    np.testing.assert_allclose(u[:, 1, 2], exact, rtol=1e-9)
    assert np.abs(u - u[:, :1, :1]).max() < 1e-15


def test_uniform_flow_through_inlet_and_outlet_is_a_fixed_point():
    """f^eq(1, (U, 0, 0)) everywhere in a duct periodic in y and z with the moving-wall
    inlet at velocity U and the zero-gradient outlet stays exactly as it is."""
    nx, ny, nz = 10, 5, 4
    U = 0.05
    feq = D.equilibrium(1.0, U, 0.0, 0.0)
    S0 = np.broadcast_to(feq[:, None, None, None], (27, nz, ny, nx)).copy()
    s = D.OracleSim3(np.zeros((nz, ny, nx), np.uint8), tau=0.6, uin=np.full((nz, ny), U),
                     bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC)
    s.set_state(S0)
    s.step(5)
    np.testing.assert_allclose(s.state(), S0, rtol=0, atol=2e-16)


def test_box_admissibility_per_axis():
    """A box may span a whole periodic axis (an extruded body through it); along a
    bounded axis it must lie one node inside with the body strictly inside."""
    nx, ny, nz = 40, 20, 8
    m = d3.extrude(workloads.cylinder_mask(nx, ny, 15, 9.5, 4), nz)
    kw = dict(bc_y=D.BC_WALL, bc_z=D.BC_PERIODIC)
    assert D.box_admissible(m, (5, 26, 2, 18, 0, nz), **kw)
    assert not D.box_admissible(m, (5, 26, 2, 18, 1, nz - 1), **kw)
    assert not D.box_admissible(m, (5, 26, 2, 18, 0, nz), bc_y=D.BC_WALL, bc_z=D.BC_WALL)
    assert not D.box_admissible(m, (0, 26, 2, 18, 0, nz), **kw)
    assert not D.box_admissible(m, (5, 26, 6, 18, 0, nz), **kw)


# --------------------------------------------------------------------------------------
# Regularized BGK in three dimensions (not in the paper; the stabilized variant for
# tau_lb close to 1/2).  The span-invariant reduction above covers it as well.
# --------------------------------------------------------------------------------------

def _moments(f, C):
    rho = f.sum()
    u = C.T @ f / rho
    return rho, u


def _pi_neq(f, C):
    rho, u = _moments(f, C)
    neq = f - D.equilibrium(rho, *u)
    return np.einsum("i,ia,ib->ab", neq, C, C)


def test_regularized_conserves_and_relaxes_the_stress_exactly(lat):
    """Mass and momentum are conserved and the non-equilibrium stress is multiplied by
    exactly (1 - omega): the Hermite projection keeps the second moment."""
    cx, cy, cz, _, _ = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    f = d3.near_rest_state3(1, 1, 1, seed=6, amp=0.3)[:, 0, 0, 0]
    for om in (0.7, 1.3, 1.95):
        out = D.collide_node(f, om, collision="regularized")
        assert abs(out.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ out, C.T @ f, atol=1e-16)
        np.testing.assert_allclose(_pi_neq(out, C), (1 - om) * _pi_neq(f, C), atol=1e-15)


def test_regularized_equals_bgk_for_second_order_and_removes_ghosts(lat):
    """With a non-equilibrium part that is purely second order the regularized step is
    the BGK step; a ghost mode (no mass, momentum or stress) is removed entirely by it
    and only relaxed by BGK."""
    cx, cy, cz, _, w = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    rho, u = 1.02, np.array([0.03, -0.01, 0.02])
    feq = D.equilibrium(rho, *u)
    Pi = np.array([[2e-3, 5e-4, -3e-4], [5e-4, -1e-3, 7e-4], [-3e-4, 7e-4, -1e-3]])
    Q = np.einsum("ia,ib->iab", C, C) - np.eye(3) / 3
    f1 = w * 4.5 * np.einsum("iab,ab->i", Q, Pi)
    f = feq + f1
    np.testing.assert_allclose(D.collide_node(f, 1.4, collision="regularized"),
                               D.collide_node(f, 1.4), rtol=0, atol=3e-16)
    # a ghost: the product c_x c_y c_z weighted to kill every moment up to second order
    g = w * cx * cy * cz * 1e-3
    assert abs(g.sum()) < 1e-18 and np.abs(C.T @ g).max() < 1e-18
    assert np.abs(np.einsum("i,ia,ib->ab", g, C, C)).max() < 1e-18
    np.testing.assert_allclose(D.collide_node(feq + g, 1.4, collision="regularized"), feq,
                               rtol=0, atol=3e-16)
    np.testing.assert_allclose(D.collide_node(feq + g, 1.4), feq + (1 - 1.4) * g,
                               rtol=0, atol=3e-16)


# --------------------------------------------------------------------------------------
# Bodies in rigid motion in three dimensions (moving-wall bounce-back of Sec. II at the
# half-way point of every body link; Eq. rtt4/rtt5 and DRTT with moving walls)
# --------------------------------------------------------------------------------------

def test_comoving_body_in_a_uniform_flow_is_a_fixed_point():
    """A sphere translating with a uniform flow f^eq(1, U) on a periodic lattice: the
    state stays the equilibrium and no estimator sees a force."""
    nx, ny, nz = 24, 20, 18
    U = (0.03, -0.02, 0.01)
    m = d3.sphere_mask(nx, ny, nz, 11.5, 9.5, 8.5, 4.5)
    feq = D.equilibrium(1.0, *U)
    S0 = np.broadcast_to(feq[:, None, None, None], (27, nz, ny, nx)).copy()
    s = D.OracleSim3(m, tau=0.7, bc_x=BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC,
                     box=(3, 21, 3, 17, 2, 16), body_motion=(U, (0, 0, 0), (0, 0, 0)))
    s.set_state(S0)
    s.step(8)
    fl = m == 0
    np.testing.assert_allclose(s.state()[:, fl], S0[:, fl], rtol=0, atol=1e-14)
    F = s.forces()
    assert np.abs(F[:, [0, 1, 3]]).max() <= 1e-13
    assert np.abs(F[:, 2]).max() <= 1e-12


def test_moving_wall_rule_on_body_links_brute_force(lat):
    """A single solid node turning about an axis through a nearby point and translating:
    the population entering each neighbour from it is the neighbour's opposite
    population plus 2 w_i rho_w (c_i . u_w) / c_s^2, u_w = U + Omega x (x_w - c) at the
    link's half-way point."""
    cx, cy, cz, opp, w = lat
    nx, ny, nz = 8, 8, 8
    m = np.zeros((nz, ny, nx), np.uint8)
    m[4, 4, 4] = 1
    U, W, X = np.array([0.01, -0.02, 0.005]), np.array([0.003, -0.002, 0.004]), np.array([3.0, 5.0, 2.0])
    S = d3.near_rest_state3(nx, ny, nz, seed=12, amp=0.1)
    s = D.OracleSim3(m, tau=0.8, bc_x=BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC,
                     body_motion=(U, W, X))
    s.set_state(S)
    s.step(1)
    f = s.pre()
    for i in range(1, 27):
        x, y, z = 4 + cx[i], 4 + cy[i], 4 + cz[i]   # pulls direction i from the solid node
        xw = np.array([x, y, z]) - 0.5 * np.array([cx[i], cy[i], cz[i]])
        uw = U + np.cross(W, xw - X)
        expect = S[opp[i], z, y, x] + 2 * w[i] * (cx[i] * uw[0] + cy[i] * uw[1] + cz[i] * uw[2]) * 3
        assert abs(f[i, z, y, x] - expect) <= 1e-16


def test_rotating_sphere_mirror_symmetry_and_magnus_sign():
    """A sphere on the axis of a square duct turning about z: reversing the rotation
    mirrors the flow in y, so drag is unchanged and the y-force changes sign; with the
    flow along +x a counter-clockwise turn (Omega_z > 0) gives a negative y-force
    (Magnus); the z-force vanishes; DRTT equals MEA-B with moving walls."""
    nx, ny, nz = 40, 21, 21
    m = d3.sphere_mask(nx, ny, nz, 12, 10, 10, 3.5)
    box = d3.default_box3(m, 3)
    F = {}
    for om in (0.006, -0.006):
        s = D.OracleSim3(m, tau=0.65, uin=np.full((nz, ny), 0.04), box=box,
                         body_motion=((0, 0, 0), (0, 0, om), (12, 10, 10)))
        s.step(300)
        F[om] = s.forces()
    a, b = F[0.006], F[-0.006]
    scale = np.abs(a[:, 1]).max()
    np.testing.assert_allclose(a[:, :, 0], b[:, :, 0], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(a[:, :, 1], -b[:, :, 1], rtol=0, atol=1e-12 * scale)
    assert a[-100:, 1, 1].mean() < 0
    assert np.abs(a[:, :, 2]).max() <= 1e-12 * scale
    assert np.abs(a[:, 2] - a[:, 1]).max() <= 1e-11 * scale


def test_rotating_extruded_cylinder_reduces_to_the_two_dimensional_oracle(lat):
    """An extruded cylinder turning about an axis along z and sliding in x-y, on a
    lattice periodic across the span: every estimator's x, y forces are nz times those
    of the two-dimensional oracle with the same motion, and the z-marginal of the state
    is its state."""
    cx, cy, cz, _, _ = lat
    nx, ny, nz = 56, 24, 4
    m2 = workloads.cylinder_mask(nx, ny, 20, 11.5, 5)
    box2 = (10, 31, 3, 21)
    uin = np.full(ny, 0.03)
    mo2 = (0.01, -0.005, 0.004, 20.0, 11.5)
    o2 = OracleSim(m2, tau=0.7, uin=uin, bc_y=BCY_WALL, box=box2, body_motion=mo2)
    o3 = D.OracleSim3(d3.extrude(m2, nz), tau=0.7, uin=np.broadcast_to(uin, (nz, ny)),
                      bc_z=D.BC_PERIODIC, box=box2 + (0, nz),
                      body_motion=((0.01, -0.005, 0.0), (0.0, 0.0, 0.004), (20.0, 11.5, 1.3)))
    o2.step(30)
    o3.step(30)
    np.testing.assert_allclose(_marginal(o3.state(), lat)[:, 0], o2.state(), rtol=0, atol=1e-14)
    F2, F3 = o2.forces(), o3.forces()
    scale = np.abs(F2).max()
    np.testing.assert_allclose(F3[:, :, :2], nz * F2[:, :4], rtol=0, atol=1e-12 * nz * scale)


# --------------------------------------------------------------------------------------
# A body moving through the grid in three dimensions (mask replaced between steps)
# --------------------------------------------------------------------------------------

def test_set_mask_same_mask_changes_nothing_3d():
    w = d3.sphere_channel_64x32x32()
    S0 = d3.near_rest_state3(w.nx, w.ny, w.nz, seed=3, amp=0.03)
    runs = []
    for call in (False, True):
        s = D.OracleSim3(w.mask, tau=w.tau, uin=w.uin, box=w.box)
        s.set_state(S0)
        s.step(6)
        if call:
            before = s.state()
            assert np.all(s.set_mask(w.mask.copy()) == 0.0)
            assert np.array_equal(s.state(), before)
        s.step(6)
        runs.append((s.state(), s.forces()))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


def test_uncovered_nodes_refill_brute_force_3d(lat):
    """A 2x2x2 cube moved one node along +x and a 3x3x3 cube removed, on a periodic
    lattice, with a turning, sliding body: every uncovered node holds f^eq(rho, u_w),
    rho the mean density of its neighbours fluid in both masks (1 when none: the centre
    of the removed cube), u_w the rigid-body velocity at the node; the impulse is the
    covered momentum minus the refilled one; no other node changes."""
    cx, cy, cz, _, _ = lat
    nx, ny, nz = 12, 11, 10
    old = np.zeros((nz, ny, nx), np.uint8)
    old[3:5, 3:5, 3:5] = 1
    old[5:8, 5:8, 7:10] = 1
    new = np.zeros((nz, ny, nx), np.uint8)
    new[3:5, 3:5, 4:6] = 1
    U, W, X = np.array([0.01, 0.02, -0.01]), np.array([0.002, 0.001, -0.003]), np.array([4.5, 4.0, 3.5])
    S = d3.near_rest_state3(nx, ny, nz, seed=17, amp=0.1)
    s = D.OracleSim3(old, tau=0.8, bc_x=BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC,
                     body_motion=(U, W, X))
    s.set_state(S)
    imp = s.set_mask(new)
    T = s.state()
    C = np.stack([cx, cy, cz], 1).astype(float)
    P = np.zeros(3)
    for (z, y, x) in zip(*np.nonzero((old == 0) & (new == 1))):
        P += C.T @ S[:, z, y, x]
    changed = (old == 1) & (new == 0)
    for (z, y, x) in zip(*np.nonzero(changed)):
        rhos = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    a, b, c = (x + dx) % nx, (y + dy) % ny, (z + dz) % nz
                    if old[c, b, a] == 0 and new[c, b, a] == 0:
                        rhos.append(S[:, c, b, a].sum())
        rho = np.mean(rhos) if rhos else 1.0
        uw = U + np.cross(W, np.array([x, y, z], float) - X)
        np.testing.assert_allclose(T[:, z, y, x], D.equilibrium(rho, *uw), rtol=0, atol=1e-15)
        P -= C.T @ T[:, z, y, x]
    np.testing.assert_allclose(imp, P, rtol=0, atol=1e-14)
    assert np.array_equal(T[:, ~changed], S[:, ~changed])
    assert changed[6, 6, 8]  # the removed cube's centre: no neighbour fluid in both masks


def test_comoving_translating_sphere_keeps_a_uniform_flow_3d():
    nx, ny, nz = 32, 20, 18
    U = (0.04, 0.0, 0.0)
    feq = D.equilibrium(1.0, *U)
    S0 = np.broadcast_to(feq[:, None, None, None], (27, nz, ny, nx)).copy()
    s = D.OracleSim3(d3.sphere_mask(nx, ny, nz, 10, 9.5, 8.5, 4), tau=0.7, bc_x=BCX_PERIODIC,
                     bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC, box=(3, 29, 3, 17, 2, 16),
                     body_motion=(U, (0, 0, 0), (0, 0, 0)))
    s.set_state(S0)
    for k in range(1, 4):
        s.step(25)
        imp = s.set_mask(d3.sphere_mask(nx, ny, nz, 10 + k, 9.5, 8.5, 4))
        assert np.abs(imp).max() <= 1e-14
        fl = s._mask_keep == 0
        np.testing.assert_allclose(s.state()[:, fl], S0[:, fl], rtol=0, atol=1e-14)
    s.step(5)
    F = s.forces()
    assert np.abs(F[:, [0, 1, 3]]).max() <= 5e-14
    assert np.abs(F[:, 2]).max() <= 1e-12


def test_mask_change_bookkeeping_and_drtt_equals_b_3d(lat):
    """Fluid momentum after a change = before - impulse, and the mass balance; DRTT
    equals MEA-B at every step of a towed sphere whose box moves with it."""
    cx, cy, cz, _, _ = lat
    C = np.stack([cx, cy, cz], 1).astype(float)
    nx, ny, nz = 48, 20, 20
    m = lambda k: d3.sphere_mask(nx, ny, nz, 14 + k, 9.5, 9.5, 4)
    s = D.OracleSim3(m(0), tau=0.65, uin=np.full((nz, ny), 0.04), box=(7, 22, 3, 17, 3, 17),
                     body_motion=((0.05, 0, 0), (0, 0, 0), (0, 0, 0)))
    for k in range(1, 6):
        s.step(12)
        S = s.state()
        mo, mn = m(k - 1), m(k)
        box = (7 + k, 22 + k, 3, 17, 3, 17) if k % 2 == 0 else None
        imp = s.set_mask(mn, box)
        T = s.state()
        mom = lambda X, mk: np.einsum("ia,i...->a...", C, X)[:, mk == 0].sum(1)
        np.testing.assert_allclose(mom(T, mn), mom(S, mo) - imp, rtol=0, atol=1e-11)
        cov, fre = (mo == 0) & (mn == 1), (mo == 1) & (mn == 0)
        assert abs(T.sum(0)[mn == 0].sum() - (S.sum(0)[mo == 0].sum() - S.sum(0)[cov].sum()
                                              + T.sum(0)[fre].sum())) <= 1e-10
    s.step(12)
    F = s.forces()
    J = np.abs(s.records()[:, 6:9]).max()
    assert np.abs(F[:, 2] - F[:, 1]).max() <= 1e-12 * J


@pytest.mark.parametrize("omega", [0.7, 1.6])
def test_collide_stream_and_stream_collide_orders_commute_3d(lat, omega):
    """Sec. II (Eq. CollideAdv against Eq. AdvCollide) on the D3Q27 oracle: on a fully
    periodic lattice with a small body, the streaming S (the oracle's step with
    omega = 0) and the node-wise BGK collision C give f_{n+1} = S(C(f_n)) and
    g_{n+1} = C(S(g_n)) with g_0 = C(f_0) and g_n = C(f_n) bitwise; the oracle's BGK
    step from g_0 stores g_n and pulls f_n; the fluid's momentum is the same before and
    after collision."""
    cx, cy, cz, _, _ = lat
    nz, ny, nx, n = 4, 5, 6, 5
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[1:3, 2, 2:4] = 1
    P = D.BC_PERIODIC
    stream = D.OracleSim3(solid, omega=0.0, bc_x=BCX_PERIODIC, bc_y=P, bc_z=P)
    bgk = D.OracleSim3(solid, omega=omega, bc_x=BCX_PERIODIC, bc_y=P, bc_z=P)
    fl = solid == 0

    def C(F):
        out = F.copy()
        for z, y, x in zip(*np.nonzero(fl)):
            out[:, z, y, x] = D.collide_node(F[:, z, y, x], omega)
        return out

    def S(F):
        stream.set_state(F)
        stream.step()
        return stream.state()

    rng = np.random.default_rng(27)
    w = D.lattice()[4]
    f = w[:, None, None, None] * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, (27, nz, ny, nx)))
    g = C(f)
    bgk.set_state(g)
    for k in range(1, n + 1):
        f = S(C(f))
        g = C(S(g))
        assert np.array_equal(g[:, fl], C(f)[:, fl]), k
        bgk.step()
        assert np.array_equal(bgk.state()[:, fl], g[:, fl]), k
        assert np.array_equal(bgk.pre()[:, fl], f[:, fl]), k
        for c in (cx, cy, cz):
            jpre = np.tensordot(c, f, 1)[fl].sum()
            jpost = np.tensordot(c, g, 1)[fl].sum()
            assert abs(jpost - jpre) <= 1e-14 * f[:, fl].sum()
