"""Pins of the oracle against what the paper and the mathematics fix.

Kaushal, Succi & Ansumali, arXiv:2210.10377.  Each test names the passage it checks.
None of these compares the oracle with itself: they use exact rationals, closed forms,
conservation laws, brute-force tracking of single populations, Newton's law for the
whole fluid, and the worked one-dimensional example of the introduction.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import BCX_INLET_OUTLET, BCX_PERIODIC, BCY_PERIODIC, BCY_WALL, OracleSim


# --------------------------------------------------------------------------------------
# Lattice and equilibrium (Sec. II, Table I and the moment conditions)
# --------------------------------------------------------------------------------------

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table_d2q9():
    """tests/golden/d2q9_shells.txt: the paper's D2Q9 table (Sec. II, Table tabD2Q9)."""
    theta0, rows = None, []
    for line in open(os.path.join(GOLDEN, "d2q9_shells.txt")):
        t = line.split("#")[0].split()
        if not t:
            continue
        if t[0] == "theta0":
            theta0 = Fraction(t[1])
        else:
            rows.append((int(t[1]), int(t[2]), Fraction(t[3])))
    return theta0, rows


def test_lattice_matches_table_I(orc):
    """The oracle's velocities, weights and theta0 are exactly the printed table's; the
    opposite of each direction is its negative."""
    cx, cy, opp, w, th = orc.lattice()
    theta0, rows = _table_d2q9()
    assert len(rows) == 9
    got = sorted((int(cx[i]), int(cy[i]), w[i]) for i in range(9))
    want = sorted((a, b, float(wt)) for a, b, wt in rows)
    assert got == want
    assert th == float(theta0)
    for i in range(9):
        assert cx[opp[i]] == -cx[i] and cy[opp[i]] == -cy[i]


def test_weight_moment_conditions_exact(orc):
    """Sum w = 1, sum w c_a c_b = theta0 delta_ab, sum w c_a c_b c_c c_d = theta0^2 Delta
    (Sec. II), in exact rational arithmetic on the weights the oracle holds."""
    cx, cy, _, w, _ = orc.lattice()
    wf = [Fraction(x).limit_denominator(36) for x in w]
    for a, b in zip(wf, w):
        assert float(a) == b
    c = list(zip(cx.tolist(), cy.tolist()))
    th = Fraction(1, 3)
    assert sum(wf) == 1
    for a in range(2):
        assert sum(wf[i] * c[i][a] for i in range(9)) == 0
        for b in range(2):
            assert sum(wf[i] * c[i][a] * c[i][b] for i in range(9)) == (th if a == b else 0)
            for g in range(2):
                assert sum(wf[i] * c[i][a] * c[i][b] * c[i][g] for i in range(9)) == 0
                for d in range(2):
                    delta = ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
                    m4 = sum(wf[i] * c[i][a] * c[i][b] * c[i][g] * c[i][d] for i in range(9))
                    assert m4 == th * th * delta


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(orc, seed):
    """sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = rho u u + rho theta0 I (Sec. II)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 2)
    feq = orc.equilibrium(rho, u[0], u[1])
    cx, cy, _, _, th = orc.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    assert abs(feq.sum() - rho) <= 1e-15 * rho
    np.testing.assert_allclose(c.T @ feq, rho * u, rtol=0, atol=1e-16)
    P = np.einsum("i,ia,ib->ab", feq, c, c)
    np.testing.assert_allclose(P, rho * np.outer(u, u) + rho * th * np.eye(2), rtol=0, atol=2e-16)


@pytest.mark.parametrize("seed", range(5))
def test_collision_conserves_mass_and_momentum(orc, seed):
    """BGK (Eq. CollideAdv) relaxes towards an equilibrium with the node's own rho and
    rho u, so it conserves both."""
    rng = np.random.default_rng(seed)
    f = workloads.NEAR_REST_BASE * (1 + 0.05 * rng.uniform(-1, 1, 9))
    cx, cy, _, _, _ = orc.lattice()
    for omega in (0.3, 1.0, 1.7):
        g = orc.collide_node(f, omega)
        assert abs(g.sum() - f.sum()) <= 1e-15  # 4 ulp of 1
        assert abs(cx @ g - cx @ f) <= 1e-15
        assert abs(cy @ g - cy @ f) <= 1e-15


def test_collision_omega_one_gives_equilibrium(orc):
    """With 2 beta = 1 the post-collision state is the equilibrium of the node's own
    moments (special case of Eq. CollideAdv)."""
    rng = np.random.default_rng(7)
    f = workloads.NEAR_REST_BASE * (1 + 0.05 * rng.uniform(-1, 1, 9))
    cx, cy, _, _, _ = orc.lattice()
    rho = f.sum()
    feq = orc.equilibrium(rho, (cx @ f) / rho, (cy @ f) / rho)
    np.testing.assert_allclose(orc.collide_node(f, 1.0), feq, rtol=0, atol=1e-16)


# --------------------------------------------------------------------------------------
# Streaming and boundary rules, by tracking single populations (omega = 0)
# --------------------------------------------------------------------------------------

def _delta_state(nx, ny, i, x, y, val=1.0):
    """A lone extra population ``val`` in direction i at (x, y) on top of a uniform
    positive background (omega = 0 leaves every population as it is; the background
    keeps rho > 0 so the collision stays defined)."""
    S = np.broadcast_to(workloads.NEAR_REST_BASE[:, None, None], (9, ny, nx)).copy()
    S[i, y, x] += val
    return S


@pytest.mark.parametrize("i", range(9))
def test_pure_streaming_moves_by_c_i(orc, i):
    """Eq. CollideAdv, second line: f_i(x + c_i, t+1) = f~_i(x, t) -- with omega = 0 a
    lone population moves exactly c_i per step on a periodic lattice."""
    nx, ny = 7, 5
    cx, cy, _, _, _ = orc.lattice()
    s = OracleSim(np.zeros((ny, nx), np.uint8), omega=0.0, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    s.set_state(_delta_state(nx, ny, i, 3, 2, 0.25))
    for k in range(1, 12):
        s.step()
        S = s.state()
        want = _delta_state(nx, ny, i, (3 + k * cx[i]) % nx, (2 + k * cy[i]) % ny, 0.25)
        assert np.array_equal(S, want)


def test_wall_bounce_back_half_way(orc):
    """Stationary-wall bounce-back (Sec. II): a population moving down from row 1
    reaches row 0, meets the wall half-way to row -1 and returns reversed to row 0 one
    step later, then moves up."""
    nx, ny = 5, 6
    s = OracleSim(np.zeros((ny, nx), np.uint8), omega=0.0, bc_x=BCX_PERIODIC, bc_y=BCY_WALL)
    s.set_state(_delta_state(nx, ny, 4, 2, 1, 0.5))   # direction 4 = (0,-1)
    s.step()
    assert np.array_equal(s.state(), _delta_state(nx, ny, 4, 2, 0, 0.5))
    s.step()
    assert np.array_equal(s.state(), _delta_state(nx, ny, 2, 2, 0, 0.5))  # reversed
    s.step()
    assert np.array_equal(s.state(), _delta_state(nx, ny, 2, 2, 1, 0.5))
    # Diagonal (1,-1) at row 0 comes back as (-1,1) at the same node.
    s.set_state(_delta_state(nx, ny, 8, 2, 0, 0.5))
    s.step()
    assert np.array_equal(s.state(), _delta_state(nx, ny, 6, 2, 0, 0.5))


def test_body_bounce_back_half_way(orc):
    """Sec. II: the boundary point sits half-way along the fluid-solid link; the
    population heading into the solid node comes back reversed at the same fluid node."""
    nx, ny = 7, 7
    mask = np.zeros((ny, nx), np.uint8)
    mask[3, 4] = 1
    s = OracleSim(mask, omega=0.0, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    s.set_state(_delta_state(nx, ny, 1, 2, 3, 0.5))   # (1,0) at (2,3) -> (3,3) -> back
    s.step()
    assert np.array_equal(s.state()[:, :, :4], _delta_state(nx, ny, 1, 3, 3, 0.5)[:, :, :4])
    s.step()
    assert np.array_equal(s.state()[:, :, :4], _delta_state(nx, ny, 3, 3, 3, 0.5)[:, :, :4])


def test_inlet_returns_with_moving_wall_term(orc):
    """Moving-wall bounce-back (Sec. II) at the inlet x = -1/2 with u_w = (u_in, 0):
    a population leaving through the inlet comes back reversed plus 2 w rho c.u_w / c_s^2."""
    nx, ny, u = 6, 5, 0.03
    s = OracleSim(np.zeros((ny, nx), np.uint8), omega=0.0, uin=np.full(ny, u),
                  bc_x=BCX_INLET_OUTLET, bc_y=BCY_PERIODIC)
    b = workloads.NEAR_REST_BASE
    s.set_state(np.broadcast_to(b[:, None, None], (9, ny, nx)).copy())
    s.step()
    S = s.state()
    # Only the inlet column changes: (1,0) gains 6 w1 u, (1,+-1) gain 6 w5 u, where
    # 2 w / c_s^2 = 6 w with w1 = 4/36 and w5 = 1/36.
    want = np.broadcast_to(b[:, None, None], (9, ny, nx)).copy()
    want[1, :, 0] += 6 * (4 / 36) * u
    want[5, :, 0] += 6 * (1 / 36) * u
    want[8, :, 0] += 6 * (1 / 36) * u
    np.testing.assert_allclose(S, want, rtol=1e-15, atol=0)


def test_outlet_zero_gradient_ghost_copy(orc):
    """Outlet reading (zero gradient): the ghost column nx holds the post-collision
    populations of column nx-1, so a population moving left from the last column is
    both streamed on and copied back into the last column."""
    nx, ny = 6, 5
    s = OracleSim(np.zeros((ny, nx), np.uint8), omega=0.0, uin=np.zeros(ny),
                  bc_x=BCX_INLET_OUTLET, bc_y=BCY_PERIODIC)
    s.set_state(_delta_state(nx, ny, 3, nx - 1, 2, 0.5))   # (-1,0) at the last column
    s.step()
    want = _delta_state(nx, ny, 3, nx - 2, 2, 0.5)
    want[3, 2, nx - 1] = want[3, 2, nx - 2]
    assert np.array_equal(s.state(), want)
    # A population moving right out of the last column is lost.
    s.set_state(_delta_state(nx, ny, 1, nx - 1, 2, 0.5))
    s.step()
    assert np.array_equal(s.state(), _delta_state(nx, ny, 1, 0, 0, 0.0))


# --------------------------------------------------------------------------------------
# Conservation, fixed points and the inlet mass flux
# --------------------------------------------------------------------------------------

def test_periodic_conservation(orc):
    """Fully periodic lattice, no body: total mass and momentum are invariants of the
    collide-stream step (Sec. II)."""
    nx, ny = 24, 16
    cx, cy, _, _, _ = orc.lattice()
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=0.7, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    S0 = workloads.near_rest_state(nx, ny, seed=3, amp=0.05)
    s.set_state(S0)
    m0 = S0.sum()
    j0 = np.array([np.tensordot(cx, S0, 1).sum(), np.tensordot(cy, S0, 1).sum()])
    s.step(1000)
    S = s.state()
    assert abs(S.sum() - m0) <= 1e-13 * m0
    j = np.array([np.tensordot(cx, S, 1).sum(), np.tensordot(cy, S, 1).sum()])
    np.testing.assert_allclose(j, j0, rtol=0, atol=1e-13 * m0)


def _collide_field(orc, F, omega, solid):
    """The BGK collision (Eq. CollideAdv, first line) applied node by node to a
    population field [9, ny, nx]; solid nodes are left as they are."""
    out = F.copy()
    for y in range(F.shape[1]):
        for x in range(F.shape[2]):
            if not solid[y, x]:
                out[:, y, x] = orc.collide_node(F[:, y, x], omega)
    return out


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.7])
@pytest.mark.parametrize("body", [False, True])
def test_collide_stream_and_stream_collide_orders_commute(orc, omega, body):
    """Sec. II: the collide-then-stream order (Eq. CollideAdv) and the stream-then-collide
    order (Eq. AdvCollide) give the same dynamics.  The streaming operator S is the
    oracle's step with omega = 0 (a pure pull: every value moves unchanged), the
    collision C the node-wise BGK map.  From a random f_0 on a fully periodic lattice,
    f_{n+1} = S(C(f_n)) and g_{n+1} = C(S(g_n)) with g_0 = C(f_0) satisfy g_n = C(f_n)
    bitwise for every n, the oracle's own BGK step from g_0 stores exactly g_n and pulls
    exactly f_n, and the total momentum before and after collision is the same, so a
    force sampled on either side of the collision agrees.  With a body the trajectory
    identity still holds (bounce-back is part of S); what the body breaks is the equality
    of the momentum exchanged at the wall when sampled before or after the collision
    (algorithms A and B, pinned by the A-minus-B identity)."""
    nx, ny, n = 12, 10, 8
    cx, cy, _, _, _ = orc.lattice()
    solid = np.zeros((ny, nx), np.uint8)
    if body:
        solid[4:6, 5:8] = 1
    stream = OracleSim(solid, omega=0.0, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    bgk = OracleSim(solid, omega=omega, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)

    def S(F):
        stream.set_state(F)
        stream.step()
        return stream.state()

    f = workloads.near_rest_state(nx, ny, seed=11, amp=0.2)
    g = _collide_field(orc, f, omega, solid)
    bgk.set_state(g)
    fl = solid == 0
    for k in range(1, n + 1):
        f = S(_collide_field(orc, f, omega, solid))
        g = _collide_field(orc, S(g), omega, solid)
        Cf = _collide_field(orc, f, omega, solid)
        assert np.array_equal(g[:, fl], Cf[:, fl]), k
        bgk.step()
        assert np.array_equal(bgk.state()[:, fl], g[:, fl]), k
        assert np.array_equal(bgk.pre()[:, fl], f[:, fl]), k
        jpre = np.array([np.tensordot(cx, f, 1)[fl].sum(), np.tensordot(cy, f, 1)[fl].sum()])
        jpost = np.array([np.tensordot(cx, g, 1)[fl].sum(), np.tensordot(cy, g, 1)[fl].sum()])
        np.testing.assert_allclose(jpost, jpre, rtol=0, atol=1e-14 * f[:, fl].sum())


def test_closed_box_conserves_mass(orc):
    """Walls top and bottom, a body, and a solid column closing the channel: bounce-back
    returns every population, so mass is conserved."""
    nx, ny = 30, 14
    mask = workloads.cylinder_mask(nx, ny, 12, 7, 3)
    mask[:, 0] = 1
    mask[:, -1] = 1
    s = OracleSim(mask, tau=0.6, uin=np.zeros(ny), bc_x=BCX_INLET_OUTLET, bc_y=BCY_WALL)
    S0 = workloads.near_rest_state(nx, ny, seed=4, amp=0.05)
    s.set_state(S0)
    fl = mask == 0
    m0 = S0[:, fl].sum()
    s.step(1000)
    assert abs(s.state()[:, fl].sum() - m0) <= 1e-13 * m0


def test_inlet_mass_injection_closed_form(orc):
    """Each inlet row gains 2 rho_w u_in sum_{c_x=+1} w_i / c_s^2 = u_in of mass per step;
    the two corner rows lose the diagonal that meets the wall first (5/6 u_in)."""
    nx, ny = 20, 9
    rng = np.random.default_rng(11)
    uin = rng.uniform(0.01, 0.08, ny)
    mask = np.zeros((ny, nx), np.uint8)
    mask[:, -1] = 1  # close the outlet
    s = OracleSim(mask, tau=0.8, uin=uin, bc_x=BCX_INLET_OUTLET, bc_y=BCY_WALL)
    S0 = workloads.near_rest_state(nx, ny, seed=5, amp=0.02)
    s.set_state(S0)
    fl = mask == 0
    gain = uin.sum() - (uin[0] + uin[-1]) / 6.0
    m = S0[:, fl].sum()
    for _ in range(50):
        s.step()
        m_new = s.state()[:, fl].sum()
        assert abs((m_new - m) - gain) <= 1e-13
        m = m_new


def test_rest_state_is_fixed_point_and_forceless(orc):
    """With no inflow the rest state w_i is kept (to rounding: sum w_i is 1 only to an
    ulp in binary64), and every force vanishes."""
    w = workloads.cylinder_channel_200x80()
    s = OracleSim(w.mask, tau=w.tau, uin=np.zeros(w.ny), box=w.box)
    S0 = s.state()
    s.step(20)
    np.testing.assert_allclose(s.state(), S0, rtol=0, atol=1e-15)
    F = s.forces()
    assert np.abs(F).max() <= 1e-14


def test_uniform_flow_is_fixed_point_with_inlet_and_outlet(orc):
    """Uniform f^eq(1, (u, 0)) in a channel periodic in y: the moving-wall inlet returns
    exactly the equilibrium populations and the outlet copy keeps them."""
    nx, ny, u = 16, 6, 0.05
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=0.7, uin=np.full(ny, u),
                  bc_x=BCX_INLET_OUTLET, bc_y=BCY_PERIODIC)
    feq = orc.equilibrium(1.0, u, 0.0)
    S0 = np.broadcast_to(feq[:, None, None], (9, ny, nx)).copy()
    s.set_state(S0)
    s.step(50)
    np.testing.assert_allclose(s.state(), S0, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------------------
# Links (Sec. III: fluid-solid links, boundary point half-way)
# --------------------------------------------------------------------------------------

def test_links_single_solid_node(orc):
    m = np.zeros((5, 5), np.uint8)
    m[2, 2] = 1
    L = orc.links(m)
    # fluid node 12 - c_i links in direction i
    want = sorted(((2 - cy) * 5 + (2 - cx), i) for i, (cx, cy) in enumerate(
        [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]) if i)
    assert [tuple(r) for r in L] == want
    assert len(L) == 8


def test_links_domino(orc):
    m = np.zeros((5, 6), np.uint8)
    m[2, 2] = m[2, 3] = 1
    assert len(orc.links(m)) == 14


def _brute_links(mask, px, py):
    ny, nx = mask.shape
    C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    out = []
    for y in range(ny):
        for x in range(nx):
            if mask[y, x]:
                continue
            for i in range(1, 9):
                tx, ty = x + C[i][0], y + C[i][1]
                if px:
                    tx %= nx
                if py:
                    ty %= ny
                if 0 <= tx < nx and 0 <= ty < ny and mask[ty, tx]:
                    out.append((y * nx + x, i))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_links_random_masks_brute_force(orc, seed):
    rng = np.random.default_rng(100 + seed)
    m = (rng.uniform(size=(10, 12)) < 0.25).astype(np.uint8)
    for bcx, bcy in ((0, 0), (1, 0), (0, 1), (1, 1)):
        L = orc.links(m, bc_x=bcx, bc_y=bcy)
        assert [tuple(r) for r in L] == _brute_links(m, bcx == 1, bcy == 1)


# --------------------------------------------------------------------------------------
# Forces
# --------------------------------------------------------------------------------------

def test_newton_global_momentum_balance(orc):
    """Newton's law for the whole fluid: with body force g on N fluid nodes and every
    solid node counted as body, J(t) - J(t+1) + N g = F_B(t) at every step, where J is
    the momentum of all fluid nodes before collision (Eq. rtt2 with the whole fluid as
    control volume).  Pins MEA-B (sign, factor 2, link set) independently of its
    formula."""
    nx, ny = 32, 20
    mask = workloads.cylinder_mask(nx, ny, 15.5, 9.5, 4.0)
    mask[0, :] = 1
    mask[-1, :] = 1
    g = (2e-6, -1e-6)
    s = OracleSim(mask, tau=0.8, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC, g=g)
    cx, cy, _, _, _ = orc.lattice()
    fl = mask == 0
    N = fl.sum()
    Jprev = None
    for t in range(300):
        s.step()
        f = s.pre()
        J = np.array([np.tensordot(cx, f, 1)[fl].sum(), np.tensordot(cy, f, 1)[fl].sum()])
        if Jprev is not None:
            FB = s.forces()[t - 1, 1]
            np.testing.assert_allclose(Jprev - J + N * np.array(g), FB, rtol=0, atol=1e-13)
        Jprev = J


def test_poiseuille_magic_tau_exact(orc):
    """Body-force-driven channel between half-way bounce-back walls at y = -1/2 and
    ny - 1/2: u(y) = g/(2 nu) (y + 1/2)(ny - 1/2 - y), nu = (tau - 1/2)/3.  At
    (tau - 1/2)^2 = 3/16 the BGK bounce-back solution is the parabola itself; at steady
    state the wall force (the populations bounced at the walls) equals N g."""
    nx, ny = 2, 16
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    g = 1e-6
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=tau, bc_x=BCX_PERIODIC, bc_y=BCY_WALL,
                  g=(g, 0.0))
    s.step(8000)
    s.step(1)
    f = s.pre()
    cx, _, _, _, _ = orc.lattice()
    rho = f.sum(0)
    u = ((np.tensordot(cx, f, 1) + 0.5 * g) / rho)[:, 0]
    y = np.arange(ny)
    exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    np.testing.assert_allclose(u, exact, rtol=1e-10, atol=0)


def test_poiseuille_second_order_convergence(orc):
    """Away from the special tau the half-way bounce-back wall is second-order accurate:
    the max relative profile error falls by about 4x per doubling of ny."""
    tau, errs = 0.8, []
    for ny in (8, 16, 32):
        nu = (tau - 0.5) / 3.0
        g = 1e-6 * (8.0 / ny) ** 2
        s = OracleSim(np.zeros((ny, 2), np.uint8), tau=tau, bc_x=BCX_PERIODIC, bc_y=BCY_WALL,
                      g=(g, 0.0))
        s.step(int(40 * ny * ny / nu / 10))
        s.step(1)
        f = s.pre()
        cx, _, _, _, _ = orc.lattice()
        u = ((np.tensordot(cx, f, 1) + 0.5 * g) / f.sum(0))[:, 0]
        y = np.arange(ny)
        exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
        errs.append(np.abs(u - exact).max() / exact.max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def test_channel_wall_force_equals_body_force(orc):
    """Steady body-force-driven channel whose walls are solid rows: the total momentum
    exchange on the walls equals the applied body force on all fluid nodes."""
    nx, ny = 4, 18
    mask = np.zeros((ny, nx), np.uint8)
    mask[0, :] = 1
    mask[-1, :] = 1
    g = 1e-6
    s = OracleSim(mask, tau=0.9, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC, g=(g, 0.0))
    s.step(6000)
    FB = s.forces()[-1, 1]
    N = (mask == 0).sum()
    np.testing.assert_allclose(FB, [N * g, 0.0], rtol=1e-9, atol=1e-9 * N * g)


def test_drtt_equals_mea_b_and_is_box_invariant(orc):
    """With half-way bounce-back, collision conserving momentum node by node and an
    admissible box, J(t) - J(t+1) = (out - in through the box surface) + 2 sum_L c_i f~_i,
    so the DRTT force of the second Eq. rtt7 equals MEA-B (Eq. rtt5) step by step, for
    any such box."""
    w = workloads.cylinder_channel_200x80()
    F = []
    for box in ((10, 70, 10, 70), (25, 56, 24, 57), (5, 120, 3, 77)):
        s = OracleSim(w.mask, tau=w.tau, uin=w.uin, box=box)
        s.step(400)
        F.append(s.forces())
    for Fi in F:
        scale = np.abs(Fi[:, 1]).max()
        assert np.abs(Fi[:, 2] - Fi[:, 1]).max() <= 1e-11 * scale
    assert np.abs(F[0][:, 2] - F[1][:, 2]).max() <= 1e-11 * np.abs(F[0][:, 1]).max()


def test_drtt_empty_box_is_zero(orc):
    """No body inside the control volume: inflow minus outflow balances the change of
    box momentum exactly, so the DRTT force vanishes (second Eq. rtt7)."""
    nx, ny = 60, 30
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=0.7, uin=np.full(ny, 0.05),
                  box=(10, 40, 5, 25))
    s.set_state(workloads.near_rest_state(nx, ny, seed=9, amp=0.05))
    s.step(100)
    F = s.forces()
    R = s.records()
    # |F| at the rounding level of the box momentum (~30) versus fluxes of order 0.1
    assert np.abs(R[:, 6:8]).max() > 1e-2
    assert np.abs(F[:, 2]).max() <= 1e-12


def test_drtt_post_equals_mea_b_and_drtt(orc):
    """DRTT with the control-volume momentum taken after the collision (J^post(t), the
    stored populations of V) in place of J(t) (second Eq. rtt7; the Appendix samples J
    before the collision): every term then reads the stored populations, so
    J^post(t) - J(t+1) + Phi(t) is the momentum balance of the box over streaming and
    bounce-back alone and equals MEA-B; BGK conserves momentum node by node, so it also
    equals DRTT.  Three boxes; an empty box gives zero."""
    w = workloads.cylinder_channel_200x80()
    for box in ((10, 70, 10, 70), (25, 56, 24, 57), (5, 120, 3, 77)):
        s = OracleSim(w.mask, tau=w.tau, uin=w.uin, box=box)
        s.step(300)
        F = s.forces()
        assert F.shape == (300, 5, 2)
        # The three sums run over the n_V nodes of the box with |c_i f_i| adding to at
        # most 0.7 per node: rounding of at most 64 units each, 1.5e-14 per node.
        nv = int((w.mask[box[2]:box[3], box[0]:box[1]] == 0).sum())
        tol = 1.5e-14 * nv
        assert np.abs(F[:, 4] - F[:, 1]).max() <= tol
        assert np.abs(F[:, 4] - F[:, 2]).max() <= tol
        assert np.abs(F[:, 1]).max() > 1e3 * tol
    nx, ny = 60, 30
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=0.7, uin=np.full(ny, 0.05),
                  box=(10, 40, 5, 25))
    s.set_state(workloads.near_rest_state(nx, ny, seed=9, amp=0.05))
    s.step(50)
    assert np.abs(s.forces()[:, 4]).max() <= 1e-12


def test_drtt_post_separates_momentum_added_by_the_collision(orc):
    """A collision that adds momentum (the Guo body force g on each node, a test-only
    extension) separates the two samplings of the box momentum: J^post(t) = J(t) + N_V g
    for the N_V fluid nodes of the box, so DRTT = MEA-B - N_V g at every step (the closed
    form), while DRTT-post = MEA-B (the box balance over streaming only).  A reading that
    sampled both J at the same side of the collision would fail one of the two."""
    nx, ny = 40, 24
    mask = workloads.cylinder_mask(nx, ny, 19.5, 11.5, 4.0)
    g = (3e-6, -2e-6)
    box = (8, 32, 4, 20)
    s = OracleSim(mask, tau=0.8, bc_x=BCX_PERIODIC, bc_y=BCY_WALL, box=box, g=g)
    s.set_state(workloads.near_rest_state(nx, ny, seed=5, amp=0.02))
    s.step(200)
    F = s.forces()
    R = s.records()
    nv = int((mask[box[2]:box[3], box[0]:box[1]] == 0).sum())
    np.testing.assert_allclose(R[:, 10:12] - R[:, 4:6], np.broadcast_to(nv * np.array(g), (200, 2)),
                               rtol=0, atol=1e-12 * nv)
    np.testing.assert_allclose(F[:, 2], F[:, 1] - nv * np.array(g), rtol=0, atol=1.5e-14 * nv)
    np.testing.assert_allclose(F[:, 4], F[:, 1], rtol=0, atol=1.5e-14 * nv)
    # the separated term N_V g is far above the rounding bound
    assert nv * min(abs(g[0]), abs(g[1])) > 1e6 * 1.5e-14 * nv


def test_a_minus_b_is_the_collision_of_the_outgoing_populations(orc):
    """Eq. rtt4: algorithm A takes the outgoing population before collision, B after, with
    the same returned populations, so F_A - F_B = 2 beta sum_L c_i (f_i - f_i^eq) -- the
    two-dimensional form of the term that Eq. lbb3 has and algorithm A misses."""
    w = workloads.cylinder_channel_200x80()
    s = OracleSim(w.mask, tau=w.tau, uin=w.uin, box=w.box)
    links = orc.links(w.mask)
    cx, cy, _, _, _ = orc.lattice()
    for t in range(60):
        s.step()
        f = s.pre()
        d = np.zeros(2)
        for node, i in links:
            y, x = divmod(int(node), w.nx)
            fn = f[:, y, x]
            rho = fn.sum()
            feq = orc.equilibrium(rho, (cx @ fn) / rho, (cy @ fn) / rho)
            d += (fn[i] - feq[i]) * np.array([cx[i], cy[i]])
        F = s.forces()[t]
        np.testing.assert_allclose(F[0] - F[1], s.omega * d, rtol=1e-12, atol=1e-14)


def test_first_step_pure_streaming_single_solid(orc):
    """Uniform flow f^eq(1, u) around one solid node with omega = 0: every direction has
    exactly one link and the outgoing populations are the equilibrium ones, so
    F_A(0) = F_B(0) = F_DRTT(0) = 2 sum_i c_i f_i^eq = 2 rho u."""
    nx, ny = 9, 9
    m = np.zeros((ny, nx), np.uint8)
    m[4, 4] = 1
    u = np.array([0.04, -0.02])
    s = OracleSim(m, omega=0.0, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC, box=(2, 7, 2, 7))
    feq = orc.equilibrium(1.0, u[0], u[1])
    s.set_state(np.broadcast_to(feq[:, None, None], (9, ny, nx)).copy())
    s.step(1)
    F = s.forces()[0]
    for k in range(3):
        np.testing.assert_allclose(F[k], 2 * u, rtol=1e-14, atol=1e-17)


def test_symmetric_cylinder_has_no_lift(orc):
    """Cylinder on the channel centre line (walls at -1/2 and ny-1/2, centre row
    (ny-1)/2): mirror symmetry gives F_y = 0 for every scheme."""
    nx, ny = 90, 41
    mask = workloads.cylinder_mask(nx, ny, 20, 20, 5)
    s = OracleSim(mask, tau=0.65, uin=np.full(ny, 0.05), box=(8, 34, 8, 33))
    s.step(600)
    F = s.forces()
    for k in range(3):
        assert np.abs(F[:, k, 1]).max() <= 1e-12 * np.abs(F[:, k, 0]).max()
    assert F[-1, 1, 0] > 0  # drag points downstream


def test_positive_incidence_gives_positive_lift(orc):
    """NACA0012 at +8 deg (nose up) in a uniform stream: the lift of every scheme points
    to +y once the flow is established."""
    w = workloads.naca_channel(192, 96, 48, 8.0, 100.0, 0)
    s = OracleSim(w.mask, tau=w.tau, uin=w.uin, box=w.box)
    s.step(1500)
    F = s.forces()[-200:].mean(0)
    assert np.all(F[:, 1] > 0) and np.all(F[:, 0] > 0)


# --------------------------------------------------------------------------------------
# The one-dimensional toy of the introduction (Eq. lbb1-lbb4)
# --------------------------------------------------------------------------------------

def _toy_state(n, seed):
    from oracle import d1q3
    rng = np.random.default_rng(seed)
    return [[d1q3.W[i] * (1 + 0.1 * rng.uniform(-1, 1)) for i in range(3)] for _ in range(n)]


@pytest.mark.parametrize("seed", range(4))
def test_d1q3_momentum_balance(seed):
    from oracle import d1q3
    beta = 0.37
    nodes = _toy_state(8, seed)
    f1, fm1 = nodes[0][1], nodes[0][2]
    J0 = d1q3.momentum(nodes, len(nodes))
    for collided in (False, True):
        new, post = d1q3.step(nodes, beta, collided)
        # momentum through the far right surface is bookkept separately (the toy's
        # control volume is semi-infinite)
        right = -post[-1][1] - new[-1][2]
        dJ = d1q3.momentum(new, len(new)) - J0 - right
        F1 = new[0][1]
        # Eq. lbb2
        assert abs(dJ - (F1 + fm1 - f1 + post[0][1])) <= 1e-15
        rho = sum(nodes[0])
        feq = d1q3.equilibrium(rho, (f1 - fm1) / rho)
        if not collided:   # Eq. lbb3: un-collided return
            assert abs(dJ - (2 * fm1 + 2 * beta * (feq[1] - f1))) <= 1e-15
        else:              # Eq. lbb4: collided return
            assert abs(dJ - 2 * post[0][2]) <= 1e-15


# --------------------------------------------------------------------------------------
# Input geometry (the synthetic stand-ins for the paper's bodies)
# --------------------------------------------------------------------------------------

def test_cylinder_mask_gauss_circle():
    """Integer points with a^2 + b^2 <= 100: N(10) = 317 (Gauss circle problem); 12 of
    them on the circle (a^2 + b^2 = 100)."""
    m = workloads.cylinder_mask(200, 80, 40, 40, 10)
    assert int(m.sum()) == 317
    iy, ix = np.nonzero(m)
    assert int(((ix - 40) ** 2 + (iy - 40) ** 2 == 100).sum()) == 12


def test_naca_mask_area_symmetry_and_incidence():
    c = 256
    m0 = workloads.naca0012_mask(1024, 512, c, 320, 256, 0.0)
    # area of the open-trailing-edge NACA0012: 10 t c^2 (0.2969*2/3 - 0.126/2 - 0.3516/3
    # + 0.2843/4 - 0.1015/5)
    area = 10 * 0.12 * c * c * (0.2969 * 2 / 3 - 0.126 / 2 - 0.3516 / 3 + 0.2843 / 4 - 0.1015 / 5)
    assert abs(m0.sum() - area) <= 0.02 * area
    assert np.array_equal(m0[256 + 1:256 + 100], m0[256 - 1:256 - 100:-1])
    ys, xs = np.nonzero(m0)
    assert xs.min() == 256 and xs.max() in (511, 512)
    m8 = workloads.naca0012_mask(1024, 512, c, 320, 256, 8.0)
    ys, xs = np.nonzero(m8)
    assert ys[xs == xs.min()].mean() > 256 > ys[xs == xs.max()].mean()  # nose up


# --------------------------------------------------------------------------------------
# Complex-step derivatives of the time-averaged force (the adjoint's reference)
# --------------------------------------------------------------------------------------

def test_complex_step_matches_central_differences(orc):
    """The oracle in complex arithmetic (Im J(theta + i h v) / h) gives the same
    directional derivatives of the mean algorithm-B drag as FP64 central differences of
    the real oracle, for tau and for the inlet profile."""
    nx, ny = 64, 32
    mask = workloads.cylinder_mask(nx, ny, 18, 15.5, 3)
    y = np.arange(ny)
    uin = 0.03 + 0.02 * np.sin(np.pi * (y + 0.5) / ny)
    tau, n, t0, T = 0.8, 160, 100, 60
    h = 1e-30
    # tau
    cs = orc.objective(mask, 1 / complex(tau, h), uin, n, t0, T).imag / h
    e = 1e-6
    fd = (orc.objective(mask, 1 / (tau + e), uin, n, t0, T).real
          - orc.objective(mask, 1 / (tau - e), uin, n, t0, T).real) / (2 * e)
    assert abs(cs - fd) <= 1e-6 * abs(cs)
    # inlet direction
    v = np.random.default_rng(5).normal(size=ny)
    cs = orc.objective(mask, 1 / tau, uin + 1j * h * v, n, t0, T).imag / h
    e = 1e-7
    fd = (orc.objective(mask, 1 / tau, uin + e * v, n, t0, T).real
          - orc.objective(mask, 1 / tau, uin - e * v, n, t0, T).real) / (2 * e)
    assert abs(cs - fd) <= 1e-6 * abs(cs)
    # the real part is the real objective
    Jr = orc.objective(mask, 1 / tau, uin, n, t0, T)
    o = OracleSim(mask, tau=tau, uin=uin)
    o.step(n)
    assert abs(Jr.real - o.forces()[t0:t0 + T, 1, 0].mean()) <= 1e-15


# --------------------------------------------------------------------------------------
# Regularized collision (Latt & Chopard 2006; the stated variant for tau_lb -> 1/2, not
# in the paper)
# --------------------------------------------------------------------------------------

def _random_f(seed, amp=0.2):
    rng = np.random.default_rng(seed)
    return workloads.NEAR_REST_BASE * (1.0 + amp * rng.uniform(-1.0, 1.0, 9))


@pytest.mark.parametrize("seed", range(4))
def test_regularized_conserves_mass_and_momentum(orc, seed):
    cx, cy, _, _, _ = orc.lattice()
    f = _random_f(seed)
    for omega in (0.3, 1.0, 1.7, 1.999):
        g = orc.collide_node(f, omega, collision="regularized")
        assert abs(g.sum() - f.sum()) <= 4e-16
        assert abs(cx @ g - cx @ f) <= 4e-16 and abs(cy @ g - cy @ f) <= 4e-16


@pytest.mark.parametrize("seed", range(4))
def test_regularized_equals_bgk_on_second_order_hermite_subspace(orc, seed):
    """For f = f^eq(rho, u) + w_i (c_i c_i - theta0 I) : A (A symmetric), the
    non-equilibrium part already lies in the second-order Hermite subspace, so the
    projection is the identity and the regularized collision is BGK (Eq. CollideAdv)."""
    cx, cy, _, w, th = orc.lattice()
    rng = np.random.default_rng(100 + seed)
    rho, ux, uy = 1.0 + 0.1 * rng.uniform(), 0.05 * rng.uniform(-1, 1), 0.05 * rng.uniform(-1, 1)
    a, b, c = 1e-3 * rng.uniform(-1, 1, 3)
    q = (cx * cx - th) * a + 2 * cx * cy * b + (cy * cy - th) * c
    f = orc.equilibrium(rho, ux, uy) + w * q
    for omega in (0.5, 1.3, 1.95):
        np.testing.assert_allclose(orc.collide_node(f, omega, collision="regularized"),
                                   orc.collide_node(f, omega), rtol=0, atol=3e-16)


@pytest.mark.parametrize("seed", range(4))
def test_regularized_discards_modes_above_second_order(orc, seed):
    """Populations differing by a vector with no mass, momentum or second moment (the
    null space of the six moments 1, c_x, c_y, c_x^2, c_x c_y, c_y^2) collide to the same
    result under the regularized collision, while BGK keeps the difference."""
    from scipy.linalg import null_space
    cx, cy, _, _, _ = orc.lattice()
    M = np.array([np.ones(9), cx, cy, cx * cx, cx * cy, cy * cy], dtype=np.float64)
    K = null_space(M)
    assert K.shape == (9, 3)
    f = _random_f(seed)
    g = f + 2e-3 * K @ np.random.default_rng(seed).uniform(-1, 1, 3)
    omega = 1.6
    r_f = orc.collide_node(f, omega, collision="regularized")
    r_g = orc.collide_node(g, omega, collision="regularized")
    np.testing.assert_allclose(r_f, r_g, rtol=0, atol=1e-16)
    assert np.abs(orc.collide_node(f, omega) - orc.collide_node(g, omega)).max() > 1e-5


def test_regularized_rest_and_uniform_flow_are_fixed_points(orc):
    feq = orc.equilibrium(1.02, 0.04, -0.01)
    np.testing.assert_allclose(orc.collide_node(feq, 1.8, collision="regularized"), feq,
                               rtol=0, atol=1e-17)
    nx, ny = 24, 12
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=0.5005, bc_x=BCX_PERIODIC,
                  bc_y=BCY_PERIODIC, collision="regularized")
    S0 = np.repeat(np.repeat(feq[:, None, None], ny, 1), nx, 2)
    s.set_state(S0)
    s.step(20)
    np.testing.assert_allclose(s.state(), S0, rtol=0, atol=1e-16)


def test_regularized_drtt_equals_mea_b(orc):
    """The regularized collision conserves momentum node by node, so the identity
    DRTT = MEA-B (second Eq. rtt7 against Eq. rtt5) holds for it as for BGK."""
    w = workloads.cylinder_channel_200x80()
    s = OracleSim(w.mask, tau=0.51, uin=w.uin, box=w.box, collision="regularized")
    s.step(400)
    F = s.forces()
    scale = np.abs(F[:, 1]).max()
    assert scale > 0
    assert np.abs(F[:, 2] - F[:, 1]).max() <= 1e-11 * scale


# --------------------------------------------------------------------------------------
# Entropic KBC collision (Karlin, Boesch & Chikatamarla 2014; a stated variant for tau_lb
# -> 1/2, not in the paper).  Pinned by properties of its output only.
# --------------------------------------------------------------------------------------

def _moments9(cx, cy):
    """Rows: 1, c_x, c_y, c_x^2 + c_y^2, c_x^2 - c_y^2, c_x c_y, c_x^2 c_y, c_x c_y^2,
    c_x^2 c_y^2 (an invertible basis of D2Q9)."""
    cx = cx.astype(np.float64)
    cy = cy.astype(np.float64)
    return np.array([np.ones(9), cx, cy, cx * cx + cy * cy, cx * cx - cy * cy, cx * cy,
                     cx * cx * cy, cx * cy * cy, cx * cx * cy * cy])


def _eq_of(orc, f):
    cx, cy, _, _, _ = orc.lattice()
    rho = f.sum()
    return orc.equilibrium(rho, (cx @ f) / rho, (cy @ f) / rho)


@pytest.mark.parametrize("seed", range(4))
def test_kbc_conserves_mass_and_momentum(orc, seed):
    cx, cy, _, _, _ = orc.lattice()
    f = _random_f(seed)
    for omega in (0.8, 1.5, 1.99, 1.999):
        g = orc.collide_node(f, omega, collision="kbc")
        assert abs(g.sum() - f.sum()) <= 4e-16
        assert abs(cx @ g - cx @ f) <= 4e-16 and abs(cy @ g - cy @ f) <= 4e-16


@pytest.mark.parametrize("seed", range(4))
def test_kbc_relaxes_shear_stress_as_bgk(orc, seed):
    """The deviatoric stresses (c_x^2 - c_y^2 and c_x c_y moments) relax with the BGK
    rate, (M f~ - M f^eq) = (1 - omega)(M f - M f^eq): same viscosity as Eq.
    CollideAdv."""
    cx, cy, _, _, _ = orc.lattice()
    M = _moments9(cx, cy)
    f = _random_f(seed)
    feq = _eq_of(orc, f)
    for omega in (1.2, 1.9, 1.995):
        g = orc.collide_node(f, omega, collision="kbc")
        for row in (4, 5):
            np.testing.assert_allclose(M[row] @ g - M[row] @ feq,
                                       (1 - omega) * (M[row] @ f - M[row] @ feq),
                                       rtol=1e-12, atol=1e-17)


@pytest.mark.parametrize("seed", range(3))
def test_kbc_equals_bgk_for_pure_shear_nonequilibrium(orc, seed):
    """If f - f^eq carries only the deviatoric stresses (every other moment of the
    invertible D2Q9 basis zero), the higher-order part vanishes and KBC is BGK."""
    cx, cy, _, _, _ = orc.lattice()
    M = _moments9(cx, cy)
    rng = np.random.default_rng(7 + seed)
    feq = orc.equilibrium(1.0 + 0.05 * rng.uniform(), 0.04 * rng.uniform(-1, 1),
                          0.04 * rng.uniform(-1, 1))
    target = np.zeros(9)
    target[4], target[5] = 1e-3 * rng.uniform(-1, 1, 2)
    f = feq + np.linalg.solve(M, target)
    for omega in (1.3, 1.98):
        np.testing.assert_allclose(orc.collide_node(f, omega, collision="kbc"),
                                   orc.collide_node(f, omega), rtol=0, atol=2e-16)


@pytest.mark.parametrize("seed", range(4))
def test_kbc_stabilizer_minimizes_quadratic_entropy(orc, seed):
    """The post-collision states of the KBC family differ by multiples of the
    higher-order part dh, which the output itself reveals:
    (f~ - f^eq) - (1 - omega)(f - f^eq) = beta (2 - gamma) dh.  The entropic stabilizer
    makes f~ - f^eq orthogonal to dh in <X|Y> = sum X Y / f^eq (the stationarity of the
    quadratic entropy along the family)."""
    f = _random_f(seed, amp=0.3)
    feq = _eq_of(orc, f)
    for omega in (1.5, 1.99):
        g = orc.collide_node(f, omega, collision="kbc")
        post = g - feq
        dh_dir = post - (1 - omega) * (f - feq)
        assert np.abs(dh_dir).max() > 1e-6           # a genuine entropic correction
        ip = np.sum(post * dh_dir / feq)
        scale = np.sqrt(np.sum(post * post / feq) * np.sum(dh_dir * dh_dir / feq))
        assert abs(ip) <= 1e-12 * scale


def test_kbc_rest_and_uniform_flow_are_fixed_points(orc):
    feq = orc.equilibrium(0.98, -0.03, 0.02)
    np.testing.assert_allclose(orc.collide_node(feq, 1.99, collision="kbc"), feq, rtol=0,
                               atol=4e-16)
    nx, ny = 24, 12
    s = OracleSim(np.zeros((ny, nx), np.uint8), tau=0.5002, bc_x=BCX_PERIODIC,
                  bc_y=BCY_PERIODIC, collision="kbc")
    S0 = np.repeat(np.repeat(feq[:, None, None], ny, 1), nx, 2)
    s.set_state(S0)
    s.step(20)
    np.testing.assert_allclose(s.state(), S0, rtol=0, atol=4e-16)


def test_kbc_drtt_equals_mea_b(orc):
    """KBC conserves momentum node by node: DRTT = MEA-B as for BGK."""
    w = workloads.cylinder_channel_200x80()
    s = OracleSim(w.mask, tau=0.505, uin=w.uin, box=w.box, collision="kbc")
    s.step(400)
    F = s.forces()
    scale = np.abs(F[:, 1]).max()
    assert scale > 0
    assert np.abs(F[:, 2] - F[:, 1]).max() <= 1e-11 * scale


def test_kbc_keeps_an_instance_finite_where_bgk_blows_up(orc):
    """The reason for the entropic variant: a batched-workload cylinder (72x36, D 7.2,
    Re 1305, tau_lb 0.50083) blows up under BGK within 1000 steps and stays finite under
    KBC for 3000."""
    w = [w for w in workloads.batched_instances() if w.name.startswith("b188_")][0]
    assert abs(w.tau - 0.50083) < 1e-5
    for coll, finite in (("bgk", False), ("kbc", True)):
        s = OracleSim(w.mask, w.tau, w.uin, box=w.box, collision=coll)
        s.step(1000 if coll == "bgk" else 3000)
        assert bool(np.isfinite(s.forces()).all()) == finite, coll


# --------------------------------------------------------------------------------------
# Stress integration over the staircase surface (Sec. III, Eq. stress_int and the
# non-equilibrium stress that follows it)
# --------------------------------------------------------------------------------------

def _state_pulling_to(orc, mask, f):
    """A stored state S whose pull on a doubly periodic lattice gives exactly the
    pre-collision field f at every fluid node: S_i(x) = f_i(x + c_i), and where x + c_i
    is solid the bounce-back reads S_i(x) as f_opp(i)(x)."""
    cx, cy, opp, _, _ = orc.lattice()
    ny, nx = mask.shape
    S = np.zeros_like(f)
    for i in range(9):
        S[i] = np.roll(np.roll(f[i], -int(cy[i]), axis=0), -int(cx[i]), axis=1)
        solid_ahead = np.roll(np.roll(mask, -int(cy[i]), axis=0), -int(cx[i]), axis=1) == 1
        S[i][solid_ahead] = f[opp[i]][solid_ahead]
    return S


def _spans(mask):
    """Number of solid runs and total solid length per row and per column."""
    def runs(rows):
        n = length = 0
        for r in rows:
            d = np.diff(np.concatenate([[0], r.astype(int), [0]]))
            n += int((d == 1).sum())
            length += int(r.sum())
        return n, length
    return runs(mask), runs(mask.T)


def test_si_pressure_part_closed_form(orc):
    """At rest with a linear density rho = 1 + a x, the pressure tractions on the
    staircase faces sum to F_x = -theta0 a sum_runs (len + 1) per row (each run's left
    and right faces sample p one node outside the body), F_y = 0."""
    cx, cy, _, w, th = orc.lattice()
    ny, nx = 30, 40
    mask = workloads.cylinder_mask(nx, ny, 19.5, 14.5, 6.0)
    a = 1e-3
    X = np.arange(nx)[None, :].repeat(ny, 0)
    f = np.zeros((9, ny, nx))
    for i in range(9):
        f[i] = w[i] * (1.0 + a * (X - 20))
    s = OracleSim(mask, tau=0.8, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    s.set_state(_state_pulling_to(orc, mask, f))
    s.step(1)
    np.testing.assert_allclose(s.pre()[:, mask == 0], f[:, mask == 0], rtol=0, atol=0)
    (nruns, length), _ = _spans(mask)
    F = s.forces()[0, 3]
    np.testing.assert_allclose(F[0], -th * a * (length + nruns), rtol=1e-12)
    assert abs(F[1]) <= 1e-15


def test_si_viscous_part_closed_form(orc):
    """At rest with a non-equilibrium part eps(x) w_i c_ix c_iy / theta0^2 (no mass, no
    momentum, Pi^neq_xy = eps(x)), eps = e0 + b x: the shear tractions give
    F_y = -(1 - omega/2) b sum_runs (len + 1) per row and F_x = 0; the pressure part
    cancels on the closed surface."""
    cx, cy, _, w, th = orc.lattice()
    ny, nx = 30, 40
    mask = workloads.cylinder_mask(nx, ny, 19.5, 14.5, 6.0)
    b, e0, tau = 2e-5, 1e-4, 0.8
    X = np.arange(nx)[None, :].repeat(ny, 0)
    eps = e0 + b * (X - 20)
    f = np.zeros((9, ny, nx))
    for i in range(9):
        f[i] = w[i] * (1.0 + eps * cx[i] * cy[i] / th ** 2)
    s = OracleSim(mask, tau=tau, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    s.set_state(_state_pulling_to(orc, mask, f))
    s.step(1)
    (nruns, length), _ = _spans(mask)
    F = s.forces()[0, 3]
    np.testing.assert_allclose(F[1], -(1 - 0.5 / tau) * b * (length + nruns), rtol=1e-10)
    assert abs(F[0]) <= 1e-15


def test_si_poiseuille_walls_closed_form(orc):
    """Body-force-driven channel whose walls are body rows (periodic x and y, solid rows
    0 and ny-1), at the tau where half-way bounce-back Poiseuille flow is exact: the
    staircase stress integral samples the linear shear stress half a node inside the
    fluid, so SI_x = (H - 1)/H of the exact N g (H fluid rows), while MEA-B gives N g."""
    for ny in (10, 18):
        nx, g = 8, 1e-6
        mask = np.zeros((ny, nx), np.uint8)
        mask[0] = 1
        mask[-1] = 1
        s = OracleSim(mask, tau=0.5 + np.sqrt(3 / 16), bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC,
                      g=(g, 0.0))
        s.step(40000)
        F = s.forces()[-1]
        H = ny - 2
        np.testing.assert_allclose(F[3, 0], (H - 1) / H * nx * H * g, rtol=1e-8)
        np.testing.assert_allclose(F[1, 0], nx * H * g, rtol=1e-8)
        assert abs(F[3, 1]) <= 1e-14


def test_si_rest_state_zero_on_closed_body(orc):
    """Uniform rest state: no stress, uniform pressure; the closed staircase gives zero."""
    mask = workloads.cylinder_mask(40, 30, 19.5, 14.5, 6.0)
    s = OracleSim(mask, tau=0.7, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC)
    s.step(3)
    assert np.abs(s.forces()[:, 3]).max() <= 1e-15


# --------------------------------------------------------------------------------------
# Bodies in rigid motion (moving-wall bounce-back of Sec. II on the body links; the
# two-term momentum exchange of Eq. rtt4/rtt5 and DRTT with moving walls)
# --------------------------------------------------------------------------------------

def test_comoving_uniform_flow_is_a_fixed_point_without_force(orc):
    """A body translating with the fluid (uniform flow f^eq(1, U), body velocity U):
    the moving-wall rule returns exactly the equilibrium populations, so the state is a
    fixed point and no estimator sees a force."""
    nx, ny = 40, 30
    mask = workloads.cylinder_mask(nx, ny, 19.5, 14.5, 6.0)
    U = (0.04, -0.02)
    feq = orc.equilibrium(1.0, *U)
    S0 = np.repeat(np.repeat(feq[:, None, None], ny, 1), nx, 2)
    s = OracleSim(mask, tau=0.7, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC, box=(6, 34, 4, 26),
                  body_motion=(U[0], U[1], 0.0, 0.0, 0.0))
    s.set_state(S0)
    s.step(10)
    fl = mask == 0
    np.testing.assert_allclose(s.state()[:, fl], S0[:, fl], rtol=0, atol=1e-14)
    F = s.forces()
    assert np.abs(F[:, [0, 1, 3]]).max() <= 1e-14
    # DRTT: a difference of box momenta of about 16 (rounding 1e-15 relative)
    assert np.abs(F[:, 2]).max() <= 1e-12


def test_moving_wall_rule_on_a_body_link(orc):
    """Brute force on one link: the population entering a fluid node from a rotating
    body is the opposite population of the node plus 2 w_i rho_w (c_i . u_w)/c_s^2, with
    u_w the rigid-body velocity at the half-way point of the link."""
    cx, cy, opp, w, th = orc.lattice()
    nx, ny = 16, 12
    mask = np.zeros((ny, nx), np.uint8)
    mask[6, 8] = 1
    om, xc, yc = 0.01, 7.0, 4.0
    s = OracleSim(mask, tau=0.8, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC,
                  body_motion=(0.02, 0.01, om, xc, yc))
    S = workloads.near_rest_state(nx, ny, seed=5, amp=0.1)
    s.set_state(S)
    s.step(1)
    f = s.pre()
    for i in range(1, 9):
        x, y = 8 + cx[i], 6 + cy[i]          # fluid node whose pull along i starts in the body
        xw, yw = x - cx[i] / 2, y - cy[i] / 2
        uw = np.array([0.02 - om * (yw - yc), 0.01 + om * (xw - xc)])
        expect = S[opp[i], y, x] + 2 * w[i] * (cx[i] * uw[0] + cy[i] * uw[1]) / th
        assert abs(f[i, y, x] - expect) <= 1e-16


def test_rotating_cylinder_mirror_symmetry_and_magnus_sign(orc):
    """A cylinder on the centreline of a walled channel: reversing the rotation mirrors
    the flow, so drag is unchanged and lift changes sign; with the flow along +x, a
    counter-clockwise rotation (Omega > 0) drives the fluid faster below the body and
    the lift is negative (Magnus).  DRTT equals MEA-B with moving walls."""
    nx, ny = 120, 41
    mask = workloads.cylinder_mask(nx, ny, 30, 20, 6)
    box = workloads.default_box(mask, 4)
    F = {}
    for om in (0.004, -0.004):
        s = OracleSim(mask, tau=0.6, uin=np.full(ny, 0.04), box=box,
                      body_motion=(0.0, 0.0, om, 30.0, 20.0))
        s.step(1500)
        F[om] = s.forces()
    a, b = F[0.004], F[-0.004]
    scale = np.abs(a[:, 1]).max()
    np.testing.assert_allclose(a[:, :, 0], b[:, :, 0], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(a[:, :, 1], -b[:, :, 1], rtol=0, atol=1e-12 * scale)
    assert a[-500:, 1, 1].mean() < 0
    assert np.abs(a[:, 2] - a[:, 1]).max() <= 1e-11 * scale


# --------------------------------------------------------------------------------------
# A body that moves through the grid: the mask changes between steps (moving-wall
# bounce-back of Sec. II on the links of each mask; every step's forces with the
# geometry it was taken with; uncovered nodes refilled at the wall velocity)
# --------------------------------------------------------------------------------------

def test_set_mask_to_the_same_mask_changes_nothing(orc):
    """Setting the mask it already has: no impulse, same state, and the forces of the
    whole run bitwise those of a run without the call (DRTT across the call included)."""
    nx, ny = 60, 30
    mask = workloads.cylinder_mask(nx, ny, 20, 14.5, 5)
    box = (8, 33, 4, 26)
    S0 = workloads.near_rest_state(nx, ny, seed=21, amp=0.05)
    runs = []
    for call in (False, True):
        s = OracleSim(mask, tau=0.7, uin=np.full(ny, 0.03), box=box)
        s.set_state(S0)
        s.step(15)
        if call:
            before = s.state()
            imp = s.set_mask(mask.copy())
            assert np.all(imp == 0.0)
            assert np.array_equal(s.state(), before)
        s.step(15)
        runs.append((s.state(), s.forces()))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


def test_uncovered_nodes_refill_and_covered_momentum_brute_force(orc):
    """Hand-enumerated neighbours: a 2x2 body moved one node to the right, and a 3x3
    block removed.  Every uncovered node holds f^eq(rho, u_w) with rho the mean density
    of its neighbours that are fluid in both masks (rho_w = 1 when none is) and u_w the
    rigid-body velocity at the node; the impulse is the momentum of the covered nodes
    minus that of the refilled ones; no other node changes."""
    cx, cy, opp, w, th = orc.lattice()
    nx, ny = 14, 12
    old = np.zeros((ny, nx), np.uint8)
    old[4:6, 5:7] = 1          # 2x2 body at x 5..6, y 4..5
    old[8:11, 9:12] = 1        # 3x3 block at x 9..11, y 8..10
    new = np.zeros((ny, nx), np.uint8)
    new[4:6, 6:8] = 1          # the 2x2 body at x 6..7
    mo = (0.02, 0.01, 0.003, 6.5, 4.5)
    S = workloads.near_rest_state(nx, ny, seed=8, amp=0.1)
    s = OracleSim(old, tau=0.8, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC, body_motion=mo)
    s.set_state(S)
    imp = s.set_mask(new)
    T = s.state()

    def rho(x, y):
        return S[:, y, x].sum()

    def uw(x, y):
        return (mo[0] - mo[2] * (y - mo[4]), mo[1] + mo[2] * (x - mo[3]))

    # neighbours fluid in both masks, listed by hand
    fresh = {
        (5, 4): [(4, 4), (5, 3), (4, 5), (4, 3), (6, 3)],
        (5, 5): [(4, 5), (5, 6), (4, 6), (6, 6), (4, 4)],
        (10, 9): [],  # every neighbour was solid
    }
    for x in range(9, 12):
        for y in range(8, 11):
            if (x, y) == (10, 9):
                continue
            nb = []
            for i in range(1, 9):
                ax, ay = x + cx[i], y + cy[i]
                if not (9 <= ax <= 11 and 8 <= ay <= 10):
                    nb.append((ax, ay))
            fresh[(x, y)] = nb
    P = np.zeros(2)
    for (x, y) in [(7, 4), (7, 5)]:        # covered
        P += [np.dot(cx, S[:, y, x]), np.dot(cy, S[:, y, x])]
    changed = np.zeros((ny, nx), bool)
    for (x, y), nb in fresh.items():
        r = np.mean([rho(a, b) for a, b in nb]) if nb else 1.0
        feq = orc.equilibrium(r, *uw(x, y))
        np.testing.assert_allclose(T[:, y, x], feq, rtol=0, atol=1e-15)
        P -= [np.dot(cx, T[:, y, x]), np.dot(cy, T[:, y, x])]
        changed[y, x] = True
    np.testing.assert_allclose(imp, P, rtol=0, atol=1e-15)
    assert np.array_equal(T[:, ~changed], S[:, ~changed])


def test_comoving_translating_body_keeps_a_uniform_flow(orc):
    """A cylinder carried by a uniform flow f^eq(1, U), moved one node every 1/|U|
    steps with body velocity U: the refilled nodes get exactly the flow's equilibrium,
    the state stays uniform, no estimator sees a force and the impulses cancel (the
    shape moves unchanged)."""
    nx, ny = 48, 30
    U = (0.04, 0.0)
    feq = orc.equilibrium(1.0, *U)
    S0 = np.repeat(np.repeat(feq[:, None, None], ny, 1), nx, 2)
    s = OracleSim(workloads.cylinder_mask(nx, ny, 15, 14.5, 5), tau=0.7, bc_x=BCX_PERIODIC,
                  bc_y=BCY_PERIODIC, box=(6, 42, 4, 26), body_motion=(U[0], U[1], 0.0, 0.0, 0.0))
    s.set_state(S0)
    for k in range(1, 6):
        s.step(25)
        imp = s.set_mask(workloads.cylinder_mask(nx, ny, 15 + k, 14.5, 5))
        assert np.abs(imp).max() <= 1e-14
        fl = s._mask_keep == 0
        np.testing.assert_allclose(s.state()[:, fl], S0[:, fl], rtol=0, atol=1e-14)
    s.step(10)
    F = s.forces()
    # sums of ~40 face pressures rho/3 (and link populations) cancelling: rounding 1e-14
    assert np.abs(F[:, [0, 1, 3]]).max() <= 5e-14
    assert np.abs(F[:, 2]).max() <= 1e-12


def test_mask_change_mass_and_momentum_bookkeeping(orc):
    """Fluid momentum after a change = momentum before - impulse; fluid mass after =
    mass before - covered mass + refilled mass (periodic lattice, random state, a body
    moved diagonally and turning)."""
    nx, ny = 40, 32
    old = workloads.cylinder_mask(nx, ny, 18, 15, 6)
    new = workloads.cylinder_mask(nx, ny, 19, 16, 6)
    cx, cy, _, _, _ = orc.lattice()
    s = OracleSim(old, tau=0.7, bc_x=BCX_PERIODIC, bc_y=BCY_PERIODIC,
                  body_motion=(0.03, 0.02, 0.004, 19.0, 16.0))
    s.set_state(workloads.near_rest_state(nx, ny, seed=4, amp=0.05))
    s.step(5)
    S = s.state()
    imp = s.set_mask(new)
    T = s.state()

    def mom(X, m):
        fl = m == 0
        return np.array([np.tensordot(cx, X, 1)[fl].sum(), np.tensordot(cy, X, 1)[fl].sum()])

    np.testing.assert_allclose(mom(T, new), mom(S, old) - imp, rtol=0, atol=1e-12)
    cov = (old == 0) & (new == 1)
    fre = (old == 1) & (new == 0)
    assert cov.sum() > 0 and fre.sum() > 0
    mass_new = T.sum(0)[new == 0].sum()
    expect = S.sum(0)[old == 0].sum() - S.sum(0)[cov].sum() + T.sum(0)[fre].sum()
    assert abs(mass_new - expect) <= 1e-12
    assert np.abs(imp).max() > 0


def test_drtt_equals_mea_b_with_a_translating_body(orc):
    """DRTT equals MEA-B at every step of a run whose body moves through the grid (one
    node every 20 steps, the control volume moved with it every other time): each
    step's forces use the geometry of that step, so the identity of fixed bodies holds
    across every change."""
    nx, ny = 100, 40
    U = 0.05
    s = OracleSim(workloads.cylinder_mask(nx, ny, 30, 19.5, 6), tau=0.65,
                  uin=np.full(ny, 0.04), box=(20, 41, 8, 32),
                  body_motion=(U, 0.0, 0.0, 0.0, 0.0))
    imps = []
    for k in range(1, 11):
        s.step(20)
        box = (20 + k // 2 * 2, 41 + k // 2 * 2, 8, 32) if k % 2 == 0 else None
        imps.append(s.set_mask(workloads.cylinder_mask(nx, ny, 30 + k, 19.5, 6), box=box))
    s.step(20)
    F = s.forces()
    scale = np.abs(F[:, 1]).max()
    assert scale > 0
    assert np.abs(F[:, 2] - F[:, 1]).max() <= 1e-11 * scale
    assert np.all(np.isfinite(F))
    # the fluid ahead of the body is pushed: the fluid hands momentum to the body
    # (covered fluid moves slower than the refilled wake) with a nonzero impulse
    assert all(np.abs(i).max() > 0 for i in imps)


@pytest.mark.parametrize("threads", [2, 5])
def test_row_parallel_oracle_is_bitwise_serial(orc, threads):
    """The oracle's row loops may run on several threads; every force sum is still
    formed in the serial order, so states, records and forces are bitwise the same as
    with one thread (cylinder channel with inlet, outlet, walls and a box; complex
    arithmetic too)."""
    w = workloads.cylinder_channel_200x80()
    outs = []
    for n in (1, threads):
        old = orc.set_threads(n)
        try:
            s = OracleSim(w.mask, tau=w.tau, uin=w.uin, box=w.box)
            s.set_state(workloads.near_rest_state(w.nx, w.ny, seed=4, amp=0.03))
            s.step(30)
            J = orc.objective(w.mask, 1 / complex(w.tau, 1e-30), w.uin, 20, 10, 10, w=(1.0, 0.5))
            outs.append((s.state(), s.records(), s.forces(), J))
        finally:
            orc.set_threads(old)
    a, b = outs
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2], equal_nan=True) and a[3] == b[3]


# --------------------------------------------------------------------------------------
# Boundary pressure coefficient (Sec. V, the C_p equation)
# --------------------------------------------------------------------------------------

def _brute_boundary_nodes(mask, periodic_x=False, periodic_y=False):
    """Fluid nodes with a solid node among their eight lattice neighbours (a wrapped
    neighbour across a periodic edge counts), row-major."""
    ny, nx = mask.shape
    out = []
    for y in range(ny):
        for x in range(nx):
            if mask[y, x]:
                continue
            hit = False
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == 0 and dy == 0:
                        continue
                    tx, ty = x + dx, y + dy
                    if periodic_x:
                        tx %= nx
                    if periodic_y:
                        ty %= ny
                    if 0 <= tx < nx and 0 <= ty < ny and mask[ty, tx]:
                        hit = True
            if hit:
                out.append(y * nx + x)
    return out


def test_boundary_cp_rest_state_is_zero(orc):
    """At rest (f = w_i, p = theta0 everywhere) C_p vanishes at every boundary fluid node,
    with p_inf sampled at a reference node or taken as rho_ref theta0."""
    w = workloads.cylinder_channel_200x80()
    s = OracleSim(w.mask, tau=w.tau, uin=w.uin)
    for ref in ((5, 40), None):
        nodes, cp = s.boundary_cp(ref, rho_ref=1.0, u_ref=0.05)
        assert nodes.tolist() == _brute_boundary_nodes(w.mask)
        if ref is not None:
            assert np.all(cp == 0.0)   # the same sum of w_i on both sides
        else:
            # sum w_i = 1 up to its rounding (9 terms): |C_p| <= theta0 9 2^-53 / (U^2/2)
            assert np.abs(cp).max() <= 9 * 2.0 ** -53 / 3 / (0.5 * 0.05 ** 2)


@pytest.mark.parametrize("periodic", [False, True])
def test_boundary_cp_linear_density_closed_form(orc, periodic):
    """A linear density field rho = 1 + a x + b y at rest (f = w_i rho): at a boundary
    fluid node C_p = theta0 (a (x - x_inf) + b (y - y_inf)) / (rho_ref U^2 / 2); the
    boundary nodes are the fluid nodes next to the body (brute-force enumeration)."""
    nx, ny = 48, 30
    mask = workloads.cylinder_mask(nx, ny, 23.5, 14.0, 6.0)
    mask[0:3, 40:44] = 1          # a second body on the first rows: wraps when periodic
    bc = BCX_PERIODIC if periodic else BCX_INLET_OUTLET
    bcy = BCY_PERIODIC if periodic else BCY_WALL
    s = OracleSim(mask, tau=0.8, uin=None if periodic else np.full(ny, 0.02), bc_x=bc, bc_y=bcy)
    _, _, _, wts, th = orc.lattice()
    a, b = 3e-4, -2e-4
    yy, xx = np.mgrid[0:ny, 0:nx]
    rho = 1.0 + a * xx + b * yy
    s.set_state(wts[:, None, None] * rho[None])
    rho_ref, U, ref = 1.2, 0.04, (2, 20)
    nodes, cp = s.boundary_cp(ref, rho_ref=rho_ref, u_ref=U)
    assert nodes.tolist() == _brute_boundary_nodes(mask, periodic, periodic)
    y, x = nodes // nx, nodes % nx
    want = th * (a * (x - ref[0]) + b * (y - ref[1])) / (0.5 * rho_ref * U * U)
    np.testing.assert_allclose(cp, want, rtol=0, atol=1e-12 * np.abs(want).max())
    nodes2, cp2 = s.boundary_cp(None, rho_ref=rho_ref, u_ref=U)
    want2 = th * (rho[y, x] - rho_ref) / (0.5 * rho_ref * U * U)
    np.testing.assert_allclose(cp2, want2, rtol=0, atol=1e-12 * np.abs(want2).max())
    with pytest.raises(ValueError):
        s.boundary_cp((23, 14), rho_ref=1.0, u_ref=U)   # solid reference node


def test_boundary_cp_symmetric_cylinder_is_mirror_symmetric(orc):
    """A cylinder on the centreline of a walled channel with a uniform inlet: the flow is
    mirror symmetric about the centreline, so C_p(x, y) = C_p(x, ny - 1 - y); the front
    stagnation node carries the largest C_p, positive, and the flanks negative values."""
    nx, ny = 120, 41
    mask = workloads.cylinder_mask(nx, ny, 30, 20, 6)
    s = OracleSim(mask, tau=0.8, uin=np.full(ny, 0.04))
    s.step(600)
    nodes, cp = s.boundary_cp((3, 20), rho_ref=1.0, u_ref=0.04)
    y, x = nodes // nx, nodes % nx
    val = dict(zip(zip(x.tolist(), y.tolist()), cp.tolist()))
    for (xi, yi), c in val.items():
        assert abs(c - val[(xi, ny - 1 - yi)]) <= 1e-10 * np.abs(cp).max()
    front = val[(23, 20)]
    assert front == max(val.values()) and front > 0.5
    assert val[(30, 13)] < 0 and val[(30, 27)] < 0
