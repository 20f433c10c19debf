"""Bodies in rigid motion on the three-dimensional GPU path against the 3-D oracle:
the moving-wall bounce-back of Sec. II on every body link with the rigid-body velocity
at the link's half-way point, and the two-term momentum exchange with the returned
population (Eq. rtt4/rtt5).  FP64 to 1e-10; 32-bit storage within the bounds of the
body-at-rest runs."""
import numpy as np
import pytest

from oracle import d3q27 as D
from workloads import d3

from test_gpu3d_parity import CASES, TOL64, _force_err, _pop_err, _sim3

pytestmark = pytest.mark.gpu

MOTIONS = {
    "translation": ((0.02, -0.01, 0.015), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
    "rotation": ((0.0, 0.0, 0.0), (0.001, -0.002, 0.003), (1.5, -1.0, 0.5)),
    "both": ((-0.01, 0.01, 0.0), (0.0, 0.0, -0.003), (-1.0, 0.5, 0.0)),
}


def _motion(mask, name):
    """The motion `name` about the centroid of the solid nodes (offset as listed), the
    angular velocity capped so that no solid node moves faster than 0.03."""
    U, W, off = MOTIONS[name]
    zc, yc, xc = np.argwhere(mask).mean(axis=0)
    c = np.array([xc, yc, zc]) + np.array(off)
    zs, ys, xs = np.nonzero(mask)
    r = np.sqrt((xs - c[0]) ** 2 + (ys - c[1]) ** 2 + (zs - c[2]) ** 2).max()
    W = np.array(W)
    nw = np.linalg.norm(W)
    if nw * r > 0.03:
        W = W * 0.03 / (nw * r)
    return (np.array(U), W, c)


@pytest.mark.parametrize("motion", list(MOTIONS))
@pytest.mark.parametrize("name", ["sphere_walls_box", "sphere_periodic_box",
                                  "extruded_periodic_span", "edges_no_box"])
def test_fp64_moving_body_small_cases(name, motion):
    mk, (bx, by, bz), box, u = CASES[name]
    mask = mk()
    nz, ny, nx = mask.shape
    uin = None if bx == 1 else np.full((nz, ny), u)
    mo = _motion(mask, motion)
    S0 = d3.near_rest_state3(nx, ny, nz, seed=60 + len(name), amp=0.05)
    o = D.OracleSim3(mask, tau=0.7, uin=uin, bc_x=bx, bc_y=by, bc_z=bz, box=box, body_motion=mo)
    o.set_state(S0)
    o.step(30)
    g = _sim3(mask, 0.7, uin, precision="fp64", bc_x=bx, bc_y=by, bc_z=bz, box=box,
              max_record=64)
    g.set_body_motion(*mo)
    g.set_populations(S0)
    g.step(30)
    assert _pop_err(g.populations(), o.state(), mask) <= TOL64
    cols = (0, 1, 2, 3) if box is not None else (0, 1, 3)
    e = _force_err(g.forces(), o.forces(), cols)
    assert np.all(e <= TOL64), e


@pytest.fixture(scope="module")
def rotating_sphere_reference():
    """The sphere duct with the sphere turning about z at a surface speed of half the
    inlet speed, 300 steps from rest."""
    w = d3.sphere_channel_64x32x32()
    mo = ((0, 0, 0), (0, 0, 0.5 * 0.04 / 5.0), (20.0, 15.5, 15.5))
    o = D.OracleSim3(w.mask, tau=w.tau, uin=w.uin, box=w.box, body_motion=mo)
    o.step(300)
    return w, mo, o.state(), o.forces()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32dev", "fp32sr", "fp16dev"])
def test_rotating_sphere_duct(precision, rotating_sphere_reference):
    w, mo, So, Fo = rotating_sphere_reference
    g = _sim3(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=300)
    g.set_body_motion(*mo)
    Fg = g.run(300)
    assert np.isfinite(Fg).all()
    e = _force_err(Fg, Fo)
    print(precision, "rotating sphere force errors (A, B, DRTT, SI):", e)
    tol = {"fp64": np.full(4, TOL64), "fp32": np.array([1e-4, 1e-4, 1e-3, 1e-4]),
           "fp32dev": np.array([1e-4, 1e-4, 1e-3, 1e-4]),
           "fp32sr": np.array([1e-4, 1e-4, 1e-3, 1e-4]), "fp16dev": np.full(4, 5e-2)}[precision]
    assert np.all(e <= tol), e
    if precision == "fp64":
        assert _pop_err(g.populations(), So, w.mask) <= TOL64
    assert np.all(Fg[-50:, :, 1].mean(axis=0) < 0)   # Magnus: Omega_z > 0, flow along +x


def test_zero_motion_is_the_resting_body_and_forces_off_same_state():
    """A zero motion set after a non-zero one gives the resting body bitwise; with a
    body in motion, stepping without forces gives the same populations as with them."""
    w = d3.sphere_channel_64x32x32()
    runs = []
    for mo in (None, ((0.01, 0, 0), (0, 0.002, 0), (20, 15.5, 15.5))):
        g = _sim3(w.mask, w.tau, w.uin, precision="fp32", box=w.box, max_record=50)
        if mo is not None:
            g.set_body_motion(*mo)
            g.set_body_motion()
        g.step(40)
        runs.append((g.populations(), g.forces()))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    pops = []
    for schemes in (("A", "B", "DRTT", "SI"), ()):
        g = _sim3(w.mask, w.tau, w.uin, precision="fp64", box=w.box, max_record=50)
        g.set_body_motion((0.005, 0.0, 0.0), (0.0, 0.0, 0.004), (20.0, 15.5, 15.5))
        g.step(40, schemes)
        pops.append(g.populations())
    np.testing.assert_array_equal(pops[0], pops[1])


def test_moving_body_with_the_regularized_collision():
    """A turning sphere with the regularized collision at tau_lb 0.505, FP64, against the
    oracle: populations and forces to 1e-10."""
    mk, (bx, by, bz), box, u = CASES["sphere_walls_box"]
    mask = mk()
    nz, ny, nx = mask.shape
    mo = _motion(mask, "both")
    S0 = d3.near_rest_state3(nx, ny, nz, seed=91, amp=0.05)
    uin = np.full((nz, ny), u)
    o = D.OracleSim3(mask, tau=0.505, uin=uin, box=box, body_motion=mo, collision="regularized")
    o.set_state(S0)
    o.step(30)
    g = _sim3(mask, 0.505, uin, precision="fp64", box=box, max_record=64, collision="regularized")
    g.set_body_motion(*mo)
    g.set_populations(S0)
    g.step(30)
    assert _pop_err(g.populations(), o.state(), mask) <= TOL64
    e = _force_err(g.forces(), o.forces())
    assert np.all(e <= TOL64), e
