"""A body moving through the grid on the three-dimensional GPU path (lbm3d_set_mask)
against the 3-D oracle with the same calls: the mask (and control volume) replaced
between steps, uncovered nodes refilled at the rigid-body velocity, every step's forces
taken with its own geometry.  FP64 populations, forces and impulses to 1e-10; 32-bit
storage forces and impulses to 1e-4 of their largest value; FP16 deviations to 5e-2."""
import numpy as np
import pytest

from oracle import d3q27 as D
from workloads import d3

from test_gpu3d_parity import TOL64, _force_err, _pop_err, _sim3

pytestmark = pytest.mark.gpu

NX, NY, NZ, X0, YC, ZC, R = 48, 20, 20, 14, 9.5, 9.5, 4
U = (0.05, 0.0, 0.0)
W = (0.0, 0.0, 0.002)


def _mask(k):
    return d3.sphere_mask(NX, NY, NZ, X0 + k, YC, ZC, R)


def _towed_run(side, moves, chunk):
    """`moves` times: chunk steps, then the sphere moved one node along x with its
    motion centred on the new position, the control volume moved along every second
    time; then chunk more steps.  Returns the impulses."""
    imps = []
    for k in range(1, moves + 1):
        side.step(chunk)
        box = (7 + k, 22 + k, 3, 17, 3, 17) if k % 2 == 0 else None
        imps.append(side.set_mask(_mask(k), box))
        side.set_body_motion(U, W, (X0 + k, YC, ZC))
    side.step(chunk)
    return np.array(imps)


@pytest.fixture(scope="module")
def towed_reference():
    """Oracle run: a sphere (radius 4) towed at 0.05 through a walled duct with inflow,
    turning slowly, moved one node every 20 steps, 6 moves (140 steps)."""
    o = D.OracleSim3(_mask(0), tau=0.65, uin=np.full((NZ, NY), 0.03),
                     box=(7, 22, 3, 17, 3, 17), body_motion=(U, W, (X0, YC, ZC)))
    io = _towed_run(o, 6, 20)
    return io, o.state(), o.forces()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32dev", "fp32sr", "fp16dev"])
def test_towed_sphere_against_oracle(precision, towed_reference):
    io, So, Fo = towed_reference
    g = _sim3(_mask(0), 0.65, np.full((NZ, NY), 0.03), precision=precision,
              box=(7, 22, 3, 17, 3, 17), max_record=200)
    g.set_body_motion(U, W, (X0, YC, ZC))
    ig = _towed_run(g, 6, 20)
    Fg = g.forces()
    assert Fg.shape == Fo.shape == (140, 4, 3)
    e = _force_err(Fg, Fo)
    ei = np.abs(ig - io).max() / np.abs(io).max()
    print(precision, "towed sphere force errors (A, B, DRTT, SI):", e, "impulse", ei)
    tol = {"fp64": TOL64, "fp32": 1e-4, "fp32dev": 1e-4, "fp32sr": 1e-4, "fp16dev": 5e-2}[precision]
    assert np.all(e <= tol), e
    assert ei <= tol, ei
    if precision == "fp64":
        assert _pop_err(g.populations(), So, _mask(6)) <= TOL64
        sc = np.abs(Fg[:, 1]).max()
        assert np.abs(Fg[:, 2] - Fg[:, 1]).max() <= 1e-10 * sc


def test_body_crossing_the_periodic_seams():
    """A block moved diagonally across the periodic x and z edges from a random state
    (FP64): refills take neighbours across the seams; populations, forces and impulses
    to 1e-10."""
    nx, ny, nz = 40, 16, 14
    S0 = d3.near_rest_state3(nx, ny, nz, seed=41, amp=0.05)

    def mask(k):
        m = np.zeros((nz, ny, nx), np.uint8)
        xs = [(nx - 3 + k + j) % nx for j in range(4)]
        zs = [(nz - 2 + k + j) % nz for j in range(3)]
        m[np.ix_(zs, range(6, 10), xs)] = 1
        return m

    mo = ((0.04, 0.0, 0.04), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    o = D.OracleSim3(mask(0), tau=0.7, bc_x=D.BCX_PERIODIC, bc_y=D.BC_WALL,
                     bc_z=D.BC_PERIODIC, body_motion=mo)
    g = _sim3(mask(0), 0.7, None, precision="fp64", bc_x=1, bc_y=0, bc_z=1, max_record=100)
    g.set_body_motion(*mo)
    o.set_state(S0)
    g.set_populations(S0)
    ig, io = [], []
    for k in range(1, 6):
        o.step(8)
        g.step(8)
        io.append(o.set_mask(mask(k)))
        ig.append(g.set_mask(mask(k)))
    o.step(8)
    g.step(8)
    assert _pop_err(g.populations(), o.state(), mask(5)) <= TOL64
    e = _force_err(g.forces(), o.forces(), (0, 1, 3))
    assert np.all(e <= TOL64), e
    io, ig = np.array(io), np.array(ig)
    assert np.abs(ig - io).max() <= 1e-10 * np.abs(io).max()


def test_set_mask_to_the_same_mask_is_bitwise_a_no_op():
    """Re-setting the present mask and box between two calls changes nothing: state and
    forces bitwise those of the uninterrupted run (FP32, sphere duct)."""
    w = d3.sphere_channel_64x32x32()
    runs = []
    for call in (False, True):
        g = _sim3(w.mask, w.tau, w.uin, precision="fp32", box=w.box, max_record=100)
        g.step(50)
        if call:
            imp = g.set_mask(w.mask, w.box)
            assert np.all(imp == 0.0)
        g.step(50)
        runs.append((g.populations(), g.forces()))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


def test_removed_body_leaves_a_uniform_state_and_the_plan_follows():
    """Uniform flow past a sphere on a fully periodic lattice; the sphere removed: the
    impulse is the covered-minus-refilled momentum of the oracle (FP64, 1e-10), the plan
    reports no links, and the next steps record zero body forces."""
    nx, ny, nz = 32, 16, 16
    m = d3.sphere_mask(nx, ny, nz, 12, 7.5, 7.5, 3.5)
    S0 = d3.near_rest_state3(nx, ny, nz, seed=43, amp=0.02)
    o = D.OracleSim3(m, tau=0.8, bc_x=D.BCX_PERIODIC, bc_y=D.BC_PERIODIC, bc_z=D.BC_PERIODIC)
    g = _sim3(m, 0.8, None, precision="fp64", bc_x=1, bc_y=1, bc_z=1, max_record=20)
    o.set_state(S0)
    g.set_populations(S0)
    o.step(10)
    g.step(10)
    empty = np.zeros_like(m)
    io, ig = o.set_mask(empty), g.set_mask(empty)
    assert np.abs(ig - io).max() <= 1e-10 * max(np.abs(io).max(), 1e-12)
    assert g.info().n_links == 0 and g.info().n_fluid == nx * ny * nz
    o.step(5)
    g.step(5)
    assert _pop_err(g.populations(), o.state(), empty) <= TOL64
    F = g.forces()
    assert F.shape == (15, 4, 3)
    assert np.all(F[10:, [0, 1, 3]] == 0.0)
