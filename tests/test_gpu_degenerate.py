"""Degenerate lattices on the GPU against the oracles: the smallest grids the ABI
accepts (3 x 3 in two dimensions, 2 x 2 x 2 in three), a single fluid node walled in by
the body on every side (every pull a bounce-back, every direction a link), and grids
with no fluid node at all (nothing moves, every force is zero).  FP64 to 1e-10; the
reduced storages (binary32 with rounding to nearest or stochastic, binary32 and binary16
deviations) to bounds set by their rounding."""
import numpy as np
import pytest

import workloads
from oracle import BCX_INLET_OUTLET, BCX_PERIODIC, BCY_PERIODIC, BCY_WALL, OracleSim
from oracle import d3q27 as D
from workloads import d3

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _close(Sg, So, mask):
    fl = mask == 0
    return float((np.abs(Sg - So)[:, fl] / np.abs(So)[:, fl]).max())


def _forces_close(Fg, Fo, cols):
    """Relative to the largest force of the run: the stress integral of a node walled in
    on all sides cancels to zero (exactly on the GPU, to rounding in the oracle)."""
    scale = max(np.abs(Fo[:, k]).max() for k in cols)
    assert scale > 0
    for k in cols:
        assert np.abs(Fg[:, k] - Fo[:, k]).max() <= TOL * scale, k


CASES_2D = {
    # name: (mask, bc_x, bc_y, inlet speed)
    "3x3_periodic": (np.zeros((3, 3), np.uint8), BCX_PERIODIC, BCY_PERIODIC, None),
    "3x3_channel": (np.zeros((3, 3), np.uint8), BCX_INLET_OUTLET, BCY_WALL, 0.04),
    "single_fluid_node": (np.pad(np.zeros((1, 1), np.uint8), 2, constant_values=1),
                          BCX_PERIODIC, BCY_PERIODIC, None),
}


@pytest.mark.parametrize("name", list(CASES_2D))
def test_degenerate_2d_against_oracle(name):
    from paper_2210_10377_amd import Sim
    mask, bx, by, u = CASES_2D[name]
    ny, nx = mask.shape
    uin = None if u is None else np.full(ny, u)
    S0 = workloads.near_rest_state(nx, ny, seed=90 + len(name), amp=0.05)
    g = Sim(mask, 0.7, uin, precision="fp64", bc_x=bx, bc_y=by, max_record=32)
    o = OracleSim(mask, tau=0.7, uin=uin, bc_x=bx, bc_y=by)
    g.set_populations(S0)
    o.set_state(S0)
    g.step(25)
    o.step(25)
    assert _close(g.populations(), o.state(), mask) <= TOL
    Fg, Fo = g.forces(), o.forces()
    assert Fg.shape == (25, 5, 2)
    if mask.any():
        assert g.info().n_links == 8
        _forces_close(Fg, Fo, (0, 1, 3))
    else:
        assert np.all(Fg[:, [0, 1, 3]] == 0.0)


def test_no_fluid_node_2d():
    """An all-solid channel: the step writes nothing (after an even number of steps the
    buffer that was set holds exactly what was set) and every body force is exactly
    zero; DRTT, without a box, is NaN."""
    from paper_2210_10377_amd import Sim
    mask = np.ones((20, 40), np.uint8)
    S0 = workloads.near_rest_state(40, 20, seed=97, amp=0.05)
    g = Sim(mask, 0.7, np.full(20, 0.03), precision="fp64", max_record=8)
    assert g.info().n_fluid == 0 and g.info().n_links == 0
    g.set_populations(S0)
    g.step(4)
    np.testing.assert_array_equal(g.populations(), S0)
    F = g.forces()
    assert F.shape == (4, 5, 2)
    assert np.all(F[:, [0, 1, 3]] == 0.0) and np.all(np.isnan(F[:, 2]))


CASES_3D = {
    "2x2x2_periodic": (np.zeros((2, 2, 2), np.uint8), (1, 1, 1), None),
    "2x2x2_channel": (np.zeros((2, 2, 2), np.uint8), (0, 0, 0), 0.04),
    "single_fluid_node": (np.pad(np.zeros((1, 1, 1), np.uint8), 2, constant_values=1),
                          (1, 1, 1), None),
}


@pytest.mark.parametrize("name", list(CASES_3D))
def test_degenerate_3d_against_oracle(name):
    from paper_2210_10377_amd import Sim3
    mask, (bx, by, bz), u = CASES_3D[name]
    nz, ny, nx = mask.shape
    uin = None if u is None else np.full((nz, ny), u)
    S0 = d3.near_rest_state3(nx, ny, nz, seed=95 + len(name), amp=0.05)
    g = Sim3(mask, 0.7, uin, precision="fp64", bc_x=bx, bc_y=by, bc_z=bz, max_record=32)
    o = D.OracleSim3(mask, tau=0.7, uin=uin, bc_x=bx, bc_y=by, bc_z=bz)
    g.set_populations(S0)
    o.set_state(S0)
    g.step(25)
    o.step(25)
    assert _close(g.populations(), o.state(), mask) <= TOL
    Fg, Fo = g.forces(), o.forces()
    assert Fg.shape == (25, 4, 3)
    if mask.any():
        assert g.info().n_links == 26
        _forces_close(Fg, Fo, (0, 1, 3))
    else:
        assert np.all(Fg[:, [0, 1, 3]] == 0.0)


def test_no_fluid_node_3d():
    from paper_2210_10377_amd import Sim3
    mask = np.ones((6, 6, 6), np.uint8)
    S0 = d3.near_rest_state3(6, 6, 6, seed=99, amp=0.05)
    g = Sim3(mask, 0.7, None, precision="fp64", bc_x=1, bc_y=1, bc_z=1, max_record=8)
    assert g.info().n_fluid == 0 and g.info().n_links == 0
    g.set_populations(S0)
    g.step(4)
    np.testing.assert_array_equal(g.populations(), S0)
    F = g.forces()
    assert F.shape == (4, 4, 3)
    assert np.all(F[:, [0, 1, 3]] == 0.0) and np.all(np.isnan(F[:, 2]))


# Reduced storages on the same lattices, 25 steps from a random state exactly
# representable in the storage.  Population bounds (relative): binary32 rounding of
# ~6e-8 per step (stochastic rounding up to twice that), binary32 deviations ~1e-7 of the
# population overall, binary16 deviations 2^-11 of deviations of 5 %; forces relative to
# the largest of the run.
REDUCED = [("fp32", 1e-5, 1e-4), ("fp32dev", 1e-6, 1e-4), ("fp32sr", 1e-5, 1e-4),
           ("fp16dev", 5e-3, 5e-2)]


def _state2(nx, ny, precision, seed):
    if precision == "fp16dev":
        return workloads.near_rest_state_fp16dev(nx, ny, seed=seed, amp=0.05)
    if precision == "fp32dev":
        return workloads.near_rest_state_dev(nx, ny, seed=seed, amp=0.05, dtype=np.float32)
    return workloads.near_rest_state(nx, ny, seed=seed, amp=0.05, dtype=np.float32)


def _rel_force_err(Fg, Fo, cols):
    scale = max(np.abs(Fo[:, k]).max() for k in cols)
    return max(float(np.abs(Fg[:, k] - Fo[:, k]).max()) for k in cols) / scale


@pytest.mark.parametrize("precision,tol_pop,tol_f", REDUCED)
@pytest.mark.parametrize("name", list(CASES_2D))
def test_degenerate_2d_reduced_storages(name, precision, tol_pop, tol_f):
    from paper_2210_10377_amd import Sim
    mask, bx, by, u = CASES_2D[name]
    ny, nx = mask.shape
    uin = None if u is None else np.full(ny, u)
    S0 = _state2(nx, ny, precision, 90 + len(name))
    g = Sim(mask, 0.7, uin, precision=precision, bc_x=bx, bc_y=by, max_record=32)
    o = OracleSim(mask, tau=0.7, uin=uin, bc_x=bx, bc_y=by)
    g.set_populations(S0)
    o.set_state(S0)
    g.step(25)
    o.step(25)
    err = _close(g.populations(), o.state(), mask)
    Fg, Fo = g.forces(), o.forces()
    print(name, precision, "population error", err)
    assert err <= tol_pop
    if mask.any():
        assert _rel_force_err(Fg, Fo, (0, 1)) <= tol_f
    else:
        assert np.all(Fg[:, [0, 1, 3]] == 0.0)


@pytest.mark.parametrize("precision", [p for p, _, _ in REDUCED])
def test_no_fluid_node_reduced_storages(precision):
    """All solid: every storage leaves the stored values as they were, bit for bit."""
    from paper_2210_10377_amd import Sim, Sim3
    mask = np.ones((20, 40), np.uint8)
    g = Sim(mask, 0.7, np.full(20, 0.03), precision=precision, max_record=8)
    g.set_populations(_state2(40, 20, precision, 97))
    before = g.populations()
    g.step(4)
    np.testing.assert_array_equal(g.populations(), before)
    assert np.all(g.forces()[:, [0, 1, 3]] == 0.0)
    m3 = np.ones((6, 6, 6), np.uint8)
    h = Sim3(m3, 0.7, None, precision=precision, bc_x=1, bc_y=1, bc_z=1, max_record=8)
    dt = np.float64 if precision in ("fp32dev", "fp16dev") else np.float32
    h.set_populations(d3.near_rest_state3(6, 6, 6, seed=99, amp=0.05, dtype=dt))
    before = h.populations()
    h.step(4)
    np.testing.assert_array_equal(h.populations(), before)
    assert np.all(h.forces()[:, [0, 1, 3]] == 0.0)


@pytest.mark.parametrize("precision,tol_pop,tol_f", REDUCED)
@pytest.mark.parametrize("name", list(CASES_3D))
def test_degenerate_3d_reduced_storages(name, precision, tol_pop, tol_f):
    from paper_2210_10377_amd import Sim3
    mask, (bx, by, bz), u = CASES_3D[name]
    nz, ny, nx = mask.shape
    uin = None if u is None else np.full((nz, ny), u)
    # 3-D states: binary32 values for the f storages; for the deviation storages the
    # FP64 state (the oracle then starts from the unrounded values, within the bound).
    dt = np.float64 if precision in ("fp32dev", "fp16dev") else np.float32
    S0 = d3.near_rest_state3(nx, ny, nz, seed=95 + len(name), amp=0.05, dtype=dt)
    g = Sim3(mask, 0.7, uin, precision=precision, bc_x=bx, bc_y=by, bc_z=bz, max_record=32)
    o = D.OracleSim3(mask, tau=0.7, uin=uin, bc_x=bx, bc_y=by, bc_z=bz)
    g.set_populations(S0)
    o.set_state(S0)
    g.step(25)
    o.step(25)
    err = _close(g.populations(), o.state(), mask)
    Fg, Fo = g.forces(), o.forces()
    print(name, precision, "3-D population error", err)
    assert err <= tol_pop
    if mask.any():
        assert _rel_force_err(Fg, Fo, (0, 1)) <= tol_f
    else:
        assert np.all(Fg[:, [0, 1, 3]] == 0.0)
