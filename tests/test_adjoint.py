"""Adjoint (reverse-mode) gradients of the time-averaged body force.

Reference values: directional derivatives by complex step through the FP64 oracle
(miniature channels), and FP64 central differences of the GPU FP64 path (the NACA0012
1024x512 channel of the adjoint workload, 10 000 steps, checkpoint every 500).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _sim(mask, tau, uin, precision, box=None, bc_x=0, bc_y=0):
    from paper_2210_10377_amd import Sim
    return Sim(mask, tau, uin, precision=precision, box=box, bc_x=bc_x, bc_y=bc_y,
               max_record=8)


MINI = [
    # nx, ny, body, bc_y, n, every, t0, T, w
    ("cylinder_walls", 96, 48, lambda: workloads.cylinder_mask(96, 48, 24, 23.5, 4), 0, 300, 40, 200, 100, (1.0, 0.0)),
    ("cylinder_periodic_y_lift", 80, 40, lambda: workloads.cylinder_mask(80, 40, 20, 17.0, 4), 1, 240, 60, 150, 90, (0.3, 1.0)),
    ("naca_walls", 160, 64, lambda: workloads.naca0012_mask(160, 64, 48, 52, 32, 6.0), 0, 200, 200, 100, 100, (1.0, 0.5)),
]


@pytest.fixture(scope="module")
def mini_refs(orc):
    out = {}
    for name, nx, ny, mk, bcy, n, every, t0, T, w in MINI:
        mask = mk()
        y = np.arange(ny)
        uin = 0.03 + 0.02 * np.sin(np.pi * (y + 0.5) / ny)
        tau = 0.75
        h = 1e-30
        v = np.random.default_rng(len(name)).normal(size=ny)
        J = orc.objective(mask, 1 / tau, uin, n, t0, T, w=w, bc_y=bcy)
        d_tau = orc.objective(mask, 1 / complex(tau, h), uin, n, t0, T, w=w, bc_y=bcy).imag / h
        d_v = orc.objective(mask, 1 / tau, uin + 1j * h * v, n, t0, T, w=w, bc_y=bcy).imag / h
        # every inlet row individually on the first few rows (full gradient spot check)
        rows = [0, 1, ny // 2, ny - 1]
        d_rows = []
        for r in rows:
            e = np.zeros(ny)
            e[r] = 1.0
            d_rows.append(orc.objective(mask, 1 / tau, uin + 1j * h * e, n, t0, T, w=w,
                                        bc_y=bcy).imag / h)
        out[name] = dict(mask=mask, uin=uin, tau=tau, v=v, J=J.real, d_tau=d_tau, d_v=d_v,
                         rows=rows, d_rows=np.array(d_rows), cfg=(n, every, t0, T, w, bcy))
    return out


@pytest.mark.parametrize("name", [m[0] for m in MINI])
# Measured: FP64 ~1e-14; FP32 deviations up to 1.2e-6; FP32 up to 6.6e-6 (tau of the
# airfoil channel).  The bounds keep about an order of magnitude of margin.
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32dev", 1e-5), ("fp32", 5e-5),
                                           ("fp32sr", 1e-5)])
def test_adjoint_matches_complex_step(mini_refs, name, precision, tol):
    r = mini_refs[name]
    n, every, t0, T, w, bcy = r["cfg"]
    g = _sim(r["mask"], r["tau"], r["uin"], precision, bc_y=bcy)
    J = g.adjoint_forward(n, every, t0, T, w)
    gu, gt = g.adjoint_backward(1.0)
    scale_j = max(abs(r["J"]), 1e-12)
    assert abs(J - r["J"]) <= (1e-12 if precision == "fp64" else 1e-4) * scale_j
    e_tau = abs(gt - r["d_tau"]) / abs(r["d_tau"])
    e_v = abs(gu @ r["v"] - r["d_v"]) / abs(r["d_v"])
    e_rows = np.abs(gu[r["rows"]] - r["d_rows"]).max() / np.abs(gu).max()
    print(name, precision, "rel errors tau", e_tau, "direction", e_v, "rows", e_rows)
    assert e_tau <= tol and e_v <= tol and e_rows <= tol


def test_adjoint_seed_scales_and_is_deterministic(mini_refs):
    r = mini_refs["cylinder_walls"]
    n, every, t0, T, w, bcy = r["cfg"]
    g = _sim(r["mask"], r["tau"], r["uin"], "fp32")
    g.adjoint_forward(n, every, t0, T, w)
    a_u, a_t = g.adjoint_backward(1.0)
    b_u, b_t = g.adjoint_backward(1.0)
    c_u, c_t = g.adjoint_backward(-2.5)
    assert np.array_equal(a_u, b_u) and a_t == b_t
    np.testing.assert_allclose(c_u, -2.5 * a_u, rtol=1e-6, atol=1e-12)
    assert abs(c_t + 2.5 * a_t) <= 1e-6 * abs(a_t)


def test_adjoint_checkpoint_interval_does_not_change_gradient(mini_refs):
    r = mini_refs["cylinder_walls"]
    n, every, t0, T, w, bcy = r["cfg"]
    out = []
    for k in (1, 7, n):
        g = _sim(r["mask"], r["tau"], r["uin"], "fp64")
        g.adjoint_forward(n, k, t0, T, w)
        out.append(g.adjoint_backward(1.0))
    for gu, gt in out[1:]:
        np.testing.assert_allclose(gu, out[0][0], rtol=1e-12, atol=1e-16)
        assert abs(gt - out[0][1]) <= 1e-12 * abs(out[0][1])


def test_adjoint_stochastic_rounding_recomputes_the_forward_states(mini_refs):
    """Binary32 populations rounded stochastically: the segment recomputation replays
    each step with the forward run's step number, so the reverse sweep reads bitwise the
    states the forward stored, whatever the checkpoint interval: the gradients of
    intervals 1, 7 and n agree to FP64 summation rounding (a recomputation with other
    draws would move them by the binary32 rounding, ~1e-6), and the objective equals the
    plain run's."""
    r = mini_refs["cylinder_walls"]
    n, every, t0, T, w, bcy = r["cfg"]
    out = []
    for k in (1, 7, n):
        g = _sim(r["mask"], r["tau"], r["uin"], "fp32sr")
        J = g.adjoint_forward(n, k, t0, T, w)
        out.append((J, g.adjoint_backward(1.0)))
    for J, (gu, gt) in out[1:]:
        assert J == out[0][0]
        np.testing.assert_allclose(gu, out[0][1][0], rtol=1e-12, atol=1e-12 * np.abs(gu).max())
        assert abs(gt - out[0][1][1]) <= 1e-12 * abs(out[0][1][1])


def test_adjoint_backward_needs_valid_forward(mini_refs):
    from paper_2210_10377_amd import LbmError
    r = mini_refs["cylinder_walls"]
    g = _sim(r["mask"], r["tau"], r["uin"], "fp32")
    with pytest.raises(LbmError):
        g.adjoint_backward(1.0)
    g.adjoint_forward(20, 5, 10, 10)
    g.set_tau(0.9)
    with pytest.raises(LbmError):
        g.adjoint_backward(1.0)


def test_autograd_function(mini_refs):
    import torch

    from paper_2210_10377_amd.autograd import ObjectiveSpec, objective
    r = mini_refs["cylinder_walls"]
    n, every, t0, T, w, bcy = r["cfg"]
    g = _sim(r["mask"], r["tau"], r["uin"], "fp64")
    u = torch.tensor(r["uin"], dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(r["tau"], dtype=torch.float64, requires_grad=True)
    J = objective(u, tau, g, ObjectiveSpec(n, every, t0, T, w))
    J.backward()
    assert abs(J.item() - r["J"]) <= 1e-12 * abs(r["J"])
    assert abs(tau.grad.item() - r["d_tau"]) <= 1e-9 * abs(r["d_tau"])
    assert abs(u.grad.numpy() @ r["v"] - r["d_v"]) <= 1e-9 * abs(r["d_v"])


def test_adjoint_naca_1024x512_against_fp64_central_differences():
    """The adjoint workload: NACA0012 chord 256 in a 1024x512 channel, Re 500, 10 000
    steps from rest, J = mean drag (algorithm B) over the last 2000 steps, checkpoint
    every 500.  FP32-deviation adjoint against FP64 central differences of the FP64 GPU
    path in two random inlet directions and in tau."""
    w = workloads.naca_1024x512_adjoint()
    n, every, t0, T = 10000, 500, 8000, 2000
    g = _sim(w.mask, w.tau, w.uin, "fp32dev", box=w.box)
    J32 = g.adjoint_forward(n, every, t0, T)
    gu, gt = g.adjoint_backward(1.0)
    from paper_2210_10377_amd import Sim
    ref = Sim(w.mask, w.tau, w.uin, precision="fp64", box=w.box, max_record=T)

    def J64(uin, tau):
        ref.set_inlet(uin)
        ref.set_tau(tau)
        ref.reset()
        ref.step(t0, schemes=())
        ref.step(T, schemes=("B",))
        return ref.forces()[:, 1, 0].mean()

    J0 = J64(w.uin, w.tau)
    assert abs(J32 - J0) <= 1e-4 * abs(J0)
    e = 1e-6 * w.tau
    d_tau = (J64(w.uin, w.tau + e) - J64(w.uin, w.tau - e)) / (2 * e)
    errs = [abs(gt - d_tau) / abs(d_tau)]
    rng = np.random.default_rng(500)
    for _ in range(2):
        v = rng.normal(size=w.ny)
        v /= np.linalg.norm(v)
        h = 1e-7
        d_v = (J64(w.uin + h * v, w.tau) - J64(w.uin - h * v, w.tau)) / (2 * h)
        errs.append(abs(gu @ v - d_v) / abs(d_v))
    print("naca 1024x512 adjoint rel errors (tau, v1, v2):", errs, "J", J0, "dJ/dtau", d_tau)
    assert max(errs) <= 1e-4, errs


def test_adjoint_same_in_both_layouts(mini_refs):
    """The adjoint runs the same arithmetic in the row-interleaved and planar layouts:
    objective and gradients bitwise equal (FP32 deviations)."""
    from paper_2210_10377_amd import Sim
    r = mini_refs["naca_walls"]
    n, every, t0, T, w, bcy = r["cfg"]
    out = []
    for layout in ("rows", "planes"):
        g = Sim(r["mask"], r["tau"], r["uin"], precision="fp32dev", bc_y=bcy, max_record=8,
                layout=layout)
        J = g.adjoint_forward(n, every, t0, T, w)
        gu, gt = g.adjoint_backward(1.0)
        out.append((J, gu, gt))
    assert out[0][0] == out[1][0]
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_adjoint_whole_tile_rounds_and_tail(orc):
    """A 512x130 cylinder channel: 2 tiles per row, 260 tiles.  The reverse kernel hands
    tiles to the XCDs in runs (32 tiles at 4-byte adjoint values, 16 at 8-byte), over
    whole rounds of 8 runs, and the last 4 tiles (the tail) keep the identity mapping; the
    objective and gradients must not depend on which block takes which tile.  FP64 and
    FP32-deviation adjoints against complex-step derivatives through the oracle."""
    nx, ny = 512, 130
    mask = workloads.cylinder_mask(nx, ny, 120, 64.5, 13)
    y = np.arange(ny)
    uin = 0.03 + 0.02 * np.sin(np.pi * (y + 0.5) / ny)
    tau, n, every, t0, T, w = 0.75, 400, 100, 200, 200, (1.0, 0.3)
    h = 1e-30
    v = np.random.default_rng(130).normal(size=ny)
    J_ref = orc.objective(mask, 1 / tau, uin, n, t0, T, w=w).real
    d_tau = orc.objective(mask, 1 / complex(tau, h), uin, n, t0, T, w=w).imag / h
    d_v = orc.objective(mask, 1 / tau, uin + 1j * h * v, n, t0, T, w=w).imag / h
    # measured: FP64 ~2e-14, FP32 deviations ~8e-7
    for precision, tol in (("fp64", 1e-9), ("fp32dev", 1e-5)):
        g = _sim(mask, tau, uin, precision)
        J = g.adjoint_forward(n, every, t0, T, w)
        gu, gt = g.adjoint_backward(1.0)
        e_tau = abs(gt - d_tau) / abs(d_tau)
        e_v = abs(gu @ v - d_v) / abs(d_v)
        print("512x130", precision, "J", J, J_ref, "rel errors tau", e_tau, "direction", e_v)
        assert abs(J - J_ref) <= (1e-12 if precision == "fp64" else 1e-4) * abs(J_ref)
        assert e_tau <= tol and e_v <= tol


def test_adjoint_follows_a_mask_change():
    """After lbm_set_mask the adjoint differentiates the new geometry: a handle that ran
    an adjoint on one cylinder, then had its body moved and its state reset, gives
    bitwise the objective and gradients of a fresh handle created with the moved body."""
    nx, ny = 160, 64
    m0 = workloads.cylinder_mask(nx, ny, 40, 31.5, 6)
    m1 = workloads.cylinder_mask(nx, ny, 52, 33.5, 7)
    y = np.arange(ny)
    uin = 0.03 + 0.01 * np.cos(np.pi * (y + 0.5) / ny)
    tau, n, every, t0, T, w = 0.7, 160, 40, 80, 80, (1.0, 0.4)
    for precision in ("fp64", "fp32dev"):
        g = _sim(m0, tau, uin, precision)
        g.adjoint_forward(n, every, t0, T, w)
        g.adjoint_backward(1.0)
        g.set_mask(m1)
        g.reset()
        J = g.adjoint_forward(n, every, t0, T, w)
        gu, gt = g.adjoint_backward(1.0)
        f = _sim(m1, tau, uin, precision)
        Jf = f.adjoint_forward(n, every, t0, T, w)
        fu, ft = f.adjoint_backward(1.0)
        assert J == Jf, precision
        np.testing.assert_array_equal(gu, fu)
        assert gt == ft


def test_autograd_two_objectives_on_one_sim(mini_refs):
    """Two objectives evaluated on one lattice before a single backward (the second
    forward replaces the first's checkpoints on the handle): each gets the gradient of
    its own run, as separate lattices give it."""
    import torch

    from paper_2210_10377_amd.autograd import ObjectiveSpec, objective
    r = mini_refs["cylinder_walls"]
    n, every, t0, T, w, bcy = r["cfg"]
    s1 = ObjectiveSpec(n, every, t0, T, (1.0, 0.0))
    s2 = ObjectiveSpec(n, every, t0 + 20, T - 20, (0.0, 1.0))
    u2 = r["uin"] * 1.1
    g = _sim(r["mask"], r["tau"], r["uin"], "fp64")
    ua = torch.tensor(r["uin"], dtype=torch.float64, requires_grad=True)
    ub = torch.tensor(u2, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(r["tau"], dtype=torch.float64, requires_grad=True)
    J1 = objective(ua, tau, g, s1)
    J2 = objective(ub, tau, g, s2)
    (J1 + 2.0 * J2).backward()
    refs = []
    for u, s in ((r["uin"], s1), (u2, s2)):
        h = _sim(r["mask"], r["tau"], u, "fp64")
        Jr = h.adjoint_forward(s.n_steps, s.every, s.t0, s.T, s.w)
        refs.append((Jr,) + h.adjoint_backward(1.0))
    assert J1.item() == refs[0][0] and J2.item() == refs[1][0]
    np.testing.assert_allclose(ua.grad.numpy(), refs[0][1], rtol=1e-14, atol=0)
    np.testing.assert_allclose(ub.grad.numpy(), 2.0 * refs[1][1], rtol=1e-14, atol=0)
    assert abs(tau.grad.item() - (refs[0][2] + 2.0 * refs[1][2])) <= 1e-13 * abs(tau.grad.item())
    # A step between forward and backward invalidates the handle's run; backward
    # recomputes it.
    J3 = objective(ua, tau, g, s1)
    g.step(3, schemes=())
    ua.grad = None
    J3.backward()
    np.testing.assert_allclose(ua.grad.numpy(), refs[0][1], rtol=1e-14, atol=0)


def test_adjoint_on_a_grid_above_the_overlap_threshold():
    """Grids of more than 16,384 tiles keep one segment store and recompute each segment
    on the caller's stream before its reverse sweep (no overlap): an 8192 x 514 channel
    (32 x 514 = 16,448 wide tiles) with a cylinder gives the same gradient with a
    checkpoint every 10 steps (three segments through the one store) as with a single
    segment."""
    nx, ny = 8192, 514
    # the body 18 nodes from the inlet, so the inlet reaches the forces of the window
    mask = workloads.cylinder_mask(nx, ny, 30, 256.5, 12)
    uin = np.full(ny, 0.05)
    n, t0, T = 30, 10, 20
    out = []
    for every in (10, n):
        g = _sim(mask, 0.6, uin, "fp64")
        assert g.info().n_tiles > 16384
        J = g.adjoint_forward(n, every, t0, T, (1.0, 0.0))
        out.append((J,) + tuple(g.adjoint_backward(1.0)))
        del g
    (J0, gu0, gt0), (J1, gu1, gt1) = out
    assert J0 == J1
    assert np.abs(gu0).max() > 0 and gt0 != 0
    np.testing.assert_allclose(gu0, gu1, rtol=1e-12, atol=1e-16)
    assert abs(gt0 - gt1) <= 1e-12 * abs(gt1)


def test_adjoint_full_inlet_gradient_128x64(orc):
    """The whole gradient of a 128 x 64 miniature (cylinder between walls, 1000 steps,
    mean drag over the last 200, checkpoint every 100): all 64 inlet rows and tau by
    complex-step differentiation through the oracle, one oracle run per component,
    against the GPU adjoint in FP64 (1e-9 of the largest component) and in the 32-bit
    storages (1e-5 / 5e-5, the mini-channel bounds)."""
    import os

    import oracle
    nx, ny = 128, 64
    mask = workloads.cylinder_mask(nx, ny, 32, 31.5, 6)
    y = np.arange(ny)
    uin = 0.03 + 0.02 * np.sin(np.pi * (y + 0.5) / ny)
    tau, n, every, t0, T, w = 0.7, 1000, 100, 800, 200, (1.0, 0.0)
    h = 1e-30
    prev = oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        ref_u = np.empty(ny)
        for r in range(ny):
            e = np.zeros(ny)
            e[r] = 1.0
            ref_u[r] = orc.objective(mask, 1 / tau, uin + 1j * h * e, n, t0, T, w=w).imag / h
        ref_t = orc.objective(mask, 1 / complex(tau, h), uin, n, t0, T, w=w).imag / h
    finally:
        oracle.set_threads(prev)
    scale = np.abs(ref_u).max()
    assert scale > 0 and ref_t != 0
    for precision, tol in (("fp64", 1e-9), ("fp32dev", 1e-5), ("fp32", 5e-5)):
        g = _sim(mask, tau, uin, precision)
        g.adjoint_forward(n, every, t0, T, w)
        gu, gt = g.adjoint_backward(1.0)
        e_u = np.abs(gu - ref_u).max() / scale
        e_t = abs(gt - ref_t) / abs(ref_t)
        print("128x64 full gradient", precision, "rel errors rows", e_u, "tau", e_t)
        assert e_u <= tol and e_t <= tol, precision
