"""Binary32 populations rounded stochastically (LBM_FP32SR) on the GPU, through the C ABI:
the rounding is unbiased against the FP64 step, the runs are reproducible bit for bit
(however the steps are split into calls, across a checkpoint and after a reset, in a
batch as alone).  Its accuracy against the oracle is held with the other
storages in test_gpu_parity.py and test_gpu_fixtures.py."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _sim(w, precision, max_record=64):
    from paper_2210_10377_amd import Sim
    return Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=max_record)


def _channel():
    """Cylinder channel with walls, inlet, outlet and a control volume (every strip class)."""
    nx, ny = 192, 64
    mask = workloads.cylinder_mask(nx, ny, 48, 31.5, 8)
    return workloads.Workload(name="sr_channel", nx=nx, ny=ny, mask=mask, tau=0.52,
                              uin=workloads.uniform_inlet(ny, 0.05),
                              box=workloads.default_box(mask, 4), steps=60, u_ref=0.05,
                              l_ref=16.0)


def test_stochastic_rounding_is_unbiased():
    """From one state (exactly representable in binary32), one step repeated M times with
    different step numbers.  Every stored value takes one of two adjacent binary32 values
    (the neighbours of the collision's binary32 result), and the mean over the repeats
    converges to the FP64 step: the per-value deviation of the mean is a Bernoulli
    average, at most 0.5 / sqrt(M) units in the last place (ulp) in standard deviation,
    plus the binary32 arithmetic of the collision on deviations of ~1e-2 w_i (a few 1e-2
    ulp; up to about one ulp at inlet nodes, whose random start is far from the inlet's
    equilibrium); rounding to nearest would leave a fixed error of 0.29 ulp RMS."""
    w = _channel()
    S0 = workloads.near_rest_state(w.nx, w.ny, seed=5, amp=0.01, dtype=np.float32)
    ref = _sim(w, "fp64")
    ref.set_populations(S0)
    ref.step(1, ())
    R = ref.populations()
    g = _sim(w, "fp32sr")
    fl = w.mask == 0
    M = 256
    acc = np.zeros_like(R)
    lo = np.full(R.shape, np.inf, np.float32)
    hi = np.full(R.shape, -np.inf, np.float32)
    for _ in range(M):
        g.set_populations(S0)
        g.step(1, ())
        P = g.populations().astype(np.float32)  # stored binary32 values, exactly
        lo = np.minimum(lo, P)
        hi = np.maximum(hi, P)
        acc += P
    ulp = np.spacing(np.abs(R).astype(np.float32)).astype(np.float64)
    steps_apart = (hi.view(np.int32).astype(np.int64) - lo.view(np.int32).astype(np.int64))[:, fl]
    worst = float((np.abs(acc / M - R) / ulp)[:, fl].max())
    bias = ((acc / M - R) / ulp)[:, fl]
    rms, mean = float(np.sqrt((bias ** 2).mean())), float(bias.mean())
    print(f"stochastic rounding over {M} repeats: values per element "
          f"{np.bincount(steps_apart.ravel() + 1)[1:]} (1 or 2 adjacent), bias of the mean: "
          f"RMS {rms:.4f} ulp, mean {mean:.5f} ulp, max {worst:.3f} ulp over {bias.size} values")
    assert steps_apart.min() >= 0 and steps_apart.max() <= 1
    assert rms <= 0.06
    assert abs(mean) <= 0.005


def test_stochastic_rounding_runs_are_reproducible():
    """Stores draw from the step number counted since create (or reset), so the same
    steps give the same bits: two handles, one call against several, a checkpoint
    restored into a fresh handle, and a reset followed by the same steps."""
    w = _channel()
    a = _sim(w, "fp32sr")
    a.step(60)
    Fa, Sa = a.forces(), a.populations()
    b = _sim(w, "fp32sr")
    b.step(17)
    F1 = b.forces()
    b.step(25)
    F2 = b.forces()
    blob = b.get_state()
    b.step(18)
    F3 = b.forces()
    assert np.array_equal(np.concatenate([F1, F2, F3]), Fa)
    assert np.array_equal(b.populations(), Sa)
    c = _sim(w, "fp32sr")
    c.set_state(blob)
    c.step(18)
    assert np.array_equal(c.forces(), F3)
    assert np.array_equal(c.populations(), Sa)
    c.reset()
    c.step(60)
    assert np.array_equal(c.forces(), Fa)
    # The draws differ from step to step: the same state stepped at two step numbers
    # stores different bits somewhere, and both stay within one ulp of each other.
    S0 = workloads.near_rest_state(w.nx, w.ny, seed=9, amp=0.01, dtype=np.float32)
    d = _sim(w, "fp32sr")
    d.set_populations(S0)
    d.step(1, ())
    P1 = d.populations()
    d.set_populations(S0)
    d.step(1, ())
    P2 = d.populations()
    fl = w.mask == 0
    assert not np.array_equal(P1[:, fl], P2[:, fl])
    gap = np.spacing(np.abs(P1).astype(np.float32)).astype(np.float64)
    assert float((np.abs(P1 - P2) / gap)[:, fl].max()) <= 2.0


@pytest.mark.parametrize("schedule", [
    dict(grid_blocks=0, graph_steps=0),
    dict(grid_blocks=0, graph_steps=4, tile_shape="narrow"),
    dict(grid_blocks=24, graph_steps=0, tile_queue=1)])
def test_stochastic_rounding_batch_bitwise_equals_singles(schedule):
    """Batched members draw with their own step numbers (members stepped alone before the
    batch included): every instance bitwise equals the member stepped alone with the same
    calls, with and without forces, under direct launches, graphs and the tile queue."""
    from paper_2210_10377_amd import Batch
    ws = workloads.batched_instances(5)
    pre = [0, 3, 1, 7, 2]

    def members():
        sims = [Sim_(w) for w in ws]
        for s, w, k in zip(sims, ws, pre):
            s.set_populations(workloads.near_rest_state(w.nx, w.ny, 40 + k, amp=0.02,
                                                        dtype=np.float32))
            if k:
                s.step(k, schemes=())
        return sims

    sims = members()
    b = Batch(sims, max_record=64)
    b.set_schedule(**schedule)
    b.step(9, schemes=())
    b.step(11)
    Fb, bad = b.forces()
    assert not bad.any()
    for i, r in enumerate(members()):
        r.step(9, schemes=())
        r.step(11)
        assert np.array_equal(r.forces(), Fb[i], equal_nan=True)
        assert np.array_equal(r.populations(), sims[i].populations())


def Sim_(w):
    from paper_2210_10377_amd import Sim
    return Sim(w.mask, w.tau, w.uin, precision="fp32sr", box=w.box, max_record=64)


def test_stochastic_rounding_is_independent_of_tile_shape_and_layout():
    """The draws are keyed on the node index, not on a buffer offset or a thread: wide
    (256 x 1) and narrow (64 x 4) tiles and the two state layouts store the same bits."""
    from paper_2210_10377_amd import Sim
    w = _channel()
    S0 = workloads.near_rest_state(w.nx, w.ny, seed=21, amp=0.03, dtype=np.float32)
    runs = []
    for tile, layout in (("wide", "rows"), ("narrow", "rows"), ("wide", "planes")):
        g = Sim(w.mask, w.tau, w.uin, precision="fp32sr", box=w.box, max_record=64, tile=tile,
                layout=layout)
        g.set_populations(S0)
        g.step(40)
        runs.append((g.populations(), g.forces()))
    F0 = runs[0][1]
    for P, F in runs[1:]:
        assert np.array_equal(P, runs[0][0])
        # forces: the same stored values, partials numbered in strip order for every
        # tile shape and layout
        assert np.array_equal(F, F0, equal_nan=True)


def test_stochastic_rounding_3d_is_reproducible_and_unbiased():
    """D3Q27: the same draws for the same step numbers (one call against several, a
    checkpoint restored into a fresh handle, a reset), and one step repeated 64 times
    from one state with different step numbers stores, per value, one of two adjacent
    binary32 values whose mean approaches the FP64 step (RMS bias under 0.12 ulp, where
    rounding to nearest leaves 0.29)."""
    import workloads.d3 as d3
    from paper_2210_10377_amd import Sim3
    w = d3.sphere_channel_64x32x32()

    def sim(prec):
        return Sim3(w.mask, w.tau, w.uin, precision=prec, box=w.box, max_record=64)

    a = sim("fp32sr")
    a.step(40)
    Fa, Sa = a.forces(), a.populations()
    b = sim("fp32sr")
    b.step(13)
    F1 = b.forces()
    blob = b.get_state()
    b.step(27)
    F2 = b.forces()
    assert np.array_equal(np.concatenate([F1, F2]), Fa, equal_nan=True)
    assert np.array_equal(b.populations(), Sa)
    c = sim("fp32sr")
    c.set_state(blob)
    c.step(27)
    assert np.array_equal(c.forces(), F2, equal_nan=True)
    c.reset()
    c.step(40)
    assert np.array_equal(c.populations(), Sa)

    S0 = d3.near_rest_state3(w.nx, w.ny, w.nz, seed=3, amp=0.01, dtype=np.float32)
    ref = sim("fp64")
    ref.set_populations(S0)
    ref.step(1, ())
    R = ref.populations()
    g = sim("fp32sr")
    fl = w.mask == 0
    M = 64
    acc = np.zeros_like(R)
    lo = np.full(R.shape, np.inf, np.float32)
    hi = np.full(R.shape, -np.inf, np.float32)
    for _ in range(M):
        g.set_populations(S0)
        g.step(1, ())
        P = g.populations().astype(np.float32)
        lo = np.minimum(lo, P)
        hi = np.maximum(hi, P)
        acc += P
    apart = (hi.view(np.int32).astype(np.int64) - lo.view(np.int32).astype(np.int64))[:, fl]
    ulp = np.spacing(np.abs(R).astype(np.float32)).astype(np.float64)
    bias = ((acc / M - R) / ulp)[:, fl]
    rms, mean = float(np.sqrt((bias ** 2).mean())), float(bias.mean())
    print(f"3-D stochastic rounding over {M} repeats: bias of the mean RMS {rms:.4f} ulp, "
          f"mean {mean:.5f} ulp over {bias.size} values")
    assert apart.min() >= 0 and apart.max() <= 1
    assert rms <= 0.12
    assert abs(mean) <= 0.01

