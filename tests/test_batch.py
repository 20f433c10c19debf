"""Batched stepping: every instance of a batch equals the same instance stepped alone.

The batch runs the single-lattice tile code of every instance inside one launch per
step, so the populations and all three forces of each instance must be bitwise those of
``Sim.step`` with the same call lengths, whatever the schedule (one workgroup per tile or
a persistent grid, direct launches or graph replays, any tile order).  The single path is
itself held to the oracle (test_gpu_parity.py); an FP64 mini batch is also compared with
the oracle directly.
"""
import numpy as np
import pytest

import workloads
from oracle import OracleSim

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _members(ws, precision="fp32"):
    from paper_2210_10377_amd import Sim
    return [Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=512,
                u_ref=w.u_ref, l_ref=w.l_ref) for w in ws]


def _batch(ws, precision="fp32", max_record=512):
    from paper_2210_10377_amd import Batch
    return Batch(_members(ws, precision), max_record=max_record)


def _seed_states(sims, ws, seed0=100):
    for i, (s, w) in enumerate(zip(sims, ws)):
        S = workloads.near_rest_state(w.nx, w.ny, seed0 + i, amp=0.02, dtype=np.float32)
        s.set_populations(S)


def _singles(ws, calls, precision="fp32", seed0=100):
    """Each instance stepped alone with the given call lengths; (populations, forces)."""
    sims = _members(ws, precision)
    _seed_states(sims, ws, seed0)
    pops, forces = [], []
    for s in sims:
        F = []
        for n in calls:
            s.step(n)
            F.append(s.forces())
        pops.append(s.populations())
        forces.append(np.concatenate(F))
    return pops, forces


def _batched(ws, calls, precision="fp32", schedule=None, seed0=100):
    b = _batch(ws, precision)
    _seed_states(b.members, ws, seed0)
    if schedule:
        b.set_schedule(**schedule)
    F = []
    for n in calls:
        b.step(n)
        Fi, bad = b.forces()
        assert not bad.any()
        F.append(Fi)
    return [m.populations() for m in b.members], np.concatenate(F, axis=1), b


def _assert_same(pa, fa, pb, fb):
    for i in range(len(pa)):
        np.testing.assert_array_equal(pa[i], pb[i], err_msg=f"populations of instance {i}")
        np.testing.assert_array_equal(fa[i], fb[i], err_msg=f"forces of instance {i}")


MINI = workloads.batched_instances(8)
CALLS = (37, 6, 1)

SCHEDULES = {
    "one_block_per_tile": dict(grid_blocks=0, graph_steps=0),
    "persistent_small_grid": dict(grid_blocks=24, graph_steps=0),
    "graph_chunks": dict(grid_blocks=0, graph_steps=8),
    "persistent_graph_shuffled": dict(grid_blocks=40, graph_steps=4, tile_order=12345),
    "tile_queue": dict(grid_blocks=24, graph_steps=0, tile_queue=1),
    "tile_queue_graph_shuffled": dict(grid_blocks=40, graph_steps=4, tile_order=777, tile_queue=1),
    # every instance in one tile shape in the batch (the members keep their own)
    "all_wide_tiles": dict(grid_blocks=0, graph_steps=0, tile_shape="wide"),
    "all_narrow_tiles_graph_shuffled": dict(grid_blocks=0, graph_steps=4, tile_order=99,
                                            tile_shape="narrow"),
    "narrow_tiles_tile_queue": dict(grid_blocks=24, graph_steps=0, tile_queue=1,
                                    tile_shape="narrow"),
}


@pytest.fixture(scope="module")
def mini_singles():
    return _singles(MINI, CALLS)


@pytest.mark.parametrize("name", list(SCHEDULES))
def test_mini_batch_bitwise_equals_singles(name, mini_singles):
    pb, fb, b = _batched(MINI, CALLS, schedule=SCHEDULES[name])
    ps, fs = mini_singles
    _assert_same(ps, [f for f in fs], pb, [fb[i] for i in range(len(MINI))])
    inf = b.info()
    assert inf.steps_done == sum(CALLS)
    for m in b.members:
        assert m.info().steps_done == sum(CALLS)


def test_fp64_mini_batch_against_oracle():
    ws = workloads.batched_instances(4)
    b = _batch(ws, "fp64")
    _seed_states(b.members, ws)
    n = 40
    b.step(n)
    F, bad = b.forces()
    assert not bad.any()
    for i, w in enumerate(ws):
        o = OracleSim(w.mask, w.tau, w.uin, box=w.box)
        o.set_state(workloads.near_rest_state(w.nx, w.ny, 100 + i, amp=0.02, dtype=np.float32))
        o.step(n)
        Fo = o.forces()
        So = o.state()
        Sg = b.members[i].populations()
        fl = w.mask == 0
        assert (np.abs(Sg - So)[:, fl] / np.abs(So)[:, fl]).max() <= TOL64
        for k in range(3):
            scale = np.abs(Fo[:, k]).max()
            assert np.abs(F[i, :, k] - Fo[:, k]).max() / scale <= TOL64, (i, k)


def test_members_changed_between_batch_calls():
    """A member stepped alone, or given a new tau, between batch calls is picked up."""
    ws = MINI[:4]
    b = _batch(ws)
    _seed_states(b.members, ws)
    b.set_schedule(grid_blocks=0, graph_steps=4)
    ref = _members(ws)
    _seed_states(ref, ws)
    b.step(5)
    b.forces()
    for r in ref:
        r.step(5)
        r.forces()
    # instance 1 takes 3 steps alone (its buffers swap parity against the others)
    b.members[1].step(3)
    b.members[1].forces()
    ref[1].step(3)
    ref[1].forces()
    # instance 2 gets a new relaxation time
    b.members[2].set_tau(0.61)
    ref[2].set_tau(0.61)
    b.step(9)
    Fb, _ = b.forces()
    for i, r in enumerate(ref):
        r.step(9)
        np.testing.assert_array_equal(r.forces(), Fb[i])
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())


def test_steps_without_forces_and_ring_overflow():
    from paper_2210_10377_amd import LbmError
    ws = MINI[:3]
    b = _batch(ws, max_record=10)
    _seed_states(b.members, ws)
    ref = _members(ws)
    _seed_states(ref, ws)
    b.set_schedule(grid_blocks=16, graph_steps=6)
    b.step(13, schemes=())
    for r in ref:
        r.step(13, schemes=())
    for i, r in enumerate(ref):
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())
    b.step(10)
    with pytest.raises(LbmError):
        b.step(1)
    F, _ = b.forces()
    assert F.shape == (3, 10, 5, 2)


def test_nonfinite_instance_is_flagged_alone():
    from paper_2210_10377_amd import Sim, Batch
    ws = MINI[:3]
    sims = _members(ws)
    _seed_states(sims, ws)
    # instance 1 starts from a field with a NaN population on a link node
    S = sims[1].populations()
    ys, xs = np.nonzero(ws[1].mask)
    S[1, ys[0], xs[0] - 1] = np.nan
    sims[1].set_populations(S)
    b = Batch(sims, max_record=64)
    b.step(20)
    F, bad = b.forces()
    assert bad.tolist() == [False, True, False]
    assert np.isfinite(F[0]).all() and np.isfinite(F[2]).all()


def test_autotune_keeps_results_bitwise():
    ws = MINI
    b = _batch(ws)
    _seed_states(b.members, ws)
    sched, ms = b.autotune(steps=4)
    assert ms > 0
    assert sched["graph_steps"] in (0, 4)
    assert sched["tile_queue"] in (0, 1) and (sched["grid_blocks"] > 0 or not sched["tile_queue"])
    assert sched["tile_shape"] in ("auto", "wide", "narrow")
    # one block per tile: 2 candidates; 4 persistent grids x (stride, queue) x 2: 16; the
    # fastest with the two other tile shapes: 2
    n_tune = (2 + 16 + 2) * 2 * 4
    assert b.info().steps_done == n_tune
    b.step(7)
    Fb, _ = b.forces()
    ref = _members(ws)
    _seed_states(ref, ws)
    for i, r in enumerate(ref):
        r.step(n_tune, schemes=())
        r.step(7)
        np.testing.assert_array_equal(r.forces(), Fb[i])
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())


def test_full_256_instance_batch_bitwise_equals_singles():
    ws = workloads.batched_instances()
    calls = (10,)
    pb, fb, b = _batched(ws, calls, schedule=dict(grid_blocks=2048, graph_steps=4))
    ps, fs = _singles(ws, calls)
    _assert_same(ps, fs, pb, [fb[i] for i in range(len(ws))])


@pytest.mark.parametrize("precision", ["fp32dev", "fp32sr"])
@pytest.mark.parametrize("collision", ["regularized", "kbc"])
def test_stabilized_collision_batch_bitwise_equals_singles(collision, precision):
    """A batch whose instances all use the regularized or the KBC collision (binary32
    deviations, or binary32 rounded stochastically)."""
    ws = MINI
    from paper_2210_10377_amd import Sim, Batch
    def members():
        return [Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=64,
                    collision=collision) for w in ws]
    sims = members()
    _seed_states(sims, ws)
    b = Batch(sims, max_record=64)
    b.set_schedule(grid_blocks=0, graph_steps=4)
    b.step(21)
    Fb, bad = b.forces()
    assert not bad.any()
    ref = members()
    _seed_states(ref, ws)
    for i, r in enumerate(ref):
        r.step(21)
        np.testing.assert_array_equal(r.forces(), Fb[i])
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())


def test_mixed_collision_batch_is_rejected():
    from paper_2210_10377_amd import Sim, Batch, LbmError
    ws = MINI[:2]
    sims = [Sim(w.mask, w.tau, w.uin, precision="fp32", box=w.box, max_record=4,
                collision=c) for w, c in zip(ws, ("bgk", "kbc"))]
    with pytest.raises(LbmError):
        Batch(sims)


@pytest.mark.parametrize("precision", ["fp32", "fp32sr"])
def test_moving_members_batch_bitwise_equals_singles(precision):
    """A batch whose members mix bodies at rest and in rigid motion, with graph replays
    cached before one member starts moving: every instance bitwise equals the same
    member stepped alone with the same motions (binary32 rounded to nearest or
    stochastically)."""
    ws = MINI[:4]
    from paper_2210_10377_amd import Sim, Batch

    def members():
        return [Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=64)
                for w in ws]

    def motion(i, phase):
        w = ws[i]
        yc, xc = (np.argwhere(w.mask).mean(axis=0) if w.mask.any() else (0.0, 0.0))
        if i == 1:
            return (0.0, 0.0, 0.002, xc, yc)
        if i == 3 and phase == 1:
            return (0.005, -0.004, -0.001, xc, yc)
        return None

    sims = members()
    _seed_states(sims, ws)
    for i, s in enumerate(sims):
        if motion(i, 0):
            s.set_body_motion(*motion(i, 0))
    b = Batch(sims, max_record=64)
    b.set_schedule(grid_blocks=0, graph_steps=4)
    b.step(9)
    for i, s in enumerate(sims):
        if motion(i, 1):
            s.set_body_motion(*motion(i, 1))
    b.step(9)
    Fb, bad = b.forces()
    assert not bad.any()
    ref = members()
    _seed_states(ref, ws)
    for i, r in enumerate(ref):
        for phase in (0, 1):
            if motion(i, phase):
                r.set_body_motion(*motion(i, phase))
            r.step(9)
        np.testing.assert_array_equal(r.forces(), Fb[i])
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())


@pytest.mark.parametrize("precision", ["fp32", "fp32sr"])
@pytest.mark.parametrize("tile_shape", ["auto", "wide", "narrow"])
def test_member_moving_through_the_grid_batch_bitwise_equals_singles(tile_shape, precision):
    """A member whose body moves one node (and its control volume with it) between two
    batch calls: every instance bitwise equals the same member stepped alone with the
    same calls, also when the batch runs the instances in a tile shape of its own (its
    strip-slot tables follow the member's new plan); a member whose control volume
    changes size stops the batch."""
    from paper_2210_10377_amd import Sim, Batch, LbmError
    ws = MINI[:3]
    k = next(i for i, w in enumerate(ws) if w.box is not None)
    w = ws[k]
    shifted = np.roll(w.mask, 1, axis=1)
    x0, x1, y0, y1 = w.box
    box1 = (x0 + 1, x1 + 1, y0, y1)

    def members():
        return [Sim(v.mask, v.tau, v.uin, precision=precision, box=v.box, max_record=64)
                for v in ws]

    sims = members()
    _seed_states(sims, ws)
    b = Batch(sims, max_record=64)
    b.set_schedule(grid_blocks=0, graph_steps=4, tile_shape=tile_shape)
    b.step(10)
    imp_b = sims[k].set_mask(shifted, box1)
    b.step(10)
    Fb, bad = b.forces()
    assert not bad.any()
    ref = members()
    _seed_states(ref, ws)
    for i, r in enumerate(ref):
        r.step(10)
        if i == k:
            np.testing.assert_array_equal(r.set_mask(shifted, box1), imp_b)
        r.step(10)
        np.testing.assert_array_equal(r.forces(), Fb[i])
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())
    sims[k].set_mask(shifted, (x0 + 1, x1 + 1, y0, y1 - 1))   # one row fewer
    with pytest.raises(LbmError, match="changed size"):
        b.step(1)


def test_batch_mixing_state_layouts_bitwise_equals_singles():
    """Members in the row-interleaved and the planar layout, alternating, in one batch:
    every member bitwise equal to the same member stepped alone."""
    ws = MINI
    from paper_2210_10377_amd import Sim, Batch
    def members():
        return [Sim(w.mask, w.tau, w.uin, precision="fp32", box=w.box, max_record=64,
                    layout=("rows", "planes")[i % 2]) for i, w in enumerate(ws)]
    sims = members()
    _seed_states(sims, ws)
    b = Batch(sims, max_record=64)
    b.set_schedule(grid_blocks=24, graph_steps=4)
    b.step(21)
    Fb, bad = b.forces()
    assert not bad.any()
    ref = members()
    _seed_states(ref, ws)
    for i, r in enumerate(ref):
        r.step(21)
        np.testing.assert_array_equal(r.forces(), Fb[i])
        np.testing.assert_array_equal(r.populations(), b.members[i].populations())


def test_schedule_validation():
    """A tile queue needs a persistent grid; tile_queue takes 0 or 1."""
    from paper_2210_10377_amd import LbmError
    b = _batch(MINI[:2])
    with pytest.raises(LbmError):
        b.set_schedule(grid_blocks=0, tile_queue=1)
    with pytest.raises(LbmError):
        b.set_schedule(grid_blocks=16, tile_queue=2)
    b.set_schedule(grid_blocks=16, tile_queue=1)
    assert b.info().schedule.tile_queue == 1
    # tile_shape takes LBM_TILE_AUTO, LBM_TILE_WIDE or LBM_TILE_NARROW
    import ctypes
    from paper_2210_10377_amd import _capi as C
    s = C.lbm_batch_schedule(0, 0, 0, 0, 7)
    assert C.load().lbm_batch_set_schedule(b._h, ctypes.byref(s)) == C.LBM_EINVAL
    b.set_schedule(tile_shape="narrow")
    assert b.info().schedule.tile_shape == C.LBM_TILE_NARROW
