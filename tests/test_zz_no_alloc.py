"""The allocation-free entry point lbm_step_static (the step on caller-owned state
buffers with the library's static device scratch) against lbm_step, through the C ABI:
two calls in a row, the second on a smaller grid, states and force rows bitwise equal."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _state_bytes(info, ny):
    return max(9 * info.plane_stride, info.pitch * ny) * info.elem_bytes


def _align256(v):
    return (v + 255) // 256 * 256


def _initial_state(w, precision, seed):
    if precision == "fp16dev":
        return workloads.near_rest_state_fp16dev(w.nx, w.ny, seed=seed, amp=0.03)
    if precision == "fp32dev":
        return workloads.near_rest_state_dev(w.nx, w.ny, seed=seed, amp=0.03, dtype=np.float32)
    dt = np.float32 if precision == "fp32" else np.float64
    return workloads.near_rest_state(w.nx, w.ny, seed=seed, amp=0.03, dtype=dt)


def _compare(w, precision, n, schemes, seed):
    import torch

    from paper_2210_10377_amd import Sim, _capi as C
    from paper_2210_10377_amd.sim import NSCHEMES, scheme_mask
    L = C.load()
    print(f"lbm_step_static vs lbm_step: {w.name} {precision} n={n} schemes={schemes}", flush=True)
    ref = Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=max(n, 1))
    ref.set_populations(_initial_state(w, precision, seed))
    info = ref.info()
    B = _state_bytes(info, w.ny)
    # Both state buffers of the bound handle (buffer 0 holds the state just set).
    state = torch.empty(2 * _align256(B), dtype=torch.uint8, device=ref.device)
    state.copy_(ref.workspace[: 2 * _align256(B)])
    torch.cuda.synchronize()
    # An unbound handle of the same configuration drives the static form.
    mask = np.ascontiguousarray(w.mask, dtype=np.uint8)
    g = C.lbm_grid()
    ctypes.memmove(ctypes.byref(g), ctypes.byref(ref._grid), ctypes.sizeof(g))
    uin = np.ascontiguousarray(w.uin, dtype=np.float64)
    inlet = C.lbm_inlet(uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0)
    hh = ctypes.c_void_p()
    C.check(L.lbm_create(ctypes.byref(g), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                         float(w.tau), ctypes.byref(inlet), ctypes.byref(hh)))
    try:
        m = scheme_mask(schemes)
        ref.step(n, schemes)
        Fr = ref.forces()
        F = np.full((max(n, 1), NSCHEMES, 2), -7.0)
        stream = torch.cuda.current_stream(ref.device)
        p0 = state.data_ptr()
        p1 = p0 + _align256(B)
        rc = L.lbm_step_static(hh, ctypes.c_void_p(p0), ctypes.c_void_p(p1), B, n, m,
                               F.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), max(n, 1),
                               ctypes.c_void_p(stream.cuda_stream))
        C.check(rc, hh)
        torch.cuda.synchronize()
        got = state.cpu().numpy()
        want = ref.workspace[: 2 * _align256(B)].cpu().numpy()
        assert np.array_equal(got, want), "state buffers differ"
        if m:
            assert np.array_equal(F[:n], Fr, equal_nan=True)
        return Fr
    finally:
        L.lbm_destroy(hh)


def test_static_step_matches_bound_step_twice_second_smaller():
    big = workloads.naca_2048x1024(aoa=4.0, re=1000.0)
    Fr = _compare(big, "fp32", 20, ("A", "B", "DRTT", "SI", "DRTT_POST"), seed=3)
    assert np.isfinite(Fr).all()
    small = workloads.cylinder_channel_200x80()
    Fr = _compare(small, "fp64", 7, ("B", "DRTT_POST"), seed=4)
    assert np.isfinite(Fr[:, 1]).all() and np.isnan(Fr[:, 0]).all()


def test_static_step_without_forces_and_deviation_storage():
    small = workloads.cylinder_channel_200x80()
    _compare(small, "fp16dev", 6, (), seed=5)
    _compare(small, "fp32dev", 5, ("A", "B"), seed=6)
