"""CPU tests of the C ABI library: it loads, exports every entry point the header
declares, and its host-side plan (validation, link classification) matches the oracle's
bit for bit.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(capi):
    lib = capi.load()
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(capi.EXPORTS) == names


def test_struct_layout_matches_header(capi, tmp_path):
    """The ctypes mirrors of lbm_grid, lbm_inlet and lbm_info have the C compiler's
    sizes and field offsets."""
    import subprocess
    structs = {"lbm_grid": capi.lbm_grid, "lbm_inlet": capi.lbm_inlet, "lbm_info": capi.lbm_info,
               "lbm_batch_schedule": capi.lbm_batch_schedule,
               "lbm_batch_info": capi.lbm_batch_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


@pytest.mark.parametrize("seed", range(8))
def test_links_bitwise_vs_oracle_random_masks(orc, seed):
    from paper_2210_10377_amd import Plan
    rng = np.random.default_rng(500 + seed)
    ny, nx = rng.integers(3, 30, size=2)
    m = (rng.uniform(size=(ny, nx)) < rng.uniform(0.05, 0.5)).astype(np.uint8)
    for bcx in (0, 1):
        for bcy in (0, 1):
            p = Plan(m, 0.8, np.full(ny, 0.01), bc_x=bcx, bc_y=bcy)
            assert np.array_equal(p.links(), orc.links(m, bc_x=bcx, bc_y=bcy))


def test_links_bitwise_workload_geometries(orc):
    from paper_2210_10377_amd import Plan
    w = workloads.cylinder_channel_200x80()
    p = Plan(w.mask, w.tau, w.uin, box=w.box)
    assert np.array_equal(p.links(), orc.links(w.mask))
    for aoa in (0.0, 4.0, 8.0):
        m = workloads.naca0012_mask(1024, 512, 256, 320, 256, aoa)
        p = Plan(m, 0.6, np.full(512, 0.05))
        L = p.links()
        assert np.array_equal(L, orc.links(m))
        assert len(L) > 1500


def test_info_counts():
    from paper_2210_10377_amd import Plan
    w = workloads.cylinder_channel_200x80()
    p = Plan(w.mask, w.tau, w.uin, box=w.box)
    inf = p.info()
    assert inf.n_fluid == 200 * 80 - 317
    assert inf.n_box == 60 * 60 - 317
    assert inf.n_links == len(p.links())


def _create(capi, mask, tau=0.8, uin=0.05, box=None, **kw):
    from paper_2210_10377_amd import Plan
    return Plan(mask, tau, None if uin is None else np.full(mask.shape[0], uin), box=box, **kw)


@pytest.mark.parametrize("case", ["small", "tau", "tau_nan", "mask", "box_edge", "box_body",
                                  "bcx", "prec", "no_inlet", "inlet_nan", "max_record"])
def test_create_rejects_invalid(capi, case):
    from paper_2210_10377_amd import LbmError
    m = np.zeros((20, 30), np.uint8)
    m[8:11, 10:13] = 1
    kw = {}
    if case == "small":
        m = np.zeros((2, 10), np.uint8)
    elif case == "tau":
        kw["tau"] = 0.5
    elif case == "tau_nan":
        kw["tau"] = float("nan")
    elif case == "mask":
        m[0, 0] = 2
    elif case == "box_edge":
        kw["box"] = (0, 20, 2, 18)
    elif case == "box_body":
        kw["box"] = (5, 12, 2, 18)    # body column 12 not strictly inside
    elif case == "bcx":
        kw["bc_x"] = 7
    elif case == "prec":
        pass
    elif case == "no_inlet":
        kw["uin"] = None
    elif case == "inlet_nan":
        kw["uin"] = float("nan")
    elif case == "max_record":
        kw["max_record"] = 0
    with pytest.raises(LbmError) as e:
        if case == "prec":
            from paper_2210_10377_amd import sim
            sim.PRECISIONS["bogus"] = 9
            try:
                _create(capi, m, precision="bogus", **kw)
            finally:
                del sim.PRECISIONS["bogus"]
        else:
            _create(capi, m, **kw)
    assert e.value.code == capi.LBM_EINVAL


def test_box_admissibility_agrees_with_oracle(capi, orc):
    """The library and the oracle accept and reject the same boxes."""
    from paper_2210_10377_amd import LbmError
    w = workloads.cylinder_channel_200x80()
    rng = np.random.default_rng(3)
    for _ in range(40):
        x0, y0 = rng.integers(0, 40, 2)
        x1, y1 = x0 + rng.integers(1, 100), y0 + rng.integers(1, 60)
        box = (int(x0), int(x1), int(y0), int(y1))
        want = orc.box_admissible(w.mask, box)
        try:
            _create(capi, w.mask, box=box)
            got = True
        except LbmError:
            got = False
        assert got == want, box


def test_grid_too_large_is_enomem(capi):
    from paper_2210_10377_amd import LbmError
    m = np.zeros((3, 3), np.uint8)
    g = capi.lbm_grid()
    g.nx, g.ny = 1 << 16, 1 << 16
    g.precision = capi.LBM_FP32
    for k in range(4):
        g.box[k] = -1
    g.max_record = 1
    g.bc_x = capi.LBM_BCX_PERIODIC
    big = np.zeros(1, np.uint8)  # never read: the size check comes first
    h = ctypes.c_void_p()
    rc = capi.load().lbm_create(ctypes.byref(g), big.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                0.8, None, ctypes.byref(h))
    assert rc == capi.LBM_ENOMEM
    del m


def test_step_unbound_is_estate(capi):
    from paper_2210_10377_amd import Plan
    p = Plan(np.zeros((8, 8), np.uint8), 0.8, np.full(8, 0.01))
    assert capi.load().lbm_step(p._h, 1, 7) == capi.LBM_ESTATE
    out = np.zeros(6)
    k = ctypes.c_int64()
    assert capi.load().lbm_forces(p._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1,
                                  ctypes.byref(k)) == capi.LBM_ESTATE


def test_workspace_size_accounts_for_buffers(capi):
    """Both state layouts hold two buffers of nine populations per node: row-interleaved
    (the default: directions a padded row apart, rows nine padded rows apart) and
    planar (rows a padded row apart, directions a padded plane apart)."""
    from paper_2210_10377_amd import Plan
    for prec, s in (("fp64", 8), ("fp32", 4), ("fp16dev", 2), ("fp32dev", 4)):
        m = np.zeros((100, 300), np.uint8)
        p = Plan(m, 0.8, np.full(100, 0.01), precision=prec)
        inf = p.info()
        assert inf.elem_bytes == s
        assert inf.plane_stride >= 300 and inf.plane_stride % 64 == 0
        assert inf.pitch == 9 * inf.plane_stride
        assert p.workspace_bytes() >= 2 * inf.pitch * 100 * s + 300 * 100 * 4
        q = Plan(m, 0.8, np.full(100, 0.01), precision=prec, layout="planes")
        inf = q.info()
        assert inf.pitch >= 300 and inf.pitch % 64 == 0
        assert inf.plane_stride >= inf.pitch * 100
        assert q.workspace_bytes() >= 2 * 9 * inf.plane_stride * s + 300 * 100 * 4


def test_layout_validation(capi):
    """An unknown layout is refused; the row-interleaved layout beyond 32-bit offsets is
    LBM_ENOMEM before the mask is read."""
    L = capi.load()

    def create(nx, ny, layout):
        g = capi.lbm_grid()
        g.nx, g.ny, g.bc_x, g.bc_y = nx, ny, capi.LBM_BCX_PERIODIC, capi.LBM_BCY_PERIODIC
        for k in range(4):
            g.box[k] = -1
        g.precision, g.max_record, g.layout = capi.LBM_FP16DEV, 4, layout
        g.rho_ref = g.u_ref = g.l_ref = 1.0
        m = np.zeros((ny, nx), np.uint8)   # zero pages: never touched when refused
        h = ctypes.c_void_p()
        rc = L.lbm_create(ctypes.byref(g), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          0.8, None, ctypes.byref(h))
        info = capi.lbm_info()
        if rc == capi.LBM_OK:
            L.lbm_get_info(h, ctypes.byref(info))
            L.lbm_destroy(h)
        return rc, info

    assert create(16, 16, 7)[0] == capi.LBM_EINVAL
    # 9 x 16384 rows of 32896 elements (32768 + 128) = 4.85e9 >= 2^31
    rc, _ = create(32768, 16384, capi.LBM_LAYOUT_ROWS)
    assert rc == capi.LBM_ENOMEM
    assert "row-interleaved" in L.lbm_last_error(None).decode()


def test_batch_create_rejects_bad_members(capi):
    """lbm_batch_create validates its members without a GPU: null, unbound, repeated."""
    from paper_2210_10377_amd import Plan
    L = capi.load()
    p = Plan(workloads.cylinder_mask(40, 20, 10, 9.5, 3), uin=0.05)
    out = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 2)(p._h.value, p._h.value)
    assert L.lbm_batch_create(arr, 2, 8, ctypes.byref(out)) == capi.LBM_EINVAL
    assert b"unbound" in L.lbm_batch_last_error(None)
    assert L.lbm_batch_create(arr, 0, 8, ctypes.byref(out)) == capi.LBM_EINVAL
    assert L.lbm_batch_create(None, 1, 8, ctypes.byref(out)) == capi.LBM_EINVAL
    assert L.lbm_batch_create(arr, 1, 0, ctypes.byref(out)) == capi.LBM_EINVAL
    nul = (ctypes.c_void_p * 1)(None)
    assert L.lbm_batch_create(nul, 1, 8, ctypes.byref(out)) == capi.LBM_EINVAL
    assert L.lbm_batch_destroy(None) == capi.LBM_OK


def test_batched_instances_recipe():
    """The batched instance list: sizes, body types and parameter ranges of the recipe,
    and every control volume admissible."""
    import oracle
    ws = workloads.batched_instances()
    assert len(ws) == 256
    assert all(64 <= w.nx <= 512 and w.ny == w.nx // 2 for w in ws)
    assert all(0.5 < w.tau < 0.7 for w in ws)
    kinds = [w.meta["type"] for w in ws]
    assert 100 < kinds.count("cylinder") < 156
    assert all(oracle.box_admissible(w.mask, w.box) for w in ws[:32])
    assert 12e6 < sum(w.nx * w.ny for w in ws) < 14e6


def test_collision_code_validation_and_adjoint_bgk_only(capi):
    """Unknown collision codes are rejected at create; the adjoint entry points refuse
    the regularized collision before touching the device."""
    from paper_2210_10377_amd import Plan
    L = capi.load()
    mask = workloads.cylinder_mask(40, 20, 10, 9.5, 3)
    g = capi.lbm_grid()
    g.nx, g.ny, g.bc_x, g.bc_y, g.precision = 40, 20, 1, 0, capi.LBM_FP32
    for k in range(4):
        g.box[k] = -1
    g.max_record, g.rho_ref, g.u_ref, g.l_ref = 4, 1.0, 1.0, 1.0
    g.collision = 7
    h = ctypes.c_void_p()
    m = np.ascontiguousarray(mask)
    assert L.lbm_create(ctypes.byref(g), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0.6,
                        None, ctypes.byref(h)) == capi.LBM_EINVAL
    assert b"collision" in L.lbm_last_error(None)
    J = ctypes.c_double()
    reg = Plan(mask, uin=0.05, collision="regularized")
    rc = L.lbm_adjoint_forward(reg._h, ctypes.c_void_p(256), 1 << 20, 10, 5, 0, 5, 1.0, 0.0,
                               ctypes.byref(J))
    assert rc == capi.LBM_EINVAL and b"BGK" in L.lbm_last_error(reg._h)
    bgk = Plan(mask, uin=0.05)
    rc = L.lbm_adjoint_forward(bgk._h, ctypes.c_void_p(256), 1 << 20, 10, 5, 0, 5, 1.0, 0.0,
                               ctypes.byref(J))
    assert rc == capi.LBM_ESTATE
    # The adjoint covers the FP64, FP32 and FP32-deviation storages; binary16 deviations
    # are refused by both calls before anything else.
    h16 = Plan(mask, uin=0.05, precision="fp16dev")
    rc = L.lbm_adjoint_forward(h16._h, ctypes.c_void_p(256), 1 << 20, 10, 5, 0, 5, 1.0, 0.0,
                               ctypes.byref(J))
    assert rc == capi.LBM_EINVAL and b"storages" in L.lbm_last_error(h16._h)
    gu = np.zeros(20)
    gt = ctypes.c_double()
    rc = L.lbm_adjoint_backward(h16._h, 1.0, gu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.byref(gt))
    assert rc == capi.LBM_EINVAL


def test_body_motion_validation_and_adjoint_refusal(capi):
    """lbm_set_body_motion rejects non-finite values (unbound handle, no device call);
    a handle with a body in motion is refused by the adjoint before touching the
    device, and a zero motion is a body at rest again."""
    from paper_2210_10377_amd import Plan
    L = capi.load()
    mask = workloads.cylinder_mask(40, 20, 10, 9.5, 3)
    p = Plan(mask, uin=0.05)
    assert L.lbm_set_body_motion(p._h, float("nan"), 0.0, 0.0, 0.0, 0.0) == capi.LBM_EINVAL
    assert b"finite" in L.lbm_last_error(p._h)
    assert L.lbm_set_body_motion(p._h, 0.0, 0.0, float("inf"), 0.0, 0.0) == capi.LBM_EINVAL
    assert L.lbm_set_body_motion(p._h, 0.01, 0.0, 0.002, 10.0, 9.5) == capi.LBM_OK
    J = ctypes.c_double()
    rc = L.lbm_adjoint_forward(p._h, ctypes.c_void_p(256), 1 << 20, 10, 5, 0, 5, 1.0, 0.0,
                               ctypes.byref(J))
    assert rc == capi.LBM_EINVAL and b"rest" in L.lbm_last_error(p._h)
    assert L.lbm_set_body_motion(p._h, 0.0, 0.0, 0.0, 10.0, 9.5) == capi.LBM_OK
    rc = L.lbm_adjoint_forward(p._h, ctypes.c_void_p(256), 1 << 20, 10, 5, 0, 5, 1.0, 0.0,
                               ctypes.byref(J))
    assert rc == capi.LBM_ESTATE


def test_set_mask_validation_and_replanning(capi, orc):
    """lbm_set_mask on an unbound handle: the link list follows the new mask (bitwise
    the oracle's); bad mask values, a box that no longer encloses the body, adding a
    control volume, a mask needing more force slots than reserved and a larger box are
    refused and leave the handle as it was."""
    from paper_2210_10377_amd import Plan
    L = capi.load()
    nx, ny = 120, 40
    m0 = workloads.cylinder_mask(nx, ny, 30, 19.5, 6)
    m1 = workloads.cylinder_mask(nx, ny, 33, 20.5, 6)
    p = Plan(m0, uin=0.04, box=(20, 41, 8, 32))
    links0 = p.links()
    imp = np.full(2, 7.0)
    dp = ctypes.POINTER(ctypes.c_double)

    def setm(m, box=None):
        m = np.ascontiguousarray(m, dtype=np.uint8)
        bp = None if box is None else (ctypes.c_int32 * 4)(*box)
        return L.lbm_set_mask(p._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                              bp if bp is None else ctypes.cast(bp, ctypes.POINTER(ctypes.c_int32)),
                              imp.ctypes.data_as(dp))

    assert setm(m1, (22, 43, 8, 32)) == capi.LBM_OK
    assert np.all(imp == 0.0)          # unbound: no state, no impulse
    assert np.array_equal(p.links(), orc.links(m1))
    bad = m1.copy()
    bad[3, 3] = 2
    assert setm(bad) == capi.LBM_EINVAL
    assert setm(workloads.cylinder_mask(nx, ny, 60, 20.5, 6)) == capi.LBM_EINVAL  # outside box
    assert setm(m1, (-1, -1, -1, -1)) == capi.LBM_EINVAL and b"added or removed" in L.lbm_last_error(p._h)
    assert setm(m1, (10, 60, 4, 36)) == capi.LBM_ENOMEM                            # larger box
    q = Plan(np.zeros((ny, 2048), np.uint8), uin=0.04)
    mm = np.zeros((ny, 2048), np.uint8)
    mm[2:ny - 2, ::64] = 1
    rc = L.lbm_set_mask(q._h, mm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), None, None)
    assert rc == capi.LBM_ENOMEM and b"slots" in L.lbm_last_error(q._h)
    assert np.array_equal(p.links(), orc.links(m1))  # unchanged by the refusals


def test_auto_layout_falls_back_to_planes_beyond_32bit_offsets():
    """30000 x 8000 (240 M nodes): the row-interleaved buffer would pass 2^31 elements,
    so AUTO takes the planar layout (rows a padded row apart)."""
    from paper_2210_10377_amd import Plan
    m = np.zeros((8000, 30000), np.uint8)
    m[3900:4100, 5000:5200] = 1
    p = Plan(m, 0.8, np.full(8000, 0.01), precision="fp16dev")
    inf = p.info()
    assert inf.pitch == 30016 + 128 and inf.plane_stride >= inf.pitch * 8000


def test_boundary_cp_validation(capi):
    """lbm_boundary_cp refuses an unbound handle (no device work) before anything else."""
    from paper_2210_10377_amd import Plan
    L = capi.load()
    mask = workloads.cylinder_mask(40, 20, 10, 9.5, 3)
    p = Plan(mask, uin=0.05)
    n = ctypes.c_int64(-7)
    cp = np.zeros(64)
    rc = L.lbm_boundary_cp(p._h, 1, 9, cp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None,
                           64, ctypes.byref(n))
    assert rc == capi.LBM_ESTATE and b"bound" in L.lbm_last_error(p._h)


def test_static_step_validation_without_device(capi):
    """lbm_step_static checks its arguments and the size of the static scratch before any
    device call: a grid whose pull codes alone exceed LBM_STATIC_SCRATCH_BYTES is
    refused with LBM_ENOMEM, bad buffers and a short force output with LBM_EINVAL."""
    from paper_2210_10377_amd import Plan
    L = capi.load()
    big = Plan(np.zeros((2048, 4096), np.uint8), bc_x=capi.LBM_BCX_PERIODIC,
               bc_y=capi.LBM_BCY_PERIODIC)
    F = np.zeros((4, 5, 2))
    fp = F.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    vp = ctypes.c_void_p
    rc = L.lbm_step_static(big._h, vp(256), vp(512), 1 << 40, 1, 0, None, 0, None)
    assert rc == capi.LBM_ENOMEM and b"static scratch" in L.lbm_last_error(big._h)
    small = Plan(workloads.cylinder_mask(40, 20, 10, 9.5, 3), uin=0.05)
    assert L.lbm_step_static(small._h, vp(256), vp(256), 1 << 20, 1, 0, None, 0, None) == capi.LBM_EINVAL
    assert L.lbm_step_static(small._h, vp(256), vp(300), 1 << 20, 1, 0, None, 0, None) == capi.LBM_EINVAL
    assert L.lbm_step_static(small._h, vp(256), vp(512), 16, 1, 0, None, 0, None) == capi.LBM_ENOMEM
    assert L.lbm_step_static(small._h, vp(256), vp(512), 1 << 20, 5, 2, fp, 4, None) == capi.LBM_EINVAL
    assert L.lbm_step_static(small._h, vp(256), vp(512), 1 << 20, -1, 0, None, 0, None) == capi.LBM_EINVAL
    assert L.lbm_step_static(small._h, vp(256), vp(512), 1 << 20, 0, 2, None, 0, None) == capi.LBM_OK


def test_edge_word_bit_form_equals_the_rule(tmp_path):
    """The kernels' bit-operation form of the edge pull codes equals the rule the plan
    uses, at every node of small grids, for every boundary combination (compiled from
    the library's own header with g++)."""
    import subprocess
    src = tmp_path / "edge.cpp"
    src.write_text(r'''
#include <cstdio>
#include "plan.h"
using namespace lbm;
int main() {
  int bad = 0, n = 0;
  for (int nx = 3; nx <= 7; ++nx)
    for (int ny = 3; ny <= 6; ++ny)
      for (int bx = 0; bx < 2; ++bx)
        for (int by = 0; by < 2; ++by)
          for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
              ++n;
              if (edge_word(nx, ny, bx, by, x, y) != edge_word_bits(nx, ny, bx, by, x, y)) ++bad;
            }
  std::printf("%d %d\n", n, bad);
  return bad != 0;
}
''')
    exe = tmp_path / "edge"
    subprocess.check_call(["g++", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2210_10377_amd", "csrc"),
                           str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    n, bad = (int(v) for v in out.stdout.split())
    assert n > 1000 and bad == 0


def test_stochastic_rounding_storage_scope_without_device(capi):
    """LBM_FP32SR (binary32 populations rounded stochastically) plans like the other
    storages, with 4-byte elements, in 2-D and 3-D; the allocation-free step, which
    cannot carry the handle's step count, refuses it before any device call."""
    from paper_2210_10377_amd import Plan, Plan3
    L = capi.load()
    mask = workloads.cylinder_mask(40, 20, 10, 9.5, 3)
    p = Plan(mask, uin=0.05, precision="fp32sr")
    q = Plan(mask, uin=0.05, precision="fp32")
    assert p.info().elem_bytes == 4 and p.workspace_bytes() == q.workspace_bytes()
    assert np.array_equal(p.links(), q.links())
    # The adjoint takes it (an unbound handle gets LBM_ESTATE, not a storage refusal).
    J = ctypes.c_double()
    rc = L.lbm_adjoint_forward(p._h, ctypes.c_void_p(256), 1 << 20, 10, 5, 0, 5, 1.0, 0.0,
                               ctypes.byref(J))
    assert rc == capi.LBM_ESTATE
    vp = ctypes.c_void_p
    rc = L.lbm_step_static(p._h, vp(256), vp(512), 1 << 20, 1, 0, None, 0, None)
    assert rc == capi.LBM_EINVAL and b"stochastically" in L.lbm_last_error(p._h)
    p3 = Plan3(np.zeros((8, 8, 16), np.uint8), uin=0.05, precision="fp32sr")
    q3 = Plan3(np.zeros((8, 8, 16), np.uint8), uin=0.05, precision="fp32")
    assert p3.workspace_bytes() == q3.workspace_bytes()
    assert np.array_equal(p3.links(), q3.links())
