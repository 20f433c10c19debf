"""CPU checks of the three-dimensional C ABI (include/lbm3d.h): every declared symbol is
exported, the ctypes structs match the C layout, the planned link lists are bitwise the
oracle's on varied geometries and boundary codes, and bad configurations are refused."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads
from oracle import d3q27 as D
from workloads import d3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "lbm3d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm3d_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(capi):
    lib = capi.load()
    names = _header_functions()
    assert len(names) == 19
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(capi.EXPORTS3) == names


def test_struct_layout_matches_header(capi, tmp_path):
    structs = {"lbm3d_grid": capi.lbm3d_grid, "lbm3d_info": capi.lbm3d_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm3d.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout3.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout3"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


def _geometries():
    rng = np.random.default_rng(7)
    rnd = (rng.random((9, 10, 12)) < 0.15).astype(np.uint8)
    edge = np.zeros((8, 9, 10), np.uint8)
    edge[2:4, 3:5, 8:10] = 1        # touches the outlet plane
    edge[0, 4, 4] = 1               # on a z wall
    edge[5, 0:2, 0:2] = 1           # on the inlet plane and a y wall
    return {
        "sphere_walls": (d3.sphere_mask(24, 16, 14, 9, 7.5, 6.5, 4), (0, 0, 0)),
        "sphere_periodic": (d3.sphere_mask(24, 16, 14, 9, 7.5, 6.5, 4), (1, 1, 1)),
        "extruded_periodic_z": (d3.extrude(workloads.cylinder_mask(30, 14, 10, 6.5, 3), 6),
                                (0, 0, 1)),
        "random_mixed": (rnd, (1, 0, 1)),
        "random_walls": (rnd, (0, 1, 0)),
        "edges": (edge, (0, 0, 0)),
    }


@pytest.mark.parametrize("name", list(_geometries()))
def test_links_bitwise_vs_oracle(name):
    from paper_2210_10377_amd import Plan3
    mask, (bx, by, bz) = _geometries()[name]
    p = Plan3(mask, bc_x=bx, bc_y=by, bc_z=bz)
    L = p.links()
    O = D.links(mask, bc_x=bx, bc_y=by, bc_z=bz)
    assert L.shape == O.shape and L.shape[0] > 0
    assert np.array_equal(L, O)
    inf = p.info()
    assert inf.n_links == len(O)
    assert inf.n_fluid == int((mask == 0).sum())


def test_box_counts_and_admissibility_agree_with_oracle(capi):
    from paper_2210_10377_amd import Plan3
    w = d3.sphere_channel_64x32x32()
    p = Plan3(w.mask, box=w.box)
    x0, x1, y0, y1, z0, z1 = w.box
    assert p.info().n_box == int((w.mask[z0:z1, y0:y1, x0:x1] == 0).sum())
    L = capi.load()
    m = d3.extrude(workloads.cylinder_mask(40, 20, 15, 9.5, 4), 8)
    cases = [((5, 26, 2, 18, 0, 8), 1), ((5, 26, 2, 18, 1, 7), 1), ((5, 26, 2, 18, 0, 8), 0),
             ((0, 26, 2, 18, 0, 8), 1), ((5, 26, 6, 18, 0, 8), 1), ((5, 26, 2, 18, 0, 8), 1)]
    for box, bz in cases:
        ok = D.box_admissible(m, box, bc_y=D.BC_WALL, bc_z=bz)
        g = capi.lbm3d_grid()
        g.nx, g.ny, g.nz, g.bc_x, g.bc_y, g.bc_z = 40, 20, 8, 0, 0, bz
        for k in range(6):
            g.box[k] = box[k]
        g.precision, g.max_record = capi.LBM_FP32, 4
        uin = np.full((8, 20), 0.03)
        h = ctypes.c_void_p()
        mm = np.ascontiguousarray(m)
        rc = L.lbm3d_create(ctypes.byref(g), mm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            0.7, uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0,
                            ctypes.byref(h))
        assert (rc == capi.LBM_OK) == ok, (box, bz)
        if rc == capi.LBM_OK:
            L.lbm3d_destroy(h)


@pytest.mark.parametrize("case", ["tau", "bc", "mask", "precision", "record", "inlet", "size",
                                  "collision"])
def test_create_rejects_invalid(capi, case):
    L = capi.load()
    nx, ny, nz = 12, 10, 8
    m = np.zeros((nz, ny, nx), np.uint8)
    g = capi.lbm3d_grid()
    g.nx, g.ny, g.nz, g.bc_x, g.bc_y, g.bc_z = nx, ny, nz, 0, 0, 0
    for k in range(6):
        g.box[k] = -1
    g.precision, g.max_record = capi.LBM_FP32, 4
    tau = 0.7
    uin = np.full((nz, ny), 0.02)
    up = uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if case == "tau":
        tau = 0.5
    elif case == "bc":
        g.bc_z = 5
    elif case == "mask":
        m[3, 3, 3] = 2
    elif case == "precision":
        g.precision = 9
    elif case == "record":
        g.max_record = 0
    elif case == "inlet":
        up = None
    elif case == "size":
        g.nz = 1
        m = np.zeros((1, ny, nx), np.uint8)
    elif case == "collision":
        g.collision = capi.LBM_COLL_KBC   # not offered in three dimensions
    h = ctypes.c_void_p()
    rc = L.lbm3d_create(ctypes.byref(g), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), tau,
                        up, 1.0, ctypes.byref(h))
    assert rc == capi.LBM_EINVAL
    assert L.lbm3d_last_error(None)


def test_workspace_accounts_for_both_buffers_and_unbound_step_is_estate(capi):
    from paper_2210_10377_amd import Plan3
    w = d3.sphere_channel_64x32x32()
    for prec, esz in (("fp64", 8), ("fp32", 4), ("fp16dev", 2)):
        p = Plan3(w.mask, box=w.box, precision=prec)
        assert p.workspace_bytes() >= 2 * 27 * esz * w.nx * w.ny * w.nz
    L = capi.load()
    assert L.lbm3d_step(p._h, 1, 15) == capi.LBM_ESTATE


def _create3(capi, mask, box, bc=(0, 0, 0)):
    L = capi.load()
    nz, ny, nx = mask.shape
    g = capi.lbm3d_grid()
    g.nx, g.ny, g.nz = nx, ny, nz
    g.bc_x, g.bc_y, g.bc_z = bc
    for k in range(6):
        g.box[k] = box[k] if box is not None else -1
    g.precision, g.max_record = capi.LBM_FP32, 4
    uin = np.full((nz, ny), 0.03)
    h = ctypes.c_void_p()
    m = np.ascontiguousarray(mask, np.uint8)
    rc = L.lbm3d_create(ctypes.byref(g), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0.7,
                        uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0, ctypes.byref(h))
    assert rc == capi.LBM_OK
    return L, h


def _set_mask3(capi, L, h, mask, box=None):
    m = np.ascontiguousarray(mask, np.uint8)
    bp = None
    if box is not None:
        bp = ctypes.cast((ctypes.c_int32 * 6)(*box), ctypes.POINTER(ctypes.c_int32))
    imp = np.full(3, 7.0)
    rc = L.lbm3d_set_mask(h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), bp,
                          imp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, imp


def test_set_mask_validation_and_unbound_replanning(capi):
    """lbm3d_set_mask refuses a mask value other than 0/1, a box added or removed, an
    inadmissible box and a larger control-volume sweep than at create, changing nothing;
    on an unbound handle it re-plans (links and box as the oracle's) and returns a zero
    impulse."""
    nx, ny, nz = 48, 20, 20
    box = (7, 22, 3, 17, 3, 17)
    m0 = d3.sphere_mask(nx, ny, nz, 14, 9.5, 9.5, 4)
    m1 = d3.sphere_mask(nx, ny, nz, 15, 9.5, 9.5, 4)
    L, h = _create3(capi, m0, box)
    info = capi.lbm3d_info()

    def links():
        L.lbm3d_get_info(h, ctypes.byref(info))
        return info.n_links, info.n_box

    before = links()
    bad = m1.copy()
    bad[0, 0, 0] = 2
    assert _set_mask3(capi, L, h, bad)[0] == capi.LBM_EINVAL
    assert _set_mask3(capi, L, h, m1, (-1, 0, 0, 0, 0, 0))[0] == capi.LBM_EINVAL
    assert _set_mask3(capi, L, h, m1, (12, 22, 3, 17, 3, 17))[0] == capi.LBM_EINVAL
    assert _set_mask3(capi, L, h, m1, (2, 40, 2, 18, 2, 18))[0] == capi.LBM_ENOMEM
    assert L.lbm3d_last_error(h)
    assert links() == before
    rc, imp = _set_mask3(capi, L, h, m1, (8, 23, 3, 17, 3, 17))
    assert rc == capi.LBM_OK and np.all(imp == 0.0)
    O = D.links(m1)
    assert links() == (len(O), int((m1[3:17, 3:17, 8:23] == 0).sum()))
    out = np.zeros((len(O), 2), np.int64)
    n = ctypes.c_int64()
    L.lbm3d_get_links(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(O), ctypes.byref(n))
    assert np.array_equal(out, O)
    L.lbm3d_destroy(h)


def test_set_mask_refuses_more_force_slots_than_reserved(capi):
    """A mask with far more force strips than the one at create (one solid node, then
    solid nodes in every row) is refused with LBM_ENOMEM."""
    nx, ny, nz = 64, 40, 40
    m0 = np.zeros((nz, ny, nx), np.uint8)
    m0[20, 20, 30] = 1
    L, h = _create3(capi, m0, None, bc=(0, 1, 1))
    m1 = np.zeros_like(m0)
    m1[:, :, 30] = 1
    m1[::2, ::2, 30] = 0
    assert _set_mask3(capi, L, h, m1)[0] == capi.LBM_ENOMEM
    m2 = m0.copy()
    m2[10, 10, 10] = 1
    assert _set_mask3(capi, L, h, m2)[0] == capi.LBM_OK
    L.lbm3d_destroy(h)


def test_layouts_workspace_and_limits(capi):
    """The state layouts: ROWS and PLANES both hold two buffers of 27 populations per
    node; an unknown layout is refused; ROWS beyond 32-bit offsets is LBM_ENOMEM (the
    mask is never read: the check comes first)."""
    from paper_2210_10377_amd import Plan3
    w = d3.sphere_channel_64x32x32()
    sizes = {}
    for lay in ("auto", "rows", "planes"):
        sizes[lay] = Plan3(w.mask, box=w.box, precision="fp32", layout=lay).workspace_bytes()
        assert sizes[lay] >= 2 * 27 * 4 * w.nx * w.ny * w.nz
    assert sizes["auto"] == sizes["rows"]
    L = capi.load()

    def create(nx, ny, nz, layout):
        g = capi.lbm3d_grid()
        g.nx, g.ny, g.nz, g.bc_x, g.bc_y, g.bc_z = nx, ny, nz, 1, 1, 1
        for k in range(6):
            g.box[k] = -1
        g.precision, g.max_record, g.layout = capi.LBM_FP32, 4, layout
        m = np.zeros((nz, ny, nx), np.uint8)   # zero pages: never touched when refused
        h = ctypes.c_void_p()
        rc = L.lbm3d_create(ctypes.byref(g), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            0.7, None, 1.0, ctypes.byref(h))
        if rc == capi.LBM_OK:
            L.lbm3d_destroy(h)
        return rc

    assert create(12, 10, 8, 7) == capi.LBM_EINVAL
    # 27 x 160 x 120 rows of 4160 elements (4096 padded) = 2.16e9 >= 2^31
    assert create(4096, 160, 120, capi.LBM_LAYOUT_ROWS) == capi.LBM_ENOMEM
    assert "row-interleaved" in L.lbm3d_last_error(None).decode()


def test_auto_layout_falls_back_to_planes_beyond_32bit_offsets():
    """2048 x 256 x 160 (84 M nodes): the row-interleaved buffer would pass 2^31
    elements, so AUTO takes the planar layout (same workspace as PLANES)."""
    from paper_2210_10377_amd import Plan3
    m = np.zeros((160, 256, 2048), np.uint8)
    m[70:90, 118:138, 500:520] = 1
    sizes = {lay: Plan3(m, bc_x=1, bc_y=1, bc_z=1, precision="fp16dev",
                        layout=lay).workspace_bytes() for lay in ("auto", "planes")}
    assert sizes["auto"] == sizes["planes"] >= 2 * 27 * 2 * m.size


def test_parameter_and_state_calls_validate_without_a_gpu(capi):
    """lbm3d_set_tau refuses tau <= 1/2 and non-finite values; lbm3d_set_inlet refuses
    non-finite values and a lattice without an inlet; the state calls need a bound
    handle (LBM_ESTATE); lbm3d_state_bytes holds the header and one state buffer."""
    from paper_2210_10377_amd import Plan3
    w = d3.sphere_channel_64x32x32()
    L = capi.load()
    p = Plan3(w.mask, box=w.box)
    h = p._h
    assert L.lbm3d_set_tau(h, 0.5) == capi.LBM_EINVAL
    assert L.lbm3d_set_tau(h, float("nan")) == capi.LBM_EINVAL
    assert L.lbm3d_set_tau(h, 0.8) == capi.LBM_OK
    bad = np.full((w.nz, w.ny), np.inf)
    dp = ctypes.POINTER(ctypes.c_double)
    assert L.lbm3d_set_inlet(h, bad.ctypes.data_as(dp)) == capi.LBM_EINVAL
    ok = np.full((w.nz, w.ny), 0.02)
    assert L.lbm3d_set_inlet(h, ok.ctypes.data_as(dp)) == capi.LBM_OK
    q = Plan3(w.mask, bc_x=1, box=w.box)
    assert L.lbm3d_set_inlet(q._h, ok.ctypes.data_as(dp)) == capi.LBM_EINVAL
    n = ctypes.c_size_t()
    assert L.lbm3d_state_bytes(h, ctypes.byref(n)) == capi.LBM_OK
    assert n.value >= 27 * 4 * w.nx * w.ny * w.nz
    buf = ctypes.create_string_buffer(n.value)
    assert L.lbm3d_get_state(h, buf, n.value) == capi.LBM_ESTATE
    assert L.lbm3d_set_state(h, buf, n.value) == capi.LBM_ESTATE
    assert L.lbm3d_reset(h) == capi.LBM_ESTATE
