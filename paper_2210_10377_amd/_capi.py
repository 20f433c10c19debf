"""ctypes binding of the C ABI declared in include/lbm.h (argument marshalling only).

Every function of the header is bound under its own name.  Loading fails loudly when
the HIP library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE, LBM_EOVERFLOW = (
    0, -1, -2, -3, -4, -5, -6)
LBM_FP64, LBM_FP32, LBM_FP16DEV, LBM_FP32DEV, LBM_FP32SR = 0, 1, 2, 3, 4
LBM_BCX_INLET_OUTLET, LBM_BCX_PERIODIC = 0, 1
LBM_BCY_WALL, LBM_BCY_PERIODIC = 0, 1
LBM_FORCE_MEA_A, LBM_FORCE_MEA_B, LBM_FORCE_DRTT, LBM_FORCE_SI = 1, 2, 4, 8
LBM_FORCE_DRTT_POST, LBM_FORCE_ALL = 16, 31
LBM3D_FORCE_ALL = 15
LBM_COLL_BGK, LBM_COLL_REGULARIZED, LBM_COLL_KBC = 0, 1, 2
LBM_LAYOUT_AUTO, LBM_LAYOUT_ROWS, LBM_LAYOUT_PLANES = 0, 1, 2
LBM_TILE_AUTO, LBM_TILE_WIDE, LBM_TILE_NARROW = 0, 1, 2

ERROR_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP",
               -4: "LBM_ENONFINITE", -5: "LBM_ESTATE", -6: "LBM_EOVERFLOW"}

# Every entry point of include/lbm.h.
EXPORTS = ("lbm_create", "lbm_workspace_bytes", "lbm_bind", "lbm_step", "lbm_forces",
           "lbm_coefficients", "lbm_destroy", "lbm_get_links", "lbm_get_info",
           "lbm_get_populations", "lbm_set_populations", "lbm_state_bytes", "lbm_get_state",
           "lbm_set_state", "lbm_last_error", "lbm_set_inlet", "lbm_set_tau", "lbm_reset",
           "lbm_adjoint_bytes", "lbm_adjoint_forward", "lbm_adjoint_backward",
           "lbm_set_body_motion", "lbm_set_mask", "lbm_boundary_cp", "lbm_step_static",
           "lbm_batch_create", "lbm_batch_workspace_bytes", "lbm_batch_bind",
           "lbm_batch_set_schedule", "lbm_batch_autotune", "lbm_batch_step",
           "lbm_batch_forces", "lbm_batch_get_info", "lbm_batch_destroy",
           "lbm_batch_last_error")

# Every entry point of include/lbm3d.h.
EXPORTS3 = ("lbm3d_create", "lbm3d_workspace_bytes", "lbm3d_bind", "lbm3d_step",
            "lbm3d_forces", "lbm3d_get_populations", "lbm3d_set_populations",
            "lbm3d_get_links", "lbm3d_get_info", "lbm3d_destroy", "lbm3d_last_error",
            "lbm3d_set_body_motion", "lbm3d_set_mask", "lbm3d_state_bytes",
            "lbm3d_get_state", "lbm3d_set_state", "lbm3d_reset", "lbm3d_set_tau",
            "lbm3d_set_inlet")


class lbm_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("box", ctypes.c_int32 * 4),
                ("max_record", ctypes.c_int32),
                ("rho_ref", ctypes.c_double), ("u_ref", ctypes.c_double),
                ("l_ref", ctypes.c_double), ("collision", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("tile", ctypes.c_int32)]


class lbm_inlet(ctypes.Structure):
    _fields_ = [("ux", ctypes.POINTER(ctypes.c_double)), ("rho_w", ctypes.c_double)]


class lbm_info(ctypes.Structure):
    _fields_ = [("n_fluid", ctypes.c_int64), ("n_links", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_general", ctypes.c_int64),
                ("n_box", ctypes.c_int64), ("steps_done", ctypes.c_int64),
                ("n_recorded", ctypes.c_int64), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("plane_stride", ctypes.c_int64),
                ("pitch", ctypes.c_int32), ("elem_bytes", ctypes.c_int32)]


class lbm3d_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("bc_z", ctypes.c_int32),
                ("box", ctypes.c_int32 * 6), ("precision", ctypes.c_int32),
                ("max_record", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class lbm3d_info(ctypes.Structure):
    _fields_ = [("n_fluid", ctypes.c_int64), ("n_links", ctypes.c_int64),
                ("n_box", ctypes.c_int64), ("steps_done", ctypes.c_int64),
                ("n_recorded", ctypes.c_int64), ("n_general", ctypes.c_int32),
                ("n_strips", ctypes.c_int32)]


class lbm_batch_schedule(ctypes.Structure):
    _fields_ = [("grid_blocks", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("tile_order", ctypes.c_uint32), ("tile_queue", ctypes.c_int32),
                ("tile_shape", ctypes.c_int32)]


class lbm_batch_info(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("n_recorded", ctypes.c_int32),
                ("total_tiles", ctypes.c_int64), ("total_fluid", ctypes.c_int64),
                ("total_nodes", ctypes.c_int64), ("steps_done", ctypes.c_int64),
                ("n_graphs", ctypes.c_int32), ("compute_units", ctypes.c_int32),
                ("schedule", lbm_batch_schedule)]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load liblbm.so (built in-tree by ``paper_2210_10377_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run "
                          "`python -m paper_2210_10377_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, dp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint32, ctypes.POINTER(ctypes.c_double))
    sz = ctypes.c_size_t
    L.lbm_create.argtypes = [ctypes.POINTER(lbm_grid), ctypes.POINTER(ctypes.c_uint8),
                             ctypes.c_double, ctypes.POINTER(lbm_inlet), ctypes.POINTER(vp)]
    L.lbm_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.lbm_bind.argtypes = [vp, vp, sz, vp]
    L.lbm_step.argtypes = [vp, i32, u32]
    L.lbm_forces.argtypes = [vp, dp, i64, ctypes.POINTER(i64)]
    L.lbm_coefficients.argtypes = [vp, dp, i64, dp]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_get_links.argtypes = [vp, ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
    L.lbm_get_info.argtypes = [vp, ctypes.POINTER(lbm_info)]
    L.lbm_get_populations.argtypes = [vp, dp]
    L.lbm_set_populations.argtypes = [vp, dp]
    L.lbm_state_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.lbm_get_state.argtypes = [vp, vp, sz]
    L.lbm_set_state.argtypes = [vp, vp, sz]
    L.lbm_set_inlet.argtypes = [vp, dp]
    L.lbm_set_tau.argtypes = [vp, ctypes.c_double]
    L.lbm_reset.argtypes = [vp]
    L.lbm_boundary_cp.argtypes = [vp, i32, i32, dp, ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
    L.lbm_step_static.argtypes = [vp, vp, vp, sz, i32, u32, dp, i64, vp]
    L.lbm_set_body_motion.argtypes = [vp] + [ctypes.c_double] * 5
    L.lbm_set_mask.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(i32), dp]
    L.lbm_adjoint_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
    L.lbm_adjoint_forward.argtypes = [vp, vp, sz, i32, i32, i32, i32, ctypes.c_double,
                                      ctypes.c_double, dp]
    L.lbm_adjoint_backward.argtypes = [vp, ctypes.c_double, dp, dp]
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp)]
    L.lbm_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.lbm_batch_bind.argtypes = [vp, vp, sz, vp]
    L.lbm_batch_set_schedule.argtypes = [vp, ctypes.POINTER(lbm_batch_schedule)]
    L.lbm_batch_autotune.argtypes = [vp, i32, u32, ctypes.POINTER(lbm_batch_schedule),
                                     ctypes.POINTER(ctypes.c_double)]
    L.lbm_batch_step.argtypes = [vp, i32, u32]
    L.lbm_batch_forces.argtypes = [vp, dp, i64, ctypes.POINTER(i64),
                                   ctypes.POINTER(ctypes.c_uint8)]
    L.lbm_batch_get_info.argtypes = [vp, ctypes.POINTER(lbm_batch_info)]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_last_error.argtypes = [vp]
    L.lbm_batch_last_error.restype = ctypes.c_char_p
    L.lbm3d_create.argtypes = [ctypes.POINTER(lbm3d_grid), ctypes.POINTER(ctypes.c_uint8),
                               ctypes.c_double, dp, ctypes.c_double, ctypes.POINTER(vp)]
    L.lbm3d_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.lbm3d_bind.argtypes = [vp, vp, sz, vp]
    L.lbm3d_step.argtypes = [vp, i32, u32]
    L.lbm3d_forces.argtypes = [vp, dp, i64, ctypes.POINTER(i64)]
    L.lbm3d_get_populations.argtypes = [vp, dp]
    L.lbm3d_set_populations.argtypes = [vp, dp]
    L.lbm3d_get_links.argtypes = [vp, ctypes.POINTER(i64), i64, ctypes.POINTER(i64)]
    L.lbm3d_get_info.argtypes = [vp, ctypes.POINTER(lbm3d_info)]
    L.lbm3d_set_body_motion.argtypes = [vp, dp, dp, dp]
    L.lbm3d_set_mask.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(i32), dp]
    L.lbm3d_state_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.lbm3d_get_state.argtypes = [vp, vp, sz]
    L.lbm3d_set_state.argtypes = [vp, vp, sz]
    L.lbm3d_reset.argtypes = [vp]
    L.lbm3d_set_tau.argtypes = [vp, ctypes.c_double]
    L.lbm3d_set_inlet.argtypes = [vp, dp]
    L.lbm3d_destroy.argtypes = [vp]
    L.lbm3d_destroy.restype = None
    L.lbm3d_last_error.argtypes = [vp]
    L.lbm3d_last_error.restype = ctypes.c_char_p
    for name in EXPORTS + EXPORTS3:
        if not name.endswith("last_error") and name != "lbm3d_destroy":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc, handle=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(handle)
        raise LbmError(rc, msg.decode() if msg else "")
    return rc


def check3(rc, handle=None):
    if rc != LBM_OK:
        msg = load().lbm3d_last_error(handle)
        raise LbmError(rc, msg.decode() if msg else "")
    return rc


def check_batch(rc, batch=None):
    if rc != LBM_OK:
        msg = load().lbm_batch_last_error(batch)
        raise LbmError(rc, msg.decode() if msg else "")
    return rc
