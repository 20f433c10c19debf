"""Three-dimensional (D3Q27) lattice with a body and per-step forces, over the C ABI of
include/lbm3d.h (argument marshalling only; every step runs in the library's kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi as C
from .sim import COLLISIONS, LAYOUTS, PRECISIONS, scheme_mask

# The estimators of the three-dimensional lattice.
ALL_SCHEMES = ("A", "B", "DRTT", "SI")


class Sim3:
    """mask: uint8 [nz, ny, nx] (1 = solid).  tau: tau_lb.  uin: inlet x-velocity,
    scalar or [nz, ny] (ignored for periodic x).  box: (x0, x1, y0, y1, z0, z1) or None.
    bc_y, bc_z: C.LBM_BCY_WALL or C.LBM_BCY_PERIODIC.  collision: "bgk" or
    "regularized".  layout: "auto", "rows" or "planes" (device layout of the state)."""

    def __init__(self, mask, tau, uin=None, *, precision="fp32", bc_x=C.LBM_BCX_INLET_OUTLET,
                 bc_y=C.LBM_BCY_WALL, bc_z=C.LBM_BCY_WALL, box=None, max_record=1024,
                 rho_w=1.0, device="cuda", stream=None, collision="bgk", layout="auto"):
        import torch

        self._lib = C.load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.nz, self.ny, self.nx = mask.shape
        self.precision = precision
        g = C.lbm3d_grid()
        g.nx, g.ny, g.nz = self.nx, self.ny, self.nz
        g.bc_x, g.bc_y, g.bc_z = int(bc_x), int(bc_y), int(bc_z)
        b = (-1,) * 6 if box is None else tuple(int(v) for v in box)
        for k in range(6):
            g.box[k] = b[k]
        g.precision = PRECISIONS[precision]
        g.max_record = int(max_record)
        g.collision = COLLISIONS[collision]
        g.layout = LAYOUTS[layout]
        self.collision = collision
        up = None
        if uin is not None:
            self._uin = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64),
                                                             (self.nz, self.ny)))
            up = self._uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        C.check3(self._lib.lbm3d_create(ctypes.byref(g),
                                        mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        float(tau), up, float(rho_w), ctypes.byref(h)), None)
        self._h = h
        self.max_record = int(max_record)
        nbytes = ctypes.c_size_t()
        C.check3(self._lib.lbm3d_workspace_bytes(self._h, ctypes.byref(nbytes)), self._h)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        C.check3(self._lib.lbm3d_bind(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                      int(nbytes.value), ctypes.c_void_p(self.stream.cuda_stream)),
                 self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm3d_destroy(h)
            self._h = None

    def step(self, n: int, schemes=ALL_SCHEMES):
        C.check3(self._lib.lbm3d_step(self._h, int(n), scheme_mask(schemes)), self._h)

    def set_body_motion(self, u=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0),
                        centre=(0.0, 0.0, 0.0)) -> None:
        """Rigid motion of the body: translation u, angular velocity omega about centre
        (three 3-vectors); the moving-wall rule on its links from the next step."""
        vs = [np.ascontiguousarray(np.asarray(v, np.float64).reshape(3)) for v in (u, omega, centre)]
        dp = ctypes.POINTER(ctypes.c_double)
        C.check3(self._lib.lbm3d_set_body_motion(self._h, *[v.ctypes.data_as(dp) for v in vs]),
                 self._h)

    def set_mask(self, mask, box=None) -> np.ndarray:
        """Move the body through the grid: a new mask (and control volume, if given)
        from the next step.  Uncovered nodes are refilled at the wall velocity; returns
        the impulse (3,) the fluid hands to the body in the change."""
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.shape != (self.nz, self.ny, self.nx):
            raise ValueError("mask shape differs from the lattice")
        bp = None
        if box is not None:
            barr = (ctypes.c_int32 * 6)(*[int(v) for v in box])
            bp = ctypes.cast(barr, ctypes.POINTER(ctypes.c_int32))
        imp = np.zeros(3)
        C.check3(self._lib.lbm3d_set_mask(self._h,
                                          mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                          bp, imp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                 self._h)
        return imp

    def get_state(self) -> bytes:
        """Checkpoint: the exact stored state and step counter as an opaque blob."""
        n = ctypes.c_size_t()
        C.check3(self._lib.lbm3d_state_bytes(self._h, ctypes.byref(n)), self._h)
        buf = ctypes.create_string_buffer(n.value)
        C.check3(self._lib.lbm3d_get_state(self._h, buf, n.value), self._h)
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        C.check3(self._lib.lbm3d_set_state(self._h, blob, len(blob)), self._h)

    def reset(self) -> None:
        C.check3(self._lib.lbm3d_reset(self._h), self._h)

    def set_tau(self, tau: float) -> None:
        C.check3(self._lib.lbm3d_set_tau(self._h, float(tau)), self._h)

    def set_inlet(self, uin) -> None:
        """Inlet x-velocity, scalar or [nz, ny]."""
        u = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64), (self.nz, self.ny)))
        C.check3(self._lib.lbm3d_set_inlet(self._h, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                 self._h)

    def info(self) -> C.lbm3d_info:
        inf = C.lbm3d_info()
        C.check3(self._lib.lbm3d_get_info(self._h, ctypes.byref(inf)), self._h)
        return inf

    def forces(self) -> np.ndarray:
        """[k, 4 (A, B, DRTT, SI), 3 (x, y, z)] of the steps recorded since the last call."""
        k = self.info().n_recorded
        out = np.zeros((max(k, 1), 4, 3))
        got = ctypes.c_int64()
        rc = self._lib.lbm3d_forces(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    max(k, 1), ctypes.byref(got))
        if rc not in (C.LBM_OK, C.LBM_ENONFINITE):
            C.check3(rc, self._h)
        self.last_nonfinite = rc == C.LBM_ENONFINITE
        return out[:got.value]

    def run(self, n: int, schemes=ALL_SCHEMES) -> np.ndarray:
        outs, left = [], int(n)
        while left > 0:
            k = min(left, self.max_record)
            self.step(k, schemes)
            outs.append(self.forces())
            left -= k
        return np.concatenate(outs) if outs else np.zeros((0, 4, 3))

    def populations(self) -> np.ndarray:
        out = np.zeros((27, self.nz, self.ny, self.nx))
        C.check3(self._lib.lbm3d_get_populations(
            self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)
        return out

    def set_populations(self, S) -> None:
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(27, self.nz, self.ny, self.nx)
        C.check3(self._lib.lbm3d_set_populations(
            self._h, S.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)

    def links(self) -> np.ndarray:
        n = ctypes.c_int64()
        C.check3(self._lib.lbm3d_get_links(self._h, None, 0, ctypes.byref(n)), self._h)
        out = np.zeros((max(n.value, 1), 2), np.int64)
        C.check3(self._lib.lbm3d_get_links(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           n.value, ctypes.byref(n)), self._h)
        return out[:n.value]


class Plan3:
    """A planned, unbound 3-D handle (no device needed): links and info for CPU checks."""

    def __init__(self, mask, tau=0.8, uin=0.0, *, precision="fp32", bc_x=C.LBM_BCX_INLET_OUTLET,
                 bc_y=C.LBM_BCY_WALL, bc_z=C.LBM_BCY_WALL, box=None, max_record=16,
                 collision="bgk", layout="auto"):
        self._lib = C.load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        nz, ny, nx = mask.shape
        g = C.lbm3d_grid()
        g.nx, g.ny, g.nz, g.bc_x, g.bc_y, g.bc_z = nx, ny, nz, int(bc_x), int(bc_y), int(bc_z)
        b = (-1,) * 6 if box is None else tuple(int(v) for v in box)
        for k in range(6):
            g.box[k] = b[k]
        g.precision = PRECISIONS[precision]
        g.max_record = int(max_record)
        g.collision = COLLISIONS[collision]
        g.layout = LAYOUTS[layout]
        self._uin = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64), (nz, ny)))
        h = ctypes.c_void_p()
        C.check3(self._lib.lbm3d_create(ctypes.byref(g),
                                        mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        float(tau), self._uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        1.0, ctypes.byref(h)), None)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm3d_destroy(h)
            self._h = None

    links = Sim3.links
    info = Sim3.info

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        C.check3(self._lib.lbm3d_workspace_bytes(self._h, ctypes.byref(n)), self._h)
        return n.value
