"""Python front end of the HIP library: torch supplies the device workspace and the
stream; every step of the lattice Boltzmann path runs in the library's kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi as C

PRECISIONS = {"fp64": C.LBM_FP64, "fp32": C.LBM_FP32, "fp16dev": C.LBM_FP16DEV,
              "fp32dev": C.LBM_FP32DEV, "fp32sr": C.LBM_FP32SR}
SCHEMES = {"A": C.LBM_FORCE_MEA_A, "B": C.LBM_FORCE_MEA_B, "DRTT": C.LBM_FORCE_DRTT,
           "SI": C.LBM_FORCE_SI, "DRTT_POST": C.LBM_FORCE_DRTT_POST}
ALL_SCHEMES = ("A", "B", "DRTT", "SI", "DRTT_POST")
# Number of estimators in a force row: A, B, DRTT, SI, DRTT-post.
NSCHEMES = 5
COLLISIONS = {"bgk": C.LBM_COLL_BGK, "regularized": C.LBM_COLL_REGULARIZED,
              "kbc": C.LBM_COLL_KBC}
LAYOUTS = {"auto": C.LBM_LAYOUT_AUTO, "rows": C.LBM_LAYOUT_ROWS,
           "planes": C.LBM_LAYOUT_PLANES}
TILES = {"auto": C.LBM_TILE_AUTO, "wide": C.LBM_TILE_WIDE, "narrow": C.LBM_TILE_NARROW}


def scheme_mask(schemes) -> int:
    if isinstance(schemes, int):
        return schemes
    m = 0
    for s in schemes:
        m |= SCHEMES[s]
    return m


class Sim:
    """One lattice with a body, bound to a torch-allocated device workspace.

    mask: uint8 [ny, nx] (1 = solid).  tau: lattice relaxation time tau_lb.
    uin: inlet velocity per row (scalar or [ny]); ignored for periodic x.
    box: control-volume box (x0, x1, y0, y1) for the DRTT force, or None.
    collision: "bgk" (Eq. CollideAdv), "regularized" or "kbc" (entropic; for tau_lb
    close to 1/2).  layout: "auto", "rows" or "planes" (device layout of the state).
    tile: "auto", "wide" (256 x 1) or "narrow" (64 x 4) step-kernel tiles.
    """

    def __init__(self, mask, tau, uin=None, *, precision="fp32", bc_x=C.LBM_BCX_INLET_OUTLET,
                 bc_y=C.LBM_BCY_WALL, box=None, max_record=4096, rho_ref=1.0, u_ref=1.0,
                 l_ref=1.0, rho_w=1.0, device="cuda", stream=None, collision="bgk",
                 layout="auto", tile="auto"):
        import torch

        self._lib = C.load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = mask.shape
        self.precision = precision
        g = C.lbm_grid()
        g.nx, g.ny, g.bc_x, g.bc_y = self.nx, self.ny, int(bc_x), int(bc_y)
        g.precision = PRECISIONS[precision]
        b = (-1, -1, -1, -1) if box is None else tuple(int(v) for v in box)
        for k in range(4):
            g.box[k] = b[k]
        g.max_record = int(max_record)
        g.rho_ref, g.u_ref, g.l_ref = float(rho_ref), float(u_ref), float(l_ref)
        g.collision = COLLISIONS[collision]
        g.layout = LAYOUTS[layout]
        g.tile = TILES[tile]
        self.collision = collision
        self._grid = g
        inlet = None
        if uin is not None:
            self._uin = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64),
                                                             (self.ny,)))
            inlet = C.lbm_inlet(self._uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                float(rho_w))
        h = ctypes.c_void_p()
        rc = self._lib.lbm_create(ctypes.byref(g),
                                  mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  float(tau), ctypes.byref(inlet) if inlet else None,
                                  ctypes.byref(h))
        C.check(rc, None)
        self._h = h
        self.max_record = int(max_record)
        nbytes = ctypes.c_size_t()
        C.check(self._lib.lbm_workspace_bytes(self._h, ctypes.byref(nbytes)), self._h)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        C.check(self._lib.lbm_bind(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                   int(nbytes.value), ctypes.c_void_p(self.stream.cuda_stream)),
                self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm_destroy(h)
            self._h = None

    # -- stepping ---------------------------------------------------------------------
    def step(self, n: int, schemes=ALL_SCHEMES):
        """Enqueue n steps on the stream; force rows are read back with ``forces``."""
        m = scheme_mask(schemes)
        C.check(self._lib.lbm_step(self._h, int(n), m), self._h)

    def forces(self) -> np.ndarray:
        """[k, 5 (A, B, DRTT, SI, DRTT_POST), 2 (x, y)] float64 forces of the steps since
        the last call."""
        info = self.info()
        k = info.n_recorded
        out = np.zeros((max(k, 1), NSCHEMES, 2))
        got = ctypes.c_int64()
        rc = self._lib.lbm_forces(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  max(k, 1), ctypes.byref(got))
        if rc not in (C.LBM_OK, C.LBM_ENONFINITE):
            C.check(rc, self._h)
        self.last_nonfinite = rc == C.LBM_ENONFINITE
        return out[:got.value]

    def run(self, n: int, schemes=ALL_SCHEMES) -> np.ndarray:
        """n steps with forces, chunked to the ring capacity."""
        outs = []
        left = int(n)
        while left > 0:
            k = min(left, self.max_record)
            self.step(k, schemes)
            outs.append(self.forces())
            left -= k
        return np.concatenate(outs) if outs else np.zeros((0, NSCHEMES, 2))

    def coefficients(self, forces: np.ndarray) -> np.ndarray:
        f = np.ascontiguousarray(forces, dtype=np.float64)
        out = np.empty_like(f)
        C.check(self._lib.lbm_coefficients(self._h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           f.shape[0], out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                self._h)
        return out

    # -- inspection -------------------------------------------------------------------
    def info(self) -> C.lbm_info:
        inf = C.lbm_info()
        C.check(self._lib.lbm_get_info(self._h, ctypes.byref(inf)), self._h)
        return inf

    def links(self) -> np.ndarray:
        return links_of(self._h)

    def populations(self) -> np.ndarray:
        out = np.zeros((9, self.ny, self.nx))
        C.check(self._lib.lbm_get_populations(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                self._h)
        return out

    def set_populations(self, S) -> None:
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(9, self.ny, self.nx)
        C.check(self._lib.lbm_set_populations(self._h, S.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                self._h)

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        C.check(self._lib.lbm_state_bytes(self._h, ctypes.byref(n)), self._h)
        buf = ctypes.create_string_buffer(n.value)
        C.check(self._lib.lbm_get_state(self._h, buf, n.value), self._h)
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        C.check(self._lib.lbm_set_state(self._h, blob, len(blob)), self._h)

    # -- parameters -------------------------------------------------------------------
    def set_inlet(self, ux) -> None:
        u = np.ascontiguousarray(np.broadcast_to(np.asarray(ux, np.float64), (self.ny,)))
        C.check(self._lib.lbm_set_inlet(self._h, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                self._h)

    def set_tau(self, tau: float) -> None:
        C.check(self._lib.lbm_set_tau(self._h, float(tau)), self._h)

    def set_body_motion(self, ux: float = 0.0, uy: float = 0.0, omega: float = 0.0,
                        xc: float = 0.0, yc: float = 0.0) -> None:
        """Rigid motion of the body: translation (ux, uy), rotation rate omega about
        (xc, yc); the moving-wall rule on its links from the next step."""
        C.check(self._lib.lbm_set_body_motion(self._h, float(ux), float(uy), float(omega),
                                              float(xc), float(yc)), self._h)

    def set_mask(self, mask, box=None) -> np.ndarray:
        """Move the body through the grid: a new mask (and control volume, if given)
        from the next step.  Uncovered nodes are refilled at the wall velocity; returns
        the impulse (2,) the fluid hands to the body in the change."""
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.shape != (self.ny, self.nx):
            raise ValueError("mask shape differs from the lattice")
        bp = None
        if box is not None:
            barr = (ctypes.c_int32 * 4)(*[int(v) for v in box])
            bp = ctypes.cast(barr, ctypes.POINTER(ctypes.c_int32))
        imp = np.zeros(2)
        C.check(self._lib.lbm_set_mask(self._h, mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       bp, imp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                self._h)
        return imp

    def reset(self) -> None:
        C.check(self._lib.lbm_reset(self._h), self._h)

    def boundary_cp(self, ref=None):
        """Pressure coefficient (p - p_inf) / (rho_ref u_ref^2 / 2) at every boundary fluid
        node of the current state, p = rho/3; p_inf at the reference node ref = (x, y)
        (far upstream), or rho_ref/3 when ref is None.  Returns (node indices y*nx + x
        as int32 [n], C_p float64 [n]), nodes in row-major order."""
        x, y = (-1, -1) if ref is None else (int(ref[0]), int(ref[1]))
        n = ctypes.c_int64()
        ip = ctypes.POINTER(ctypes.c_int32)
        k = self.info().n_links  # every boundary node has a link: an upper bound
        cp = np.zeros(max(k, 1))
        nodes = np.zeros(max(k, 1), np.int32)
        C.check(self._lib.lbm_boundary_cp(self._h, x, y, cp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          nodes.ctypes.data_as(ip), max(k, 1), ctypes.byref(n)),
                self._h)
        return nodes[:n.value], cp[:n.value]

    # -- adjoint ----------------------------------------------------------------------
    def adjoint_forward(self, n_steps: int, every: int, t0: int, T: int, w=(1.0, 0.0)) -> float:
        """Run n_steps from the current state with checkpoints every `every` steps and
        return J = (1/T) sum_{t0 <= t < t0+T} w . F_B(t)."""
        import torch
        nb = ctypes.c_size_t()
        C.check(self._lib.lbm_adjoint_bytes(self._h, int(n_steps), int(every), ctypes.byref(nb)),
                self._h)
        ws = getattr(self, "adjoint_workspace", None)
        if ws is None or ws.numel() < nb.value:
            self.adjoint_workspace = None
            with torch.cuda.device(self.device):
                self.adjoint_workspace = torch.empty(int(nb.value), dtype=torch.uint8,
                                                     device=self.device)
        J = ctypes.c_double()
        # Every forward run replaces the one the handle holds for the backward sweep.
        self.adjoint_runs = getattr(self, "adjoint_runs", 0) + 1
        C.check(self._lib.lbm_adjoint_forward(
            self._h, ctypes.c_void_p(self.adjoint_workspace.data_ptr()),
            int(self.adjoint_workspace.numel()), int(n_steps), int(every), int(t0), int(T),
            float(w[0]), float(w[1]), ctypes.byref(J)), self._h)
        return J.value

    def adjoint_backward(self, seed: float = 1.0):
        """(dJ/du_in [ny], dJ/dtau), each times `seed`, of the last adjoint_forward run."""
        g = np.zeros(self.ny)
        gt = ctypes.c_double()
        C.check(self._lib.lbm_adjoint_backward(self._h, float(seed),
                                               g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               ctypes.byref(gt)), self._h)
        return g, gt.value


def links_of(handle) -> np.ndarray:
    lib = C.load()
    n = ctypes.c_int64()
    C.check(lib.lbm_get_links(handle, None, 0, ctypes.byref(n)), handle)
    out = np.zeros((max(n.value, 1), 2), np.int32)
    C.check(lib.lbm_get_links(handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              n.value, ctypes.byref(n)), handle)
    return out[:n.value]


class Plan:
    """A handle created but never bound: host-side classification only (no GPU)."""

    def __init__(self, mask, tau=0.8, uin=None, *, precision="fp32", bc_x=C.LBM_BCX_INLET_OUTLET,
                 bc_y=C.LBM_BCY_WALL, box=None, max_record=16, collision="bgk", layout="auto",
                 tile="auto"):
        self._lib = C.load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        ny, nx = mask.shape
        g = C.lbm_grid()
        g.nx, g.ny, g.bc_x, g.bc_y = nx, ny, int(bc_x), int(bc_y)
        g.precision = PRECISIONS[precision]
        b = (-1, -1, -1, -1) if box is None else tuple(int(v) for v in box)
        for k in range(4):
            g.box[k] = b[k]
        g.max_record = int(max_record)
        g.rho_ref = g.u_ref = g.l_ref = 1.0
        g.collision = COLLISIONS[collision]
        g.layout = LAYOUTS[layout]
        g.tile = TILES[tile]
        inlet = None
        if uin is not None:
            self._uin = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64), (ny,)))
            inlet = C.lbm_inlet(self._uin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0)
        h = ctypes.c_void_p()
        rc = self._lib.lbm_create(ctypes.byref(g), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  float(tau), ctypes.byref(inlet) if inlet else None, ctypes.byref(h))
        C.check(rc, None)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm_destroy(h)
            self._h = None

    def links(self):
        return links_of(self._h)

    def info(self):
        inf = C.lbm_info()
        C.check(self._lib.lbm_get_info(self._h, ctypes.byref(inf)), self._h)
        return inf

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        C.check(self._lib.lbm_workspace_bytes(self._h, ctypes.byref(n)), self._h)
        return n.value
