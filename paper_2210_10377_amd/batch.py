"""Batched stepping of many independent lattices (one kernel launch per step for all of
them, optionally replayed from captured HIP graphs), over the C ABI's lbm_batch_*
calls.  Every instance computes exactly what ``Sim.step`` computes for it."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi as C
from .sim import ALL_SCHEMES, NSCHEMES, Sim, scheme_mask

# Tile shape of every instance in the batch: each member's own, or one for all.
TILE_SHAPES = {"auto": C.LBM_TILE_AUTO, "wide": C.LBM_TILE_WIDE, "narrow": C.LBM_TILE_NARROW}


class Batch:
    """A batch over bound ``Sim`` members of one precision.

    The members keep their states (``member.populations()`` reads them); the batch
    records force rows in its own ring of ``max_record`` rows per instance.
    """

    def __init__(self, members, max_record: int = 1024, stream=None):
        import torch

        self._lib = C.load()
        self.members = list(members)
        if not self.members:
            raise ValueError("a batch needs at least one member")
        self.max_record = int(max_record)
        arr = (ctypes.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        h = ctypes.c_void_p()
        C.check_batch(self._lib.lbm_batch_create(arr, len(self.members), self.max_record,
                                                 ctypes.byref(h)), None)
        self._h = h
        nbytes = ctypes.c_size_t()
        C.check_batch(self._lib.lbm_batch_workspace_bytes(self._h, ctypes.byref(nbytes)), self._h)
        self.device = self.members[0].device
        self.stream = stream if stream is not None else self.members[0].stream
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        C.check_batch(self._lib.lbm_batch_bind(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                               int(nbytes.value),
                                               ctypes.c_void_p(self.stream.cuda_stream)), self._h)

    @classmethod
    def from_workloads(cls, workloads, precision: str = "fp32", max_record: int = 1024,
                       device="cuda", stream=None, collision=None, tile="auto") -> "Batch":
        """Members built from ``workloads.Workload`` descriptions (walled channels with an
        inlet, the body mask, tau, inlet profile and control volume of each); `collision`
        overrides each workload's collision operator; `tile` is every member's tile shape."""
        members = [Sim(w.mask, w.tau, w.uin, precision=precision, bc_x=w.bc_x, bc_y=w.bc_y,
                       box=w.box, max_record=1, u_ref=w.u_ref, l_ref=w.l_ref, device=device,
                       stream=stream, collision=collision or w.collision, tile=tile)
                   for w in workloads]
        return cls(members, max_record=max_record, stream=stream)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm_batch_destroy(h)
            self._h = None

    def __len__(self):
        return len(self.members)

    # -- schedule ---------------------------------------------------------------------
    def set_schedule(self, grid_blocks: int = 0, graph_steps: int = 0, tile_order: int = 0,
                     tile_queue: int = 0, tile_shape: str = "auto"):
        s = C.lbm_batch_schedule(int(grid_blocks), int(graph_steps), int(tile_order),
                                 int(tile_queue), TILE_SHAPES[tile_shape])
        C.check_batch(self._lib.lbm_batch_set_schedule(self._h, ctypes.byref(s)), self._h)

    def autotune(self, steps: int = 10, schemes=ALL_SCHEMES):
        """Time the candidate schedules (each advances every instance by 2 x steps) and
        keep the fastest; returns (schedule dict, milliseconds per step)."""
        best = C.lbm_batch_schedule()
        ms = ctypes.c_double()
        C.check_batch(self._lib.lbm_batch_autotune(self._h, int(steps), scheme_mask(schemes),
                                                   ctypes.byref(best), ctypes.byref(ms)), self._h)
        return ({"grid_blocks": best.grid_blocks, "graph_steps": best.graph_steps,
                 "tile_order": best.tile_order, "tile_queue": best.tile_queue,
                 "tile_shape": {v: k for k, v in TILE_SHAPES.items()}[best.tile_shape]},
                ms.value)

    def info(self) -> C.lbm_batch_info:
        inf = C.lbm_batch_info()
        C.check_batch(self._lib.lbm_batch_get_info(self._h, ctypes.byref(inf)), self._h)
        return inf

    # -- stepping ---------------------------------------------------------------------
    def step(self, n: int, schemes=ALL_SCHEMES):
        C.check_batch(self._lib.lbm_batch_step(self._h, int(n), scheme_mask(schemes)), self._h)

    def forces(self):
        """(F [n_inst, k, 5 (A, B, DRTT, SI, DRTT-post), 2 (x, y)], nonfinite bool [n_inst]) of the steps
        recorded since the last call."""
        k = self.info().n_recorded
        n = len(self.members)
        out = np.zeros((n, max(k, 1), NSCHEMES, 2))
        flags = np.zeros(n, np.uint8)
        got = ctypes.c_int64()
        rc = self._lib.lbm_batch_forces(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        max(k, 1), ctypes.byref(got),
                                        flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        if rc not in (C.LBM_OK, C.LBM_ENONFINITE):
            C.check_batch(rc, self._h)
        return out[:, :got.value], flags.astype(bool)

    def run(self, n: int, schemes=ALL_SCHEMES):
        """n steps with forces, chunked to the ring capacity; (F, nonfinite) as ``forces``."""
        outs, bad = [], np.zeros(len(self.members), bool)
        left = int(n)
        while left > 0:
            k = min(left, self.max_record)
            self.step(k, schemes)
            F, nf = self.forces()
            outs.append(F)
            bad |= nf
            left -= k
        if not outs:
            return np.zeros((len(self.members), 0, NSCHEMES, 2)), bad
        return np.concatenate(outs, axis=1), bad

    def coefficients(self, F: np.ndarray) -> np.ndarray:
        """Force coefficients 2F / (rho U^2 L) of every instance with its own references."""
        return np.stack([m.coefficients(F[i]) for i, m in enumerate(self.members)])
