"""torch.autograd.Function for the time-averaged body force of a lattice run.

Forward: a run of the HIP step kernel from rest with the given inlet profile and
relaxation time, checkpointed every `every` steps, returning
J = (1/T) sum_{t0 <= t < t0+T} w . F_B(t) (momentum exchange, algorithm B).
Backward: the library's adjoint sweep (recompute each checkpoint segment, then one
reverse-step kernel per step) giving dJ/du_in and dJ/dtau.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from ._capi import LBM_ESTATE, LbmError
from .sim import Sim


@dataclass(frozen=True)
class ObjectiveSpec:
    n_steps: int
    every: int
    t0: int
    T: int
    w: tuple = (1.0, 0.0)


class LbmObjective(torch.autograd.Function):
    """J(u_in, tau) for a fixed geometry held by ``sim``.  u_in: float64 [ny]; tau:
    float64 scalar tensor.  Returns a float64 scalar tensor on u_in's device.  Several
    objectives may share one ``sim``: a backward whose forward run has been replaced on
    the handle recomputes that run from its saved inputs first."""

    @staticmethod
    def _run(sim: Sim, u_in: np.ndarray, tau: float, spec: ObjectiveSpec) -> float:
        sim.set_inlet(u_in)
        sim.set_tau(tau)
        sim.reset()
        return sim.adjoint_forward(spec.n_steps, spec.every, spec.t0, spec.T, spec.w)

    @staticmethod
    def forward(ctx, u_in, tau, sim: Sim, spec: ObjectiveSpec):
        u = u_in.detach().to("cpu", torch.float64).numpy().copy()
        t = float(tau)
        J = LbmObjective._run(sim, u, t, spec)
        ctx.sim = sim
        ctx.inputs = (u, t, spec)
        ctx.run = sim.adjoint_runs
        ctx.devices = (u_in.device, tau.device)
        return torch.tensor(J, dtype=torch.float64, device=u_in.device)

    @staticmethod
    def backward(ctx, grad_out):
        sim = ctx.sim
        if sim.adjoint_runs != ctx.run:
            # Another forward run (another objective on the same lattice) has replaced
            # this one's checkpoints: recompute it from the saved inputs.
            LbmObjective._run(sim, *ctx.inputs)
            ctx.run = sim.adjoint_runs
        try:
            g_uin, g_tau = sim.adjoint_backward(float(grad_out))
        except LbmError as e:
            if e.code != LBM_ESTATE:
                raise
            # The lattice was stepped or changed since the forward run: recompute it.
            LbmObjective._run(sim, *ctx.inputs)
            ctx.run = sim.adjoint_runs
            g_uin, g_tau = sim.adjoint_backward(float(grad_out))
        du = torch.from_numpy(np.ascontiguousarray(g_uin)).to(ctx.devices[0])
        dt = torch.tensor(g_tau, dtype=torch.float64, device=ctx.devices[1])
        return du, dt, None, None


def objective(u_in, tau, sim: Sim, spec: ObjectiveSpec):
    return LbmObjective.apply(u_in, tau, sim, spec)
