"""MI355X-native D2Q9 lattice Boltzmann step with per-step flow forces.

Kaushal, Succi & Ansumali, "Flow force calculation in Lattice Boltzmann Method"
(arXiv:2210.10377): BGK collide-stream with half-way bounce-back, momentum exchange
under algorithms A and B, and the discrete Reynolds-transport-theorem force, as HIP
kernels for gfx950 behind the C ABI of include/lbm.h.
"""
from ._capi import LbmError  # noqa: F401
from .sim import ALL_SCHEMES, Plan, Sim, scheme_mask  # noqa: F401
from .batch import Batch  # noqa: F401
from .sim3 import Plan3, Sim3  # noqa: F401
