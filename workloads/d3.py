"""Seeded synthetic inputs for the three-dimensional path (inputs only, none of the lattice
Boltzmann arithmetic): sphere and extruded-airfoil masks on a [nz, ny, nx] lattice,
control-volume boxes, inlet planes and random population fields.

The shapes follow the paper's three-dimensional run (Kaushal, Succi & Ansumali,
arXiv:2210.10377, Sec. V, flow past a 3-D NACA0012 at zero incidence in a domain of
80 x 8 x 4 chords with the airfoil 24 chords from the inlet) and a sphere in a channel as
the small parity case.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import naca0012_mask, tau_from_re

# A positive base vector of 27 entries, in the direction order of the population arrays
# (rest; faces; edges; corners), close to a lattice rest state.  Any positive vector is
# a valid input; this one keeps random fields in the stable regime.
NEAR_REST_BASE3 = np.array([8.0] + [2.0] * 6 + [0.5] * 12 + [0.125] * 8) / 27.0


def sphere_mask(nx: int, ny: int, nz: int, xc: float, yc: float, zc: float,
                r: float) -> np.ndarray:
    """uint8 [nz, ny, nx]: 1 where the node (x, y, z) lies within distance r of the
    centre (closed ball)."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (((x - xc) ** 2 + (y - yc) ** 2 + (z - zc) ** 2) <= r * r).astype(np.uint8)


def extrude(mask2d: np.ndarray, nz: int, z0: int = 0, z1: int | None = None) -> np.ndarray:
    """A two-dimensional [ny, nx] mask repeated over the planes z0 <= z < z1 of a
    [nz, ny, nx] lattice (all planes by default)."""
    z1 = nz if z1 is None else z1
    out = np.zeros((nz,) + mask2d.shape, np.uint8)
    out[z0:z1] = mask2d
    return out


def default_box3(mask: np.ndarray, margin: int) -> tuple[int, int, int, int, int, int]:
    """The bounding box of the solid nodes grown by `margin` on every side, clipped to
    one node inside the domain: (x0, x1, y0, y1, z0, z1), half-open."""
    nz, ny, nx = mask.shape
    zs, ys, xs = np.nonzero(mask)
    return (max(int(xs.min()) - margin, 1), min(int(xs.max()) + 1 + margin, nx - 1),
            max(int(ys.min()) - margin, 1), min(int(ys.max()) + 1 + margin, ny - 1),
            max(int(zs.min()) - margin, 1), min(int(zs.max()) + 1 + margin, nz - 1))


def near_rest_state3(nx: int, ny: int, nz: int, seed: int, amp: float = 0.01,
                     dtype=np.float64) -> np.ndarray:
    """[27, nz, ny, nx] field base_i * (1 + amp * xi), xi ~ U(-1, 1), seeded, rounded once
    to `dtype` so that every consumer reads the same numbers."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(27, nz, ny, nx))
    S = NEAR_REST_BASE3[:, None, None, None] * (1.0 + amp * xi)
    return S.astype(dtype).astype(np.float64)


@dataclass
class Workload3:
    """One synthetic three-dimensional run."""
    name: str
    nx: int
    ny: int
    nz: int
    mask: np.ndarray
    tau: float
    uin: np.ndarray          # [nz, ny] inlet x-velocity
    box: tuple | None
    steps: int
    u_ref: float
    l_ref: float
    area_ref: float          # reference area of the force coefficients
    bc_y: int = 0            # 0 walls, 1 periodic
    bc_z: int = 0
    meta: dict = field(default_factory=dict)


def sphere_channel_64x32x32() -> Workload3:
    """Sphere of diameter 10 at (20, 15.5, 15.5) in a 64 x 32 x 32 duct with walls in y
    and z, uniform inlet 0.04, Re 20 on the diameter, control volume the sphere's box
    grown by 3 nodes, 300 steps from rest (the small parity case)."""
    nx, ny, nz, d, u, re = 64, 32, 32, 10.0, 0.04, 20.0
    mask = sphere_mask(nx, ny, nz, 20.0, 15.5, 15.5, d / 2)
    return Workload3("sphere_64x32x32_re20", nx, ny, nz, mask, tau_from_re(u, d, re),
                     np.full((nz, ny), u), default_box3(mask, 3), 300, u, d,
                     np.pi * d * d / 4, meta={"re": re, "d": d})


def naca3d(ppc: int, re: float, u: float = 0.05, steps: int = 2000) -> Workload3:
    """NACA0012 at zero incidence spanning a domain of 80 x 8 x 4 chords (ppc nodes per
    chord), periodic across the span (z), walls in y, leading edge 24 chords from the
    inlet, uniform inlet u; control volume the airfoil's box grown by a quarter chord in
    x and y over the whole (periodic) span."""
    nx, ny, nz = 80 * ppc, 8 * ppc, 4 * ppc
    xq, yq = 24 * ppc + ppc // 4, ny // 2
    m2 = naca0012_mask(nx, ny, ppc, xq, yq, 0.0)
    mask = extrude(m2, nz)
    ys, xs = np.nonzero(m2)
    q = max(2, ppc // 4)
    box = (int(xs.min()) - q, int(xs.max()) + 1 + q, int(ys.min()) - q, int(ys.max()) + 1 + q,
           0, nz)
    return Workload3(f"naca3d_{nx}x{ny}x{nz}_ppc{ppc}_re{re:g}", nx, ny, nz, mask,
                     tau_from_re(u, ppc, re), np.full((nz, ny), u), box, steps, u,
                     float(ppc), float(ppc * nz), bc_z=1,
                     meta={"re": re, "ppc": ppc, "chord": ppc, "span": nz, "xq": xq, "yq": yq})
