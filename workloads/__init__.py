"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module generates *inputs only*: body masks on the lattice, inlet profiles,
relaxation times from a Reynolds number, control-volume boxes, random population fields
and the batched instance list.  It holds none of the lattice Boltzmann arithmetic (no
streaming, collision, boundary rule or force), so both the oracle and the HIP path can
be fed from it without sharing any of the method.

Workload shapes follow the paper's runs (Kaushal, Succi & Ansumali, arXiv:2210.10377,
Sec. V: cylinder in a channel with walls; NACA0012 with the airfoil at a quarter of the
channel length; Re from 1e2 to 5e5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# A positive base vector for near-rest population fields.  Any positive vector is a
# valid input; this one is close to the rest state of a nine-velocity lattice
# (4/9, 1/9 x4, 1/36 x4), which keeps random fields in the stable regime.
NEAR_REST_BASE = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1], dtype=np.float64) / 36.0


def cylinder_mask(nx: int, ny: int, xc: float, yc: float, r: float) -> np.ndarray:
    """uint8 [ny, nx]; node (ix, iy) is solid iff (ix-xc)^2 + (iy-yc)^2 <= r^2.

    Evaluated exactly in integers when 2xc, 2yc and 2r are integers (ties count as
    solid), otherwise in plain float64.
    """
    iy, ix = np.mgrid[0:ny, 0:nx]
    if all(float(2 * v).is_integer() for v in (xc, yc, r)):
        dx = 2 * ix.astype(np.int64) - int(2 * xc)
        dy = 2 * iy.astype(np.int64) - int(2 * yc)
        return ((dx * dx + dy * dy) <= int(2 * r) ** 2).astype(np.uint8)
    dx = ix.astype(np.float64) - xc
    dy = iy.astype(np.float64) - yc
    return ((dx * dx + dy * dy) <= r * r).astype(np.uint8)


def naca_half_thickness(xi: np.ndarray, chord: float, t: float = 0.12) -> np.ndarray:
    """Public NACA 4-digit symmetric thickness law (open trailing edge):
    y_t = 5 t c [0.2969 sqrt(s) - 0.1260 s - 0.3516 s^2 + 0.2843 s^3 - 0.1015 s^4],
    s = xi / c."""
    s = np.clip(xi / chord, 0.0, None)
    poly = (0.2969 * np.sqrt(s) - 0.1260 * s - 0.3516 * s * s + 0.2843 * s * s * s
            - 0.1015 * s * s * s * s)
    return 5.0 * t * chord * poly


def naca0012_mask(nx: int, ny: int, chord: float, xq: float, yq: float,
                  aoa_deg: float) -> np.ndarray:
    """uint8 [ny, nx] mask of a NACA0012 pivoted at its quarter chord (xq, yq).

    Body-frame coordinates of node (ix, iy), with X = ix - xq, Y = iy - yq:
    xi = c/4 + X cos(a) - Y sin(a), eta = X sin(a) + Y cos(a).  Solid iff
    0 <= xi <= c and |eta| <= y_t(xi).  Positive a is nose-up (leading edge raised).
    cos and sin are evaluated once on the host; everything else is IEEE +,-,*,/,sqrt.
    """
    a = aoa_deg * math.pi / 180.0
    ca, sa = math.cos(a), math.sin(a)
    iy, ix = np.mgrid[0:ny, 0:nx]
    X = ix.astype(np.float64) - xq
    Y = iy.astype(np.float64) - yq
    xi = chord / 4.0 + X * ca - Y * sa
    eta = X * sa + Y * ca
    inside = (xi >= 0.0) & (xi <= chord)
    yt = naca_half_thickness(np.where(inside, xi, 0.0), chord)
    return (inside & (np.abs(eta) <= yt)).astype(np.uint8)


def tau_from_re(u: float, length: float, re: float) -> float:
    """Lattice relaxation time tau_lb = 3 nu + 1/2 with nu = u L / Re."""
    return 3.0 * u * length / re + 0.5


def uniform_inlet(ny: int, u: float) -> np.ndarray:
    return np.full(ny, float(u), dtype=np.float64)


def default_box(mask: np.ndarray, margin: int) -> tuple[int, int, int, int]:
    """Control-volume box [x0, x1) x [y0, y1): the bounding box of the solid nodes grown
    by ``margin`` (at least 2) nodes on each side and clipped one node inside the
    domain."""
    ny, nx = mask.shape
    ys, xs = np.nonzero(mask)
    m = max(int(margin), 2)
    x0 = max(int(xs.min()) - m, 1)
    x1 = min(int(xs.max()) + 1 + m, nx - 1)
    y0 = max(int(ys.min()) - m, 1)
    y1 = min(int(ys.max()) + 1 + m, ny - 1)
    return (x0, x1, y0, y1)


def near_rest_state(nx: int, ny: int, seed: int, amp: float = 0.01,
                    dtype=np.float64) -> np.ndarray:
    """[9, ny, nx] field base_i * (1 + amp * xi), xi ~ U(-1, 1), seeded.  With
    dtype=float32 (or float16 deviations, see ``near_rest_state_fp16dev``) the values
    are rounded once, so every consumer reads exactly the same numbers."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(9, ny, nx))
    S = NEAR_REST_BASE[:, None, None] * (1.0 + amp * xi)
    return S.astype(dtype).astype(np.float64)


def near_rest_state_dev(nx: int, ny: int, seed: int, amp: float = 0.01,
                        dtype=np.float16) -> np.ndarray:
    """Like ``near_rest_state`` but every value is base_i + h with h representable in
    ``dtype``, so the field is exactly representable as deviations from the base."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(9, ny, nx))
    h = (NEAR_REST_BASE[:, None, None] * amp * xi).astype(dtype).astype(np.float64)
    return NEAR_REST_BASE[:, None, None] + h


def near_rest_state_fp16dev(nx: int, ny: int, seed: int, amp: float = 0.01) -> np.ndarray:
    return near_rest_state_dev(nx, ny, seed, amp, np.float16)


@dataclass
class Workload:
    """One synthetic run: geometry, boundary conditions and parameters."""
    name: str
    nx: int
    ny: int
    mask: np.ndarray
    tau: float
    uin: np.ndarray
    box: tuple | None
    steps: int
    u_ref: float
    l_ref: float
    bc_x: int = 0  # 0 inlet/outlet, 1 periodic
    bc_y: int = 0  # 0 no-slip walls, 1 periodic
    meta: dict = field(default_factory=dict)
    collision: str = "bgk"  # or "regularized"


def cylinder_channel_200x80() -> Workload:
    """Cylinder of diameter 20 centred at (40, 40) in a 200x80 channel with no-slip
    walls, uniform inlet 0.05 and zero-gradient outlet, Re 20, 5000 steps from rest,
    control volume 60x60 centred on the cylinder."""
    nx, ny, d, u, re = 200, 80, 20, 0.05, 20.0
    return Workload("cylinder_200x80_re20", nx, ny, cylinder_mask(nx, ny, 40, 40, d / 2),
                    tau_from_re(u, d, re), uniform_inlet(ny, u), (10, 70, 10, 70), 5000,
                    u, float(d), meta={"re": re, "d": d})


def naca_channel(nx: int, ny: int, chord: int, aoa: float, re: float, steps: int,
                 u: float = 0.05) -> Workload:
    """NACA0012 with its leading edge at nx/4 (at zero incidence), quarter-chord pivot
    on row ny/2, uniform inlet, walls, control volume = body box + chord/4."""
    xq, yq = nx // 4 + chord // 4, ny // 2
    mask = naca0012_mask(nx, ny, chord, xq, yq, aoa)
    box = default_box(mask, chord // 4)
    return Workload(f"naca0012_{nx}x{ny}_c{chord}_a{aoa:g}_re{re:g}", nx, ny, mask,
                    tau_from_re(u, chord, re), uniform_inlet(ny, u), box, steps, u,
                    float(chord), meta={"re": re, "chord": chord, "aoa": aoa,
                                        "xq": xq, "yq": yq})


def naca_2048x1024(aoa: float = 4.0, re: float = 1000.0) -> Workload:
    return naca_channel(2048, 1024, 256, aoa, re, 20000)


def naca_8192x4096(aoa: float = 4.0, re: float = 1e4) -> Workload:
    return naca_channel(8192, 4096, 1024, aoa, re, 50000)


def naca_1024x512_adjoint() -> Workload:
    return naca_channel(1024, 512, 256, 0.0, 500.0, 10000)


BATCH_SEED = 2210_10377


def batched_instances(n: int = 256, seed: int = BATCH_SEED, u: float = 0.05,
                      steps: int = 10000) -> list[Workload]:
    """``n`` independent channel problems of uneven size, drawn from
    ``numpy.random.default_rng(seed)``; per instance, in this order: width
    W ~ U{64..512} (height H = W // 2), body type (cylinder if U(0,1) < 1/2, else
    NACA0012), angle of attack ~ U(0, 10) degrees (drawn for every instance, used by
    airfoils), Re ~ U(20, 2000).

    Cylinder: diameter D = 0.2 H centred at (0.25 W, 0.5 H), Re on D, control volume the
    body box grown by D/4 (1.5 D across).  Airfoil: chord c = W // 4 with its leading
    edge at W // 4 at zero incidence, pivot at the quarter chord on row H // 2, Re on
    c, control volume the body box grown by c/4.  Uniform inlet u, walls, outlet."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W = int(rng.integers(64, 513))
        H = W // 2
        cyl = bool(rng.random() < 0.5)
        aoa = float(rng.uniform(0.0, 10.0))
        re = float(rng.uniform(20.0, 2000.0))
        if cyl:
            d = 0.2 * H
            mask = cylinder_mask(W, H, 0.25 * W, 0.5 * H, d / 2.0)
            box = default_box(mask, max(2, int(round(d / 4.0))))
            out.append(Workload(f"b{i:03d}_cyl_{W}x{H}_re{re:.0f}", W, H, mask,
                                tau_from_re(u, d, re), uniform_inlet(H, u), box, steps, u,
                                d, meta={"type": "cylinder", "re": re, "d": d}))
        else:
            chord = W // 4
            xq, yq = W // 4 + chord // 4, H // 2
            mask = naca0012_mask(W, H, chord, xq, yq, aoa)
            box = default_box(mask, max(2, chord // 4))
            out.append(Workload(f"b{i:03d}_naca_{W}x{H}_a{aoa:.1f}_re{re:.0f}", W, H, mask,
                                tau_from_re(u, chord, re), uniform_inlet(H, u), box, steps,
                                u, float(chord), meta={"type": "naca0012", "re": re,
                                                       "aoa": aoa, "chord": chord}))
    return out
