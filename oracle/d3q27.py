"""TEST INFRASTRUCTURE ONLY -- Python access to the three-dimensional oracle
(``lbm3d_oracle.cpp``: the D3Q27 BGK step with half-way bounce-back and the per-step
forces A, B, DRTT and SI of arXiv:2210.10377 carried to three dimensions)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import LIB3, build

BCX_INLET_OUTLET, BCX_PERIODIC = 0, 1
BC_WALL, BC_PERIODIC = 0, 1


class _Cfg3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("bc_z", ctypes.c_int32),
                ("box", ctypes.c_int32 * 6), ("rho_w", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("collision", ctypes.c_int32),
                ("body_u", ctypes.c_double * 3), ("body_omega", ctypes.c_double * 3),
                ("body_c", ctypes.c_double * 3)]


COLLISIONS = {"bgk": 0, "regularized": 1}


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB3)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        cp = ctypes.POINTER(_Cfg3)
        L.orc3_lattice.argtypes = [ip, ip, ip, ip, dp]
        L.orc3_equilibrium.argtypes = [ctypes.c_double] * 4 + [dp]
        L.orc3_collide_node.argtypes = [dp] + [ctypes.c_double] * 4 + [dp]
        L.orc3_collide_node_regularized.argtypes = [dp, ctypes.c_double, dp]
        L.orc3_box_admissible.argtypes = [cp, u8]
        L.orc3_box_admissible.restype = ctypes.c_int
        L.orc3_links.argtypes = [cp, u8, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]
        L.orc3_links.restype = ctypes.c_int64
        L.orc3_create.argtypes = [cp, u8, ctypes.c_double, dp]
        L.orc3_create.restype = ctypes.c_void_p
        L.orc3_destroy.argtypes = [ctypes.c_void_p]
        for name in ("orc3_set_state", "orc3_get_state", "orc3_get_pre", "orc3_records",
                     "orc3_forces"):
            getattr(L, name).argtypes = [ctypes.c_void_p, dp]
        L.orc3_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc3_nrec.argtypes = [ctypes.c_void_p]
        L.orc3_nrec.restype = ctypes.c_int64
        L.orc3_momentum_of.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc3_set_mask.argtypes = [ctypes.c_void_p, u8, ctypes.POINTER(ctypes.c_int32), dp]
        L.orc3_set_mask.restype = ctypes.c_int
        L.orc3_set_body_motion.argtypes = [ctypes.c_void_p, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cfg(shape, bc_x, bc_y, bc_z, box, rho_w, g, collision="bgk", body_motion=None):
    nz, ny, nx = shape
    c = _Cfg3()
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.bc_x, c.bc_y, c.bc_z = int(bc_x), int(bc_y), int(bc_z)
    b = (-1,) * 6 if box is None else tuple(int(v) for v in box)
    for k in range(6):
        c.box[k] = b[k]
    c.rho_w = float(rho_w)
    for k in range(3):
        c.g[k] = float(g[k])
    c.collision = COLLISIONS[collision]
    if body_motion is not None:
        U, W, X = body_motion
        for k in range(3):
            c.body_u[k], c.body_omega[k], c.body_c[k] = float(U[k]), float(W[k]), float(X[k])
    return c


def _mask(mask):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def lattice():
    """(cx, cy, cz, opp, w) of the 27 directions."""
    cx, cy, cz, opp = (np.zeros(27, np.int32) for _ in range(4))
    w = np.zeros(27)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib().orc3_lattice(cx.ctypes.data_as(ip), cy.ctypes.data_as(ip), cz.ctypes.data_as(ip),
                       opp.ctypes.data_as(ip), _dp(w))
    return cx, cy, cz, opp, w


def equilibrium(rho, ux, uy, uz):
    out = np.zeros(27)
    lib().orc3_equilibrium(float(rho), float(ux), float(uy), float(uz), _dp(out))
    return out


def collide_node(f, omega, g=(0.0, 0.0, 0.0), collision="bgk"):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(27)
    if collision == "regularized":
        if any(g):
            raise ValueError("only the BGK collision takes a body force")
        lib().orc3_collide_node_regularized(_dp(f), float(omega), _dp(out))
    else:
        lib().orc3_collide_node(_dp(f), float(omega), float(g[0]), float(g[1]), float(g[2]),
                                _dp(out))
    return out


def box_admissible(mask, box, bc_x=BCX_INLET_OUTLET, bc_y=BC_WALL, bc_z=BC_WALL):
    m, mp = _mask(mask)
    c = _cfg(m.shape, bc_x, bc_y, bc_z, box, 1.0, (0, 0, 0))
    return bool(lib().orc3_box_admissible(ctypes.byref(c), mp))


def links(mask, bc_x=BCX_INLET_OUTLET, bc_y=BC_WALL, bc_z=BC_WALL):
    """Body links [(node, direction)] in (z, y, x, direction) order, int64 (L, 2)."""
    m, mp = _mask(mask)
    c = _cfg(m.shape, bc_x, bc_y, bc_z, None, 1.0, (0, 0, 0))
    n = lib().orc3_links(ctypes.byref(c), mp, None, 0)
    out = np.zeros((max(n, 1), 2), np.int64)
    lib().orc3_links(ctypes.byref(c), mp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n)
    return out[:n]


class OracleSim3:
    """FP64 reference simulation on a [nz, ny, nx] lattice.  ``uin`` is the inlet
    x-velocity, broadcast to [nz, ny]; ``box`` = (x0, x1, y0, y1, z0, z1); ``collision``
    "bgk" (Eq. CollideAdv) or "regularized"; ``body_motion`` = (U, Omega, centre), three
    3-vectors: rigid motion of the body."""

    def __init__(self, mask, tau=None, uin=None, bc_x=BCX_INLET_OUTLET, bc_y=BC_WALL,
                 bc_z=BC_WALL, box=None, rho_w=1.0, g=(0.0, 0.0, 0.0), omega=None,
                 collision="bgk", body_motion=None):
        m, mp = _mask(mask)
        self.nz, self.ny, self.nx = m.shape
        self.omega = float(omega) if omega is not None else 1.0 / float(tau)
        self.box = box
        self._cfg = _cfg(m.shape, bc_x, bc_y, bc_z, box, rho_w, g, collision, body_motion)
        u = None
        if uin is not None:
            self._uin = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64),
                                                             (self.nz, self.ny)))
            u = _dp(self._uin)
        self._h = lib().orc3_create(ctypes.byref(self._cfg), mp, self.omega, u)
        if not self._h:
            raise ValueError("oracle rejected the configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc3_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (27, self.nz, self.ny, self.nx)

    def set_state(self, S):
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(self.shape)
        lib().orc3_set_state(self._h, _dp(S))

    def state(self):
        out = np.zeros(self.shape)
        lib().orc3_get_state(self._h, _dp(out))
        return out

    def pre(self):
        out = np.zeros(self.shape)
        lib().orc3_get_pre(self._h, _dp(out))
        return out

    def step(self, n=1):
        lib().orc3_step(self._h, int(n))

    def records(self):
        """[t][FA(3), FB(3), J(3), Phi(3), SI(3)] of every recorded step."""
        n = lib().orc3_nrec(self._h)
        out = np.zeros((n, 15))
        if n:
            lib().orc3_records(self._h, _dp(out))
        return out

    def forces(self):
        """[t, scheme (A, B, DRTT, SI), component (x, y, z)]."""
        n = lib().orc3_nrec(self._h)
        out = np.zeros((n, 4, 3))
        if n:
            lib().orc3_forces(self._h, _dp(out))
        return out

    def set_mask(self, mask, box=None):
        """Move the body through the grid: a new mask (and box, if given) from the next
        step; uncovered nodes refilled at the wall velocity; returns the impulse (3,)."""
        m, mp = _mask(mask)
        if m.shape != (self.nz, self.ny, self.nx):
            raise ValueError("mask shape differs from the lattice")
        bp = None
        if box is not None:
            self._box_arr = (ctypes.c_int32 * 6)(*[int(v) for v in box])
            bp = ctypes.cast(self._box_arr, ctypes.POINTER(ctypes.c_int32))
        imp = np.zeros(3)
        if lib().orc3_set_mask(self._h, mp, bp, _dp(imp)) != 0:
            raise ValueError("mask or control volume not admissible")
        self._mask_keep = m
        return imp

    def set_body_motion(self, u=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0), centre=(0.0, 0.0, 0.0)):
        vs = [np.ascontiguousarray(np.asarray(v, np.float64).reshape(3)) for v in (u, omega, centre)]
        self._motion_keep = vs
        lib().orc3_set_body_motion(self._h, *[_dp(v) for v in vs])

    def momentum_of(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.shape)
        J = np.zeros(3)
        lib().orc3_momentum_of(self._h, _dp(g), _dp(J))
        return J
