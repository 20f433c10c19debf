"""TEST INFRASTRUCTURE ONLY -- Python access to the oracle.

The oracle is a plain FP64 C++ reference (``lbm_oracle.cpp``) of the D2Q9 BGK step with
half-way bounce-back and the per-step forces of Kaushal, Succi & Ansumali,
arXiv:2210.10377 (Sec. II-IV and the Appendix).  Only ``tests/``, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the product package
never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

BCX_INLET_OUTLET, BCX_PERIODIC = 0, 1
BCY_WALL, BCY_PERIODIC = 0, 1


SRC3 = os.path.join(HERE, "lbm3d_oracle.cpp")
LIB3 = os.path.join(HERE, "liboracle3d.so")


def _compile(src, lib, force):
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-fopenmp",
                               "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, lib)
    return lib


def build(force: bool = True) -> str:
    """Compile the oracles (two- and three-dimensional) with g++, no FMA contraction,
    so that they are plain IEEE."""
    _compile(SRC3, LIB3, force)
    return _compile(SRC, LIB, force)


class _Cfg(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc_x", ctypes.c_int32),
                ("bc_y", ctypes.c_int32), ("box", ctypes.c_int32 * 4),
                ("rho_w", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("collision", ctypes.c_int32), ("body_u", ctypes.c_double * 2),
                ("body_omega", ctypes.c_double), ("body_c", ctypes.c_double * 2)]

COLLISIONS = {"bgk": 0, "regularized": 1, "kbc": 2}


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        cp = ctypes.POINTER(_Cfg)
        L.orc_lattice.argtypes = [ip, ip, ip, dp, dp]
        L.orc_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_collide_node.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_collide_node_regularized.argtypes = [dp, ctypes.c_double, dp]
        L.orc_collide_node_kbc.argtypes = [dp, ctypes.c_double, dp]
        L.orc_box_admissible.argtypes = [cp, u8]
        L.orc_box_admissible.restype = ctypes.c_int
        L.orc_links.argtypes = [cp, u8, ip, ctypes.c_int64]
        L.orc_links.restype = ctypes.c_int64
        L.orc_create.argtypes = [cp, u8, ctypes.c_double, dp]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        for name in ("orc_set_state", "orc_get_state", "orc_get_pre", "orc_records",
                     "orc_forces"):
            getattr(L, name).argtypes = [ctypes.c_void_p, dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc_nrec.argtypes = [ctypes.c_void_p]
        L.orc_nrec.restype = ctypes.c_int64
        L.orc_clear_records.argtypes = [ctypes.c_void_p]
        L.orc_set_mask.argtypes = [ctypes.c_void_p, u8, ctypes.POINTER(ctypes.c_int32), dp]
        L.orc_set_mask.restype = ctypes.c_int
        L.orc_set_body_motion.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 5
        L.orc_momentum_of.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_objective_cs.argtypes = [cp, u8, ctypes.c_double, ctypes.c_double, dp, dp,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, dp]
        L.orc_objective_cs.restype = ctypes.c_int
        L.orc_boundary_cp.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_double, ip, dp, ctypes.c_int64]
        L.orc_boundary_cp.restype = ctypes.c_int64
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_set_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> int:
    """Threads of the two-dimensional oracle's row loops (1: serial, the default).  Every
    sum keeps its serial order, so results are bitwise the same for any count.  Returns
    the previous count."""
    return int(lib().orc_set_threads(int(n)))


def _cfg(nx, ny, bc_x, bc_y, box, rho_w, g, collision="bgk", body_motion=None):
    c = _Cfg()
    c.collision = COLLISIONS[collision]
    if body_motion is not None:
        ux, uy, om, xc, yc = (float(v) for v in body_motion)
        c.body_u[0], c.body_u[1], c.body_omega, c.body_c[0], c.body_c[1] = ux, uy, om, xc, yc
    c.nx, c.ny, c.bc_x, c.bc_y = int(nx), int(ny), int(bc_x), int(bc_y)
    b = (-1, -1, -1, -1) if box is None else tuple(int(v) for v in box)
    for k in range(4):
        c.box[k] = b[k]
    c.rho_w = float(rho_w)
    c.gx, c.gy = float(g[0]), float(g[1])
    return c


def lattice():
    """(cx, cy, opp, w, theta0) as the oracle holds them."""
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    opp = np.zeros(9, np.int32)
    w = np.zeros(9)
    th = np.zeros(1)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib().orc_lattice(cx.ctypes.data_as(ip), cy.ctypes.data_as(ip), opp.ctypes.data_as(ip),
                      _dp(w), _dp(th))
    return cx, cy, opp, w, float(th[0])


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_equilibrium(float(rho), float(ux), float(uy), _dp(out))
    return out


def collide_node(f, omega, g=(0.0, 0.0), collision="bgk"):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    if collision in ("regularized", "kbc"):
        if g[0] or g[1]:
            raise ValueError("only the BGK collision takes a body force")
        fn = lib().orc_collide_node_regularized if collision == "regularized" else lib().orc_collide_node_kbc
        fn(_dp(f), float(omega), _dp(out))
    else:
        lib().orc_collide_node(_dp(f), float(omega), float(g[0]), float(g[1]), _dp(out))
    return out


def _mask(mask):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def box_admissible(mask, box, bc_x=BCX_INLET_OUTLET, bc_y=BCY_WALL):
    m, mp = _mask(mask)
    ny, nx = m.shape
    c = _cfg(nx, ny, bc_x, bc_y, box, 1.0, (0.0, 0.0))
    return bool(lib().orc_box_admissible(ctypes.byref(c), mp))


def links(mask, bc_x=BCX_INLET_OUTLET, bc_y=BCY_WALL):
    """Canonical fluid-solid links as an int32 array [L, 2] of (y*nx + x, i)."""
    m, mp = _mask(mask)
    ny, nx = m.shape
    c = _cfg(nx, ny, bc_x, bc_y, None, 1.0, (0.0, 0.0))
    n = lib().orc_links(ctypes.byref(c), mp, None, 0)
    if n < 0:
        raise ValueError("invalid configuration")
    out = np.zeros((max(n, 1), 2), np.int32)
    lib().orc_links(ctypes.byref(c), mp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n)
    return out[:n]


class OracleSim:
    """FP64 reference simulation.  ``tau`` is the lattice relaxation time tau_lb
    (omega = 1/tau_lb); pass ``omega`` directly for the pure-streaming fixture
    (omega = 0).  ``collision`` is "bgk" (Eq. CollideAdv), "regularized" or "kbc" (the
    stated variants for tau_lb close to 1/2).  ``body_motion`` = (ux, uy, Omega, xc, yc):
    rigid motion of the body (translation, rotation rate about (xc, yc))."""

    def __init__(self, mask, tau=None, uin=None, bc_x=BCX_INLET_OUTLET, bc_y=BCY_WALL,
                 box=None, rho_w=1.0, g=(0.0, 0.0), omega=None, collision="bgk",
                 body_motion=None):
        m, mp = _mask(mask)
        self.ny, self.nx = m.shape
        if omega is None:
            omega = 1.0 / float(tau)
        self.omega = float(omega)
        self.box = box
        self._cfg = _cfg(self.nx, self.ny, bc_x, bc_y, box, rho_w, g, collision, body_motion)
        u = None
        if uin is not None:
            self._uin = np.ascontiguousarray(np.broadcast_to(np.asarray(uin, np.float64),
                                                             (self.ny,)))
            u = _dp(self._uin)
        self._h = lib().orc_create(ctypes.byref(self._cfg), mp, self.omega, u)
        if not self._h:
            raise ValueError("oracle rejected the configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (9, self.ny, self.nx)

    def set_state(self, S):
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(self.shape)
        lib().orc_set_state(self._h, _dp(S))

    def state(self):
        out = np.zeros(self.shape)
        lib().orc_get_state(self._h, _dp(out))
        return out

    def pre(self):
        out = np.zeros(self.shape)
        lib().orc_get_pre(self._h, _dp(out))
        return out

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def records(self):
        """[t][FAx, FAy, FBx, FBy, Jx, Jy, Phix, Phiy, SIx, SIy, Jpostx, Jposty] of every
        recorded step (J before collision, Jpost after it)."""
        n = lib().orc_nrec(self._h)
        out = np.zeros((n, 12))
        if n:
            lib().orc_records(self._h, _dp(out))
        return out

    def forces(self):
        """[t, scheme (A, B, DRTT, SI, DRTT-post), component (x, y)] of every recorded
        step; DRTT-post takes the control-volume momentum J(t) after the collision."""
        n = lib().orc_nrec(self._h)
        out = np.zeros((n, 5, 2))
        if n:
            lib().orc_forces(self._h, _dp(out))
        return out

    def clear_records(self):
        lib().orc_clear_records(self._h)

    def set_mask(self, mask, box=None):
        """Move the body: a new mask (and control volume, if given) from the next step.
        Uncovered nodes are refilled with f^eq(mean neighbour density, wall velocity);
        returns the impulse handed from the fluid to the body, (2,)."""
        m, mp = _mask(mask)
        if m.shape != (self.ny, self.nx):
            raise ValueError("mask shape differs from the lattice")
        bp = None
        if box is not None:
            self._box_arr = (ctypes.c_int32 * 4)(*[int(v) for v in box])
            bp = ctypes.cast(self._box_arr, ctypes.POINTER(ctypes.c_int32))
        imp = np.zeros(2)
        if lib().orc_set_mask(self._h, mp, bp, _dp(imp)) != 0:
            raise ValueError("mask or control volume not admissible")
        self._mask_keep = m
        if box is not None:
            self.box = tuple(int(v) for v in box)
        return imp

    def set_body_motion(self, ux=0.0, uy=0.0, omega=0.0, xc=0.0, yc=0.0):
        """Rigid motion of the body from the next step."""
        lib().orc_set_body_motion(self._h, float(ux), float(uy), float(omega), float(xc),
                                  float(yc))

    def boundary_cp(self, ref=None, rho_ref=1.0, u_ref=1.0):
        """Pressure coefficient (p - p_inf) / (rho_ref u_ref^2 / 2) at every boundary fluid
        node (row-major order), p = rho theta0 of the stored state; p_inf at the
        reference node ref = (x, y), or rho_ref theta0 when ref is None.  Returns
        (node indices y*nx + x as int32 [n], C_p float64 [n])."""
        x, y = (-1, -1) if ref is None else (int(ref[0]), int(ref[1]))
        ip = ctypes.POINTER(ctypes.c_int32)
        n = lib().orc_boundary_cp(self._h, x, y, float(rho_ref), float(u_ref), None, None, 0)
        if n < 0:
            raise ValueError("reference node outside the grid or solid")
        nodes = np.zeros(max(n, 1), np.int32)
        cp = np.zeros(max(n, 1))
        lib().orc_boundary_cp(self._h, x, y, float(rho_ref), float(u_ref),
                              nodes.ctypes.data_as(ip), _dp(cp), n)
        return nodes[:n], cp[:n]

    def momentum_of(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.shape)
        J = np.zeros(2)
        lib().orc_momentum_of(self._h, _dp(g), _dp(J))
        return J


def objective(mask, omega, uin, nsteps, t0, T, w=(1.0, 0.0), bc_x=BCX_INLET_OUTLET,
              bc_y=BCY_WALL, rho_w=1.0):
    """J = (1/T) sum_{t0 <= t < t0+T} w . F_B(t) of a run from rest, evaluated in complex
    arithmetic: ``omega`` and ``uin`` may be complex (complex-step derivatives).
    Returns a complex number."""
    m, mp = _mask(mask)
    ny, nx = m.shape
    c = _cfg(nx, ny, bc_x, bc_y, None, rho_w, (0.0, 0.0))
    om = complex(omega)
    u = np.asarray(uin, dtype=np.complex128)
    ure = np.ascontiguousarray(u.real)
    uim = np.ascontiguousarray(u.imag)
    out = np.zeros(2)
    rc = lib().orc_objective_cs(ctypes.byref(c), mp, om.real, om.imag, _dp(ure), _dp(uim),
                                int(nsteps), int(t0), int(T), float(w[0]), float(w[1]),
                                _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the configuration")
    return complex(out[0], out[1])

