"""Writes the oracle fixtures of the full-size workloads (expected values for GPU tests).

Calls only ``oracle/`` (the FP64 reference) and ``workloads/`` (geometry and inputs);
nothing here comes from the HIP library.  Run from the repository root:

    python tests/golden/make_fixtures.py [--threads N] [--only NAME ...]

Fixtures (numpy ``.npz``, plain arrays, loadable with ``allow_pickle=False``):

* ``naca2048x1024_a4_re100.npz``, ``naca2048x1024_a4_re1000.npz`` -- the NACA0012
  channel of the precision study (2048x1024, chord 256, quarter chord at (576, 512),
  angle of attack 4 degrees, uniform inlet 0.05, walls, outlet, control volume the body
  box grown by a quarter chord), 20 000 steps from rest:
    ``steps`` [K] and ``forces`` [K, 5, 2]: the oracle's forces (A, B, DRTT, SI,
    DRTT-post; x, y) at every 10th step before step 18 000 and at every step of the last
    2000; ``window_mean`` [5, 2]: their mean over the last 2000 steps;
    ``sample_y``, ``sample_x`` [M]: fluid nodes on a 16-node lattice (offset 8);
    ``rho``, ``ux``, ``uy`` [M]: density and velocity there after the last step.
* ``naca1024x512_adjoint.npz`` -- the adjoint workload (1024x512, chord 256, zero
  incidence, Re 500, 10 000 steps from rest, J = mean algorithm-B drag over steps
  8000..9999): ``J``, the complex-step derivatives ``dJ_dtau`` and ``dJ_dv`` [2] in the
  unit inlet directions ``v`` [2, 512] (normal deviates from
  ``numpy.random.default_rng(500)``, normalised), step ``h`` = 1e-30.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
STRIDE, OFFSET = 16, 8
WINDOW = 2000


def naca2048(re: float, path: str) -> None:
    w = workloads.naca_2048x1024(aoa=4.0, re=re)
    o = oracle.OracleSim(w.mask, tau=w.tau, uin=w.uin, box=w.box)
    n = w.steps
    t0 = time.time()
    chunk = 1000
    F = []
    for k in range(0, n, chunk):
        o.step(min(chunk, n - k))
        F.append(o.forces())
        o.clear_records()
        print(f"{os.path.basename(path)}: {k + chunk} / {n} steps, {time.time() - t0:.0f} s",
              flush=True)
    F = np.concatenate(F)
    steps = np.array([t for t in range(n) if t >= n - WINDOW or t % 10 == 0], np.int64)
    S = o.state()
    ys, xs = np.meshgrid(np.arange(OFFSET, w.ny, STRIDE), np.arange(OFFSET, w.nx, STRIDE),
                         indexing="ij")
    ys, xs = ys.ravel(), xs.ravel()
    fl = w.mask[ys, xs] == 0
    ys, xs = ys[fl], xs[fl]
    P = S[:, ys, xs]
    rho = P.sum(0)
    ux = np.tensordot(CX, P, 1) / rho
    uy = np.tensordot(CY, P, 1) / rho
    np.savez_compressed(path, steps=steps, forces=F[steps], window_mean=F[n - WINDOW:].mean(0),
                        sample_y=ys.astype(np.int32), sample_x=xs.astype(np.int32), rho=rho,
                        ux=ux, uy=uy, tau=np.float64(w.tau), aoa=np.float64(4.0),
                        re=np.float64(re), n_steps=np.int64(n))


def adjoint1024(path: str) -> None:
    w = workloads.naca_1024x512_adjoint()
    n, t0, T = 10000, 8000, 2000
    h = 1e-30
    rng = np.random.default_rng(500)
    v = np.zeros((2, w.ny))
    for k in range(2):
        d = rng.normal(size=w.ny)
        v[k] = d / np.linalg.norm(d)
    start = time.time()
    Jt = oracle.objective(w.mask, 1.0 / complex(w.tau, h), w.uin, n, t0, T)
    print(f"{os.path.basename(path)}: tau done, {time.time() - start:.0f} s", flush=True)
    dv = []
    for k in range(2):
        Jv = oracle.objective(w.mask, 1.0 / w.tau, w.uin + 1j * h * v[k], n, t0, T)
        dv.append(Jv.imag / h)
        print(f"{os.path.basename(path)}: direction {k} done, {time.time() - start:.0f} s",
              flush=True)
    np.savez_compressed(path, J=np.float64(Jt.real), dJ_dtau=np.float64(Jt.imag / h),
                        dJ_dv=np.array(dv), v=v, h=np.float64(h), tau=np.float64(w.tau),
                        n_steps=np.int64(n), t0=np.int64(t0), T=np.int64(T))


FIXTURES = {
    "naca2048x1024_a4_re100": lambda p: naca2048(100.0, p),
    "naca2048x1024_a4_re1000": lambda p: naca2048(1000.0, p),
    "naca1024x512_adjoint": adjoint1024,
}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None, choices=sorted(FIXTURES))
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    for name in args.only or FIXTURES:
        FIXTURES[name](os.path.join(HERE, name + ".npz"))


if __name__ == "__main__":
    main()
