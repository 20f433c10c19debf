#!/usr/bin/env python3
"""Throughput of the fused D2Q9 step with per-step forces on one MI355X.

Workload (default): NACA0012 from the analytic 4-digit thickness law, chord 1024, angle
of attack 4 deg, in an 8192 x 4096 channel (33.5 M nodes) with no-slip walls, uniform
inlet 0.05 and zero-gradient outlet, Re 1e4 (tau_lb from nu = U c / Re), FP32 population
storage, forces by momentum exchange A and B, by DRTT and by stress integration at every
step.  Synthetic input (analytic geometry, flow started from rest).

One "step" is one lattice time step of the whole grid including the four force
estimators.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS incl. per-step force + HBM GB/s % peak; adjoint MLUPS; Cd rel err vs FP64"
HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"fp64": 144, "fp32": 72, "fp32dev": 72, "fp32sr": 72, "fp16dev": 36}
CSRC = os.path.join(ROOT, "paper_2210_10377_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
BATCH_WORKLOAD = "batched_256_cylinder_naca0012_64x32_to_512x256"


SOURCES_3D = ("api3.hip", "kernels3.h", "kernels3.hip", "plan3.cpp", "plan3.h")


def kernel_hash(three_d: bool = False) -> str:
    """sha256 over the library sources of one path (kernels, launch layout and plan):
    the three-dimensional files, or all the others; the public headers included."""
    h = hashlib.sha256()
    names = [n for n in sorted(os.listdir(CSRC)) if (n in SOURCES_3D) == three_d]
    files = [os.path.join(CSRC, n) for n in names]
    files.append(os.path.join(ROOT, "include", "lbm3d.h" if three_d else "lbm.h"))
    for path in files:
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, three_d: bool = False):
    """HBM bytes per step from the committed rocprofv3 counter summary, or None when the
    path's sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get(f"{workload}/{precision}")
    if not rec or rec.get("sources_sha256") != kernel_hash(three_d):
        return None
    return rec["hbm_bytes_per_launch"]


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle may use: the CPUs this process may run on, at most 16 (the
    host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(w, steps: int, collision: str = "bgk", body_motion=None):
    """The oracle (plain FP64 C++) on a bounded sample of the same workload: `steps`
    full-grid time steps with all five force estimators, from the same initial state,
    once on one thread and once on every available host thread (row loops in parallel;
    the sums keep their serial order, so both give bitwise the same numbers).  `value` is
    the all-thread rate; the one-thread rate is reported beside it."""
    import oracle

    def run(threads):
        oracle.set_threads(threads)
        o = oracle.OracleSim(w.mask, tau=w.tau, uin=w.uin, box=w.box, collision=collision,
                             body_motion=body_motion)
        t0 = time.perf_counter()
        o.step(steps)
        o.forces()
        dt = time.perf_counter() - t0
        del o
        return dt

    n = host_threads()
    dt1 = run(1)
    dtn = run(n) if n > 1 else dt1
    oracle.set_threads(1)
    rate = lambda dt: round(w.nx * w.ny * steps / dt / 1e6, 3)
    return {"value": rate(dtn), "unit": "MLUPS", "cores": n, "kind": "oracle",
            "one_core_value": rate(dt1), "cpu_model": host_cpu_model(),
            "sample": f"{steps} full-grid steps of {w.nx}x{w.ny} from rest with the A, B, "
                      f"DRTT, SI and DRTT-post forces, FP64 ({dtn:.1f} s on {n} threads, "
                      f"{dt1:.1f} s on one)"}


def sensitivity_study(steps: int, seeds: int, every: int = 0, frozen: bool = False):
    """How far the FP64 path itself moves when perturbed by noise of the size of binary32
    rounding: the 2048x1024 NACA0012 channel (AoA 4, Re 100 and 1000) from rest; every
    population is multiplied by (1 + a xi), xi ~ U(-1, 1) seeded, once at step 100 with
    a = 2^-24 (every = 0), or at every `every`-th step with a = 2^-24 sqrt(every) (the
    accumulated size of independent per-step rounding, as a 32-bit run rounds every
    step), or with `frozen` the same pattern xi every time with a = 2^-24 every (a
    rounding error that recurs with the same sign at each node every step, as at the
    nodes of a steady flow); the window-mean (last 2000 steps) force coefficients of each
    perturbed twin against the unperturbed run.  One JSON line per Reynolds number."""
    import numpy as np

    import workloads
    from paper_2210_10377_amd import Sim

    names = ("A", "B", "DRTT", "SI", "DRTT_POST")
    for re in (100.0, 1000.0):
        w = workloads.naca_2048x1024(aoa=4.0, re=re)

        def run(seed):
            sim = Sim(w.mask, w.tau, w.uin, precision="fp64", box=w.box, max_record=steps,
                      u_ref=w.u_ref, l_ref=w.l_ref)
            rng = np.random.default_rng(seed)
            done, F = 0, []
            marks = [100] if every == 0 else list(range(every, steps, every))
            amp = 2.0 ** -24 * (1.0 if every == 0 else (every if frozen else np.sqrt(every)))
            xi0 = None
            for m in marks + [steps]:
                sim.step(m - done)
                F.append(sim.forces())
                done = m
                if seed is not None and m < steps:
                    S = sim.populations()
                    if xi0 is None or not frozen:
                        xi0 = rng.uniform(-1.0, 1.0, S.shape)
                    sim.set_populations(S * (1.0 + amp * xi0))
            C = sim.coefficients(np.concatenate(F))
            return C[-2000:].mean(0)

        base = run(None)
        errs = np.array([np.abs(run(k) - base) / np.abs(base) for k in range(seeds)])
        out = {"sensitivity": w.name, "storage": "fp64",
               "perturbation": ("relative 2^-24 at step 100" if every == 0 else
                                (f"one pattern, relative 2^-24 x {every}, every {every} steps"
                                 if frozen else
                                 f"relative 2^-24 sqrt({every}) every {every} steps")),
               "steps": steps, "twins": seeds,
               "cd_window_mean": dict(zip(names, base[:, 0].round(6).tolist())),
               "cl_window_mean": dict(zip(names, base[:, 1].round(6).tolist())),
               "cd_rel_change_max": dict(zip(names, errs[:, :, 0].max(0).tolist())),
               "cl_rel_change_max": dict(zip(names, errs[:, :, 1].max(0).tolist()))}
        print(json.dumps(out), flush=True)


def uniform_flow_state(w):
    """[9, ny, nx] equilibrium populations of density 1 and velocity (u_in(y), 0) at every
    node (the second-order equilibrium with weights 4/9, 1/9, 1/36)."""
    import numpy as np
    wts = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    u = np.asarray(w.uin, np.float64)[None, :]
    cu = cx[:, None] * u
    feq_y = wts[:, None] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u * u)   # [9, ny]
    return np.ascontiguousarray(np.broadcast_to(feq_y[:, :, None], (9, w.ny, w.nx)))


def precision_study(steps: int):
    """The 32-bit storages (binary32 populations rounded to nearest, binary32 deviations,
    binary32 populations rounded stochastically) and FP16-deviation storage against FP64
    storage (itself matched to the oracle to 1e-10) on the 2048x1024 NACA0012 channel.  Coefficient errors are relative
    to the largest FP64 coefficient magnitude of the run (per step) and to the FP64 mean
    over the last 2000 steps (window means); velocity errors are relative to the inlet
    speed."""
    import numpy as np

    import workloads
    from paper_2210_10377_amd import Sim

    def velocity(S):
        cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
        cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
        rho = S.sum(0)
        return np.tensordot(cx, S, 1) / rho, np.tensordot(cy, S, 1) / rho

    for aoa in (0.0, 4.0, 8.0):
        for re in (100.0, 1000.0):
            w = workloads.naca_2048x1024(aoa=aoa, re=re)
            runs = {}
            for prec in ("fp64", "fp32", "fp32dev", "fp32sr", "fp16dev"):
                sim = Sim(w.mask, w.tau, w.uin, precision=prec, box=w.box, max_record=5000,
                          u_ref=w.u_ref, l_ref=w.l_ref)
                t0 = time.perf_counter()
                F = sim.run(steps)
                C = sim.coefficients(F)
                runs[prec] = (C, velocity(sim.populations()), time.perf_counter() - t0)
                del sim
            C64, (u64, v64), _ = runs["fp64"]
            fl = w.mask == 0
            names = ("A", "B", "DRTT", "SI", "DRTT_POST")
            out = {"case": w.name, "steps": steps, "tau": w.tau,
                   "fp64_window_mean": {s: C64[-2000:, k].mean(0).tolist()
                                        for k, s in enumerate(names)}}
            for prec in ("fp32", "fp32dev", "fp32sr", "fp16dev"):
                C, (u, v), wall = runs[prec]
                e = {}
                for k, s in enumerate(names):
                    scale = np.abs(C64[:, k]).max(0)
                    e[s] = {"step_max_rel_cd_cl": (np.abs(C[:, k] - C64[:, k]).max(0) / scale).tolist(),
                            "window_mean_rel_cd_cl": (np.abs(C[-2000:, k].mean(0) - C64[-2000:, k].mean(0))
                                                      / np.abs(C64[-2000:, k].mean(0))).tolist()}
                du = np.hypot(u - u64, v - v64)[fl]
                e["velocity_linf_over_U"] = float(du.max() / w.u_ref)
                e["velocity_l2_rel"] = float(np.sqrt((du ** 2).sum() / (u64[fl] ** 2 + v64[fl] ** 2).sum()))
                e["finite"] = bool(np.all(np.isfinite(C)))
                out[prec] = e
            print(json.dumps(out), flush=True)


def resolution_sweep(diameters, t_conv: float, precision: str):
    """Drag of a circular cylinder at Re 100 against the grid points per diameter, for
    the four estimators (the convergence test of Sec. V: channel 60 D x 5 D, cylinder
    15 D from the inlet, uniform inlet 0.05, walls).  Each run lasts t_conv convective
    times (U t / D) from rest; Cd is the mean over the last quarter.  The limit of each
    estimator is extrapolated from the three finest grids (Richardson, with the observed
    order); one JSON line per grid, then one summary line."""
    import numpy as np

    import workloads
    from paper_2210_10377_amd import Sim

    u, re = 0.05, 100.0
    names = ("A", "B", "DRTT", "SI")
    rows = []
    for d in diameters:
        nx, ny = 60 * d, 5 * d
        mask = workloads.cylinder_mask(nx, ny, 15 * d, (ny - 1) / 2.0, d / 2.0)
        box = workloads.default_box(mask, max(2, d // 4))
        tau = workloads.tau_from_re(u, d, re)
        steps = int(round(t_conv * d / u))
        sim = Sim(mask, tau, workloads.uniform_inlet(ny, u), precision=precision, box=box,
                  max_record=20000, u_ref=u, l_ref=float(d))
        t0 = time.perf_counter()
        C = sim.coefficients(sim.run(steps))
        wall = time.perf_counter() - t0
        win = C[-(steps // 4):]
        cd = {n: float(win[:, k, 0].mean()) for k, n in enumerate(names)}
        cl_rms = {n: float(np.sqrt((win[:, k, 1] ** 2).mean())) for k, n in enumerate(names)}
        row = {"D": d, "nx": nx, "ny": ny, "tau": tau, "steps": steps, "cd_mean": cd,
               "cl_rms": cl_rms, "finite": bool(np.isfinite(C).all()), "wall_s": round(wall, 2)}
        rows.append(row)
        print(json.dumps(row), flush=True)
        del sim
    summary = {"resolution_sweep": "cylinder Re 100, channel 60D x 5D", "storage": precision,
               "convective_times": t_conv}
    if len(rows) >= 3:
        ext = _richardson(rows, names)
        ref = ext["DRTT"]["cd_limit"]
        if ref:
            for n in names:
                ext[n]["rel_err_vs_drtt_limit_by_D"] = {
                    r["D"]: abs(r["cd_mean"][n] - ref) / abs(ref) for r in rows}
        summary["extrapolated"] = ext
    print(json.dumps(summary), flush=True)


def cp_cylinder(d: int, t_conv: float, window: float, precision: str):
    """Pressure coefficient around a circular cylinder at Re 100 (Sec. V, the C_p
    equation and Fig. cp_cylinder (a): over the boundary fluid nodes, no extrapolation),
    channel 60 D x 5 D, cylinder 15 D from the inlet, uniform inlet 0.05, walls.  After
    t_conv convective times from rest, C_p is sampled every 50 steps over the last
    `window` convective times and averaged; p_inf is sampled far upstream, on the
    centreline 10 D ahead of the cylinder.  theta is the angle from the front
    stagnation point (upstream), counted towards the upper side.  One JSON line per
    15-degree bin (upper and lower halves folded), then a summary."""
    import numpy as np

    import workloads
    from paper_2210_10377_amd import Sim

    u, re = 0.05, 100.0
    nx, ny = 60 * d, 5 * d
    xc, yc = 15 * d, (ny - 1) / 2.0
    mask = workloads.cylinder_mask(nx, ny, xc, yc, d / 2.0)
    tau = workloads.tau_from_re(u, d, re)
    steps = int(round(t_conv * d / u))
    nwin = int(round(window * d / u)) // 50 * 50
    sim = Sim(mask, tau, workloads.uniform_inlet(ny, u), precision=precision, max_record=8,
              u_ref=u, l_ref=float(d))
    ref = (5 * d, ny // 2)
    sim.step(steps - nwin, schemes=())
    acc, k = None, 0
    lo = hi = None
    for _ in range(nwin // 50):
        sim.step(50, schemes=())
        nodes, cp = sim.boundary_cp(ref)
        acc = cp.copy() if acc is None else acc + cp
        lo = cp.copy() if lo is None else np.minimum(lo, cp)
        hi = cp.copy() if hi is None else np.maximum(hi, cp)
        k += 1
    cp_mean = acc / k
    y, x = nodes // nx, nodes % nx
    theta = np.degrees(np.arctan2(np.abs(y - yc), -(x - xc)))
    rows = []
    for b0 in range(0, 180, 15):
        sel = (theta >= b0) & (theta < b0 + 15) if b0 < 165 else (theta >= b0)
        if not sel.any():
            continue
        row = {"theta_deg": [b0, b0 + 15], "nodes": int(sel.sum()),
               "cp_mean": round(float(cp_mean[sel].mean()), 4),
               "cp_min": round(float(lo[sel].min()), 4), "cp_max": round(float(hi[sel].max()), 4)}
        rows.append(row)
        print(json.dumps(row), flush=True)
    front = int(np.argmin(theta))
    print(json.dumps({"cp_cylinder": f"Re 100, D = {d}, channel {nx}x{ny}", "storage": precision,
                      "tau": tau, "steps": steps, "window_steps": nwin, "samples": k,
                      "boundary_nodes": int(len(nodes)), "p_inf_node": list(ref),
                      "cp_front_stagnation": round(float(cp_mean[front]), 4),
                      "cp_min_mean": round(float(cp_mean.min()), 4),
                      "theta_of_cp_min_deg": round(float(theta[np.argmin(cp_mean)]), 1),
                      "cp_base_mean": round(float(cp_mean[theta >= 170].mean()), 4)}),
          flush=True)


def _richardson(rows, names, key="cd_mean"):
    """c(D) = c_inf + a D^-p through the three finest grids, per estimator; each grid's
    relative error against that limit."""
    from scipy.optimize import brentq
    d1, d2, d3 = (r["D"] for r in rows[-3:])
    ext = {}
    for n in names:
        c1, c2, c3 = (r[key][n] for r in rows[-3:])
        f = lambda p: (c1 - c2) / (d1 ** -p - d2 ** -p) - (c2 - c3) / (d2 ** -p - d3 ** -p)
        try:
            p = brentq(f, 0.2, 4.0)
            a = (c2 - c3) / (d2 ** -p - d3 ** -p)
            cinf = c3 - a * d3 ** -p
        except ValueError:
            p, cinf = None, None
        ext[n] = {"order": p, "cd_limit": cinf,
                  "rel_err_by_D": {r["D"]: (abs(r[key][n] - cinf) / abs(cinf) if cinf else None)
                                   for r in rows}}
    return ext


def sphere_sweep(diameters, t_conv: float, precision: str, re: float):
    """The three-dimensional analogue of the paper's grid-requirement study (Table
    comp_details: points per length needed for a drag within 2 % of the converged value,
    MEA against DRTT), on the D3Q27 path: a sphere in a square duct 16 D x 6 D x 6 D with
    walls, centred 4 D from the inlet, uniform inlet 0.05, at the given Re on D.  Each run
    lasts t_conv convective times from rest; Cd = 2 F_x / (rho U^2 pi D^2 / 4) is the mean
    over the last quarter.  The limit of each estimator is extrapolated from the three
    finest grids (self-referenced: no literature data); the summary gives each grid's
    error and the coarsest D within 2 % per estimator."""
    import numpy as np
    from workloads import d3, tau_from_re
    from paper_2210_10377_amd import Sim3

    u = 0.05
    names = ("A", "B", "DRTT", "SI")
    rows = []
    for d in diameters:
        nx, ny, nz = 16 * d, 6 * d, 6 * d
        c = (3 * d - 0.5)
        mask = d3.sphere_mask(nx, ny, nz, 4 * d, c, c, d / 2.0)
        box = d3.default_box3(mask, max(2, d // 4))
        tau = tau_from_re(u, d, re)
        steps = int(round(t_conv * d / u))
        sim = Sim3(mask, tau, np.full((nz, ny), u), precision=precision, box=box,
                   max_record=4096)
        t0 = time.perf_counter()
        F = sim.run(steps)
        wall = time.perf_counter() - t0
        C = F / (0.5 * u * u * np.pi * d * d / 4.0)
        win = C[-(steps // 4):]
        cd = {n: float(win[:, k, 0].mean()) for k, n in enumerate(names)}
        side = {n: float(np.abs(win[:, k, 1:]).max()) for k, n in enumerate(names)}
        row = {"D": d, "grid": [nx, ny, nz], "tau": tau, "steps": steps, "cd_mean": cd,
               "max_side_coefficient": side, "finite": bool(np.isfinite(C).all()),
               "wall_s": round(wall, 2), "mlups": round(nx * ny * nz * steps / wall / 1e6, 1)}
        rows.append(row)
        print(json.dumps(row), flush=True)
        del sim
    summary = {"sphere_sweep": f"sphere Re {re:g}, duct 16D x 6D x 6D", "storage": precision,
               "convective_times": t_conv}
    if len(rows) >= 3:
        ext = _richardson(rows, names)
        # A staircase sphere converges non-monotonically, so the power-law limit may not
        # exist; every estimator is also measured against the finest grid's B value.
        ref = rows[-1]["cd_mean"]["B"]
        for n in names:
            errs = ext[n]["rel_err_by_D"]
            ok = [D for D in sorted(errs) if errs[D] is not None and
                  all(errs[E] is not None and errs[E] <= 0.02 for E in errs if E >= D)]
            ext[n]["coarsest_D_within_2pct"] = ok[0] if ok else None
            fin = {r["D"]: abs(r["cd_mean"][n] - ref) / abs(ref) for r in rows}
            ext[n]["rel_err_vs_finest_B_by_D"] = fin
            ok = [D for D in sorted(fin) if all(fin[E] <= 0.02 for E in fin if E >= D)]
            ext[n]["coarsest_D_within_2pct_of_finest_B"] = ok[0] if ok else None
        summary["extrapolated"] = ext
    print(json.dumps(summary), flush=True)


def precision_study3(d: int, t_conv: float, re: float):
    """Reduced-precision storage on the D3Q27 path: the sphere duct of the sphere sweep
    (diameter d, Re re, t_conv convective times from rest) in FP64, FP32, FP32 deviations
    and FP16 deviations; Cd (mean over the last quarter) and the velocity field at the
    end against the FP64 run on the same GPU."""
    import numpy as np
    from workloads import d3, tau_from_re
    from paper_2210_10377_amd import Sim3

    u = 0.05
    nx, ny, nz = 16 * d, 6 * d, 6 * d
    c = 3 * d - 0.5
    mask = d3.sphere_mask(nx, ny, nz, 4 * d, c, c, d / 2.0)
    box = d3.default_box3(mask, max(2, d // 4))
    tau = tau_from_re(u, d, re)
    steps = int(round(t_conv * d / u))
    names = ("A", "B", "DRTT", "SI")
    q = 0.5 * u * u * np.pi * d * d / 4.0
    fl = mask == 0
    cx = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                   0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1], float)
    res, ref = {}, None
    for prec in ("fp64", "fp32", "fp32dev", "fp32sr", "fp16dev"):
        sim = Sim3(mask, tau, np.full((nz, ny), u), precision=prec, box=box, max_record=4096)
        C = sim.run(steps) / q
        S = sim.populations()
        del sim
        ux = np.tensordot(cx, S, 1)[fl] / S.sum(0)[fl]
        cd = {n: float(C[-(steps // 4):, k, 0].mean()) for k, n in enumerate(names)}
        if ref is None:
            ref = (cd, ux, C)
        row = {"storage": prec, "cd_mean": cd,
               "cd_rel_err_vs_fp64": {n: abs(cd[n] - ref[0][n]) / abs(ref[0][n]) for n in names},
               "cd_max_step_err_vs_fp64": {n: float(np.abs(C[:, k, 0] - ref[2][:, k, 0]).max()
                                                    / np.abs(ref[2][:, k, 0]).max())
                                           for k, n in enumerate(names)},
               "ux_linf_err_vs_fp64": float(np.abs(ux - ref[1]).max() / u),
               "ux_l2_err_vs_fp64": float(np.sqrt(((ux - ref[1]) ** 2).mean()) / u)}
        res[prec] = row
        print(json.dumps(row), flush=True)
    print(json.dumps({"precision_study_3d": f"sphere D {d}, Re {re:g}, duct 16D x 6D x 6D",
                      "steps": steps, "tau": tau}), flush=True)


def slab_bench(precision: str, steps: int, warmup: int, k: int = 2, parts: int = 8):
    """One GPU's share of the benchmark airfoil split into `parts` x-slabs (the
    decomposition the path would use on several GPUs): columns [k W, (k+1) W) of the
    8192 x 4096 channel with the airfoil part they hold, at that real shape.  Periodic
    x stands in for the halo columns the neighbouring slabs would provide, so every
    column streams as in the interior of the full run; A, B and SI every step (the
    control volume of the full run spans several slabs: no DRTT here)."""
    import numpy as np
    import torch
    import workloads
    from paper_2210_10377_amd import Sim, _capi as C

    w = workloads.naca_8192x4096()
    W = w.nx // parts
    mask = np.ascontiguousarray(w.mask[:, k * W:(k + 1) * W])
    sim = Sim(mask, w.tau, None, precision=precision, bc_x=C.LBM_BCX_PERIODIC,
              max_record=max(steps, warmup, 1))
    info = sim.info()
    schemes = ("A", "B", "SI")
    sim.step(warmup, schemes)
    sim.forces()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps, schemes)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    bpn = BYTES_PER_NODE[precision]
    achieved = info.n_fluid * bpn / (ms / 1e3) / 1e9
    print(json.dumps({
        "metric": "slab MLUPS incl. per-step forces", "workload": f"{w.name}_slab{k}of{parts}",
        "nx": W, "ny": w.ny, "storage": precision, "steps": steps,
        "fluid_nodes": int(info.n_fluid), "links": int(info.n_links),
        "us_per_step": round(ms * 1e3, 3), "mlups": round(W * w.ny / ms / 1e3, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)},
        "halo_bytes_per_cut_each_way": 3 * w.ny * (bpn // 18)}), flush=True)


def remask_bench(precision: str, moves: int = 8, chunk: int = 20):
    """Cost of moving a body through the grid: the benchmark airfoil (8192 x 4096) and the
    3-D airfoil (1920 x 192 x 96), each translated one node along x `moves` times with
    its control volume, `chunk` steps with all forces between moves.  Reports the wall
    time of one mask change (host re-plan, changed-node refill, plan upload; the call
    synchronises) against the time of one step."""
    import numpy as np
    import torch
    import workloads
    from workloads import d3
    from paper_2210_10377_amd import Sim, Sim3

    out = {"metric": "mask change cost (a body moving through the grid)", "storage": precision,
           "moves": moves, "steps_between": chunk}
    w = workloads.naca_8192x4096()
    w3 = d3.naca3d(24, 200.0)
    for key, ww, make in (
            ("2d", w, lambda: Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box,
                                  max_record=moves * chunk + chunk)),
            ("3d", w3, lambda: Sim3(w3.mask, w3.tau, w3.uin, precision=precision, bc_z=w3.bc_z,
                                    box=w3.box, max_record=moves * chunk + chunk))):
        sim = make()
        box = list(ww.box)
        t_mask, n_changed = 0.0, 0
        t0 = time.perf_counter()
        for k in range(1, moves + 1):
            sim.step(chunk)
            torch.cuda.synchronize()
            m = np.roll(ww.mask, k, axis=-1)
            box[0] += 1
            box[1] += 1
            n_changed += int((m != np.roll(ww.mask, k - 1, axis=-1)).sum())
            t1 = time.perf_counter()
            sim.set_mask(m, tuple(box))
            t_mask += time.perf_counter() - t1
        sim.step(chunk)
        sim.forces()
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(chunk)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        out[key] = {"workload": ww.name, "ms_per_mask_change": round(t_mask / moves * 1e3, 2),
                    "changed_nodes_per_move": n_changed // moves,
                    "ms_per_step": round(e0.elapsed_time(e1) / chunk, 4),
                    "wall_s": round(total, 2)}
        del sim
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def small_grid_bench(precision: str, steps: int):
    """The 200x80 cylinder channel (D 20, Re 20; the FP64 parity configuration): a grid
    of 16,000 nodes is bound by launch latency, not by HBM.  Direct `lbm_step` launches
    against the same lattice as a one-member batch replaying captured HIP graphs of 64
    launches (bitwise the same results); all four forces every step."""
    import torch
    import workloads
    from paper_2210_10377_amd import Batch, Sim

    w = workloads.cylinder_channel_200x80()
    out = {"metric": "small-grid MLUPS incl. per-step forces", "workload": w.name,
           "storage": precision, "steps": steps}
    sim = Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=steps + 200)
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    sim.step(200)
    sim.forces()
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_direct = e0.elapsed_time(e1) / steps
    F_direct = sim.forces()
    del sim
    b = Batch([Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=1)],
              max_record=steps + 200)
    b.set_schedule(grid_blocks=0, graph_steps=64)
    b.step(200)
    b.forces()
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / steps
    F_graph, _ = b.forces()
    nodes = w.nx * w.ny
    out.update({"direct_us_per_step": round(ms_direct * 1e3, 3),
                "direct_mlups": round(nodes / ms_direct / 1e3, 1),
                "graph_us_per_step": round(ms_graph * 1e3, 3),
                "graph_mlups": round(nodes / ms_graph / 1e3, 1),
                "same_forces": bool((F_direct == F_graph[0]).all())})
    print(json.dumps(out), flush=True)


def adjoint_bench(precision: str, large: bool = False, tile: str = "auto", emit: bool = True):
    """Forward (checkpointed) and backward (recompute + reverse kernels) throughput of
    the adjoint workload; MLUPS = nx * ny * steps / wall time of each phase.  `large`:
    the same objective on the 8192 x 4096 airfoil (chord 1024, AoA 4, Re 1e4) over a
    short run (200 steps, checkpoint every 20, mean drag over the last 100), where each
    reverse launch moves gigabytes and the kernel is bound by HBM rather than by the
    latency of a single wave of workgroups."""
    import torch

    import workloads
    from paper_2210_10377_amd import Sim

    if large:
        # From rest the inlet's pressure wave needs about 4000 steps to reach the
        # leading edge (x = 2049, at about 0.58 nodes per step): the adjoint window
        # starts after 5000 plain steps, so the drag and its gradient are not zero.
        w = workloads.naca_8192x4096()
        n, every, t0, T, develop = 200, 20, 100, 100, 5000
    else:
        w = workloads.naca_1024x512_adjoint()
        n, every, t0, T, develop = 10000, 500, 8000, 2000, 0
    sim = Sim(w.mask, w.tau, w.uin, precision=precision, box=w.box, max_record=8,
              u_ref=w.u_ref, l_ref=w.l_ref, tile=tile)
    if develop:
        sim.step(develop, schemes=())
    sim.adjoint_forward(n, every, t0, T)   # warm-up and workspace allocation
    sim.adjoint_backward(1.0)
    sim.reset()
    if develop:
        sim.step(develop, schemes=())
    torch.cuda.synchronize()
    t = time.perf_counter()
    J = sim.adjoint_forward(n, every, t0, T)
    t_f = time.perf_counter() - t
    t = time.perf_counter()
    gu, gt = sim.adjoint_backward(1.0)
    t_b = time.perf_counter() - t
    sim.reset()
    t = time.perf_counter()
    sim.step(n, schemes=())
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    nodes = w.nx * w.ny
    fluid = int(sim.info().n_fluid)
    s = BYTES_PER_NODE[precision] // 18          # bytes per stored population
    s_adj = 8 if precision == "fp64" else 4      # bytes per adjoint value
    fwd_bytes = fluid * 18 * s * n               # the forward run (checkpoint copies aside)
    # Backward: each segment of len steps recomputes len - 1 of them (2 Q s per node),
    # n - ceil(n / every) in all; the reverse kernel runs every step (Q s + 2 Q s_adj).
    recomputed = n - (n + every - 1) // every
    bwd_bytes = fluid * (18 * s * recomputed + (9 * s + 18 * s_adj) * n)
    out = {
        "metric": "adjoint MLUPS", "workload": w.name, "storage": precision, "steps": n,
        "tile": tile,
        "developed_steps": develop,
        "roofline": {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "forward_achieved": round(fwd_bytes / t_f / 1e9, 1),
                     "backward_achieved": round(bwd_bytes / t_b / 1e9, 1),
                     "backward_bytes_per_node_step": round(bwd_bytes / fluid / n, 2),
                     "backward_frac": round(bwd_bytes / t_b / 1e9 / HBM_PEAK_GBS, 4)},
        "checkpoint_every": every, "J_mean_drag": J, "dJ_dtau": gt,
        "dJ_duin_norm": float((gu ** 2).sum() ** 0.5),
        "forward_s": round(t_f, 4), "backward_s": round(t_b, 4), "plain_run_s": round(t_plain, 4),
        "forward_mlups": round(nodes * n / t_f / 1e6, 1),
        "backward_mlups": round(nodes * n / t_b / 1e6, 1),
        "plain_mlups": round(nodes * n / t_plain / 1e6, 1),
        "fwd_plus_bwd_over_plain": round((t_f + t_b) / t_plain, 3)}
    if emit:
        print(json.dumps(out), flush=True)
    return out


def accuracy_summary(storages, steps: int = 20000, window: int = 2000):
    """Window-mean force coefficients of the precision-study channel (NACA0012 2048 x
    1024, chord 256, AoA 4, Re 1000, `steps` steps from rest) in each storage against the
    FP64 storage on the same GPU (which matches the oracle's fixtures of this run to
    1e-10): relative errors of the mean drag and lift over the last `window` steps, per
    estimator."""
    import numpy as np

    import workloads
    from paper_2210_10377_amd import Sim

    w = workloads.naca_2048x1024(aoa=4.0, re=1000.0)
    names = ("A", "B", "DRTT", "SI", "DRTT_POST")
    means = {}
    for prec in ["fp64"] + list(storages):
        sim = Sim(w.mask, w.tau, w.uin, precision=prec, box=w.box, max_record=window,
                  u_ref=w.u_ref, l_ref=w.l_ref)
        sim.step(steps - window, schemes=())
        C = sim.coefficients(sim.run(window))
        means[prec] = C.mean(0)
        del sim
    ref = means["fp64"]
    out = {"workload": w.name, "steps": steps, "window": window, "reference": "fp64"}
    for prec in storages:
        err = np.abs(means[prec] - ref) / np.abs(ref)
        out[prec] = {"cd": {n: float(f"{err[k, 0]:.3g}") for k, n in enumerate(names)},
                     "cl": {n: float(f"{err[k, 1]:.3g}") for k, n in enumerate(names)}}
    return out


def batch_accuracy(steps: int, window: int, collision: str = "bgk"):
    """Per-instance force coefficients of the 256-instance batch in each storage against
    the FP64 batch (itself matched to the oracle to 1e-10 on a mini batch, and bitwise to
    single runs): every instance `steps` steps from rest, window means over the last
    `window` steps.  Drag errors are relative to the instance's FP64 window-mean drag; lift
    errors are given in the same unit (relative to that drag), since the cylinders' mean
    lift is zero.  Instances whose FP64 run is not finite are counted apart; so are
    unsteady ones (FP64 drag varying by more than 1 % over the window), whose window means
    depend on the phase of the shedding."""
    import numpy as np

    import workloads
    from paper_2210_10377_amd import Batch

    ws = workloads.batched_instances(steps=steps)
    res = {}
    for prec in ("fp64", "fp32", "fp32dev", "fp16dev"):
        b = Batch.from_workloads(ws, precision=prec, max_record=window, collision=collision)
        if steps > window:
            b.step(steps - window, schemes=())
        F, bad = b.run(window)
        res[prec] = (b.coefficients(F), bad)
        del b
    C64, bad64 = res["fp64"]
    cd64 = C64[:, :, 1, 0]          # algorithm B drag, [instance, step]
    mean64 = cd64.mean(1)
    unsteady = (cd64.max(1) - cd64.min(1)) > 0.01 * np.abs(mean64)
    ok = ~bad64 & np.isfinite(mean64)
    out = {"batch_accuracy": workloads.__name__ + ".batched_instances", "collision": collision,
           "steps": steps,
           "window": window, "instances": len(ws), "fp64_nonfinite": int((~ok).sum()),
           "unsteady": int((unsteady & ok).sum())}
    names = ("A", "B", "DRTT", "SI", "DRTT_POST")
    for prec in ("fp32", "fp32dev", "fp16dev"):
        C, bad = res[prec]
        e = {"nonfinite": int((bad & ok).sum())}
        for k, name in enumerate(names):
            m64 = C64[:, :, k].mean(1)
            m = C[:, :, k].mean(1)
            ref = np.abs(C64[:, :, 1, 0].mean(1))
            ecd = np.abs(m[:, 0] - m64[:, 0]) / np.abs(m64[:, 0])
            ecl = np.abs(m[:, 1] - m64[:, 1]) / ref
            for label, sel in (("steady", ok & ~unsteady & ~bad), ("unsteady", ok & unsteady & ~bad)):
                if sel.any():
                    e[f"{name}_{label}"] = {
                        "cd_rel_err_median": float(np.median(ecd[sel])),
                        "cd_rel_err_max": float(ecd[sel].max()),
                        "cl_err_over_cd_max": float(ecl[sel].max()),
                        "n_cd_above_1e-4": int((ecd[sel] > 1e-4).sum())}
        out[prec] = e
    print(json.dumps(out), flush=True)


def batched_bench(precision: str, steps: int, seq_steps: int, collision: str):
    """The 256-instance batch (uneven cylinder and airfoil channels, one launch per step
    for all of them): autotuned schedule, then `steps` timed steps with all four forces.
    Beside it: the same instances stepped one after another through the single-lattice
    call, and the batch in FP64 storage."""
    import numpy as np
    import torch

    import workloads
    from paper_2210_10377_amd import Batch

    ws = workloads.batched_instances()
    nodes = sum(w.nx * w.ny for w in ws)

    def timed_batch(prec, k, tune):
        b = Batch.from_workloads(ws, precision=prec, max_record=max(k, 16), collision=collision)
        sched, tune_ms = b.autotune(steps=8) if tune else (None, None)
        b.step(16)
        b.forces()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(k)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        F, bad = b.forces()
        info = b.info()
        return b, sched, tune_ms, ms, F, bad, info

    b, sched, tune_ms, ms, F, bad, info = timed_batch(precision, steps, True)
    Cf = b.coefficients(F[:, -1:])[:, 0]
    fluid = int(info.total_fluid)
    t_step = ms / 1e3 / steps
    mlups = nodes / t_step / 1e6
    achieved = fluid * BYTES_PER_NODE[precision] / t_step / 1e9
    # the same instances, one lbm_step call per instance per chunk, same stream
    seq = b.members
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    for m in seq:
        m.step(seq_steps, schemes=())
    e1.record(b.stream)
    torch.cuda.synchronize()
    seq_mlups = nodes * seq_steps / (e0.elapsed_time(e1) / 1e3) / 1e6
    del b, seq
    torch.cuda.empty_cache()
    b64, _, _, ms64, _, _, _ = timed_batch("fp64", max(steps // 4, 16), False)
    mlups64 = nodes / (ms64 / 1e3 / max(steps // 4, 16)) / 1e6
    del b64
    torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "batched MLUPS incl. per-step forces",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "ms_per_step": round(ms / steps, 5), "higher_is_better": True,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32dev": "f32", "fp32sr": "f32",
                  "fp16dev": "f16 storage / f32 arithmetic"}[precision],
        "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD,
                   "instances": len(ws), "nodes": nodes, "fluid_nodes": fluid,
                   "storage": precision, "collision": collision, "schedule": sched,
                   "autotune_ms_per_step": tune_ms},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(BATCH_WORKLOAD, precision)},
        "nonfinite_instances": int(bad.sum()),
        "sequential_single_calls_mlups": round(seq_mlups, 1),
        "batch_fp64_mlups": round(mlups64, 1),
        "cd_cl_B_last_step_first8": [[round(float(v), 5) for v in Cf[i, 1]] for i in range(8)],
    }), flush=True)


def three_d_bench(precision: str, steps: int, warmup: int, ppc: int, re: float,
                  cpu: bool, collision: str = "bgk", layout: str = "auto",
                  from_rest: bool = False):
    """The D3Q27 path on the three-dimensional NACA0012 of the paper's Sec. V (zero
    incidence, domain 80 x 8 x 4 chords, periodic span, control volume over the whole
    span), all four estimators every step.  From rest the inlet's pressure wave needs
    about 25 chords / c_s steps to reach the leading edge; unless `from_rest`, that many
    plain steps run untimed first, so the timed steps carry real forces."""
    import numpy as np
    import torch
    from workloads import d3
    from paper_2210_10377_amd import Sim3

    w = d3.naca3d(ppc, re)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sim = Sim3(w.mask, w.tau, w.uin, precision=precision, bc_z=w.bc_z, box=w.box,
               max_record=max(steps, warmup, 1), device=dev, stream=stream,
               collision=collision, layout=layout)
    info = sim.info()
    develop = 0 if from_rest else int(round(25 * w.meta["chord"] * np.sqrt(3.0)))
    if develop:
        sim.step(develop, ())
    sim.step(warmup)
    sim.forces()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    F = sim.forces()
    k_off = min(steps, 300)
    e0.record(stream)
    sim.step(k_off, ())
    e1.record(stream)
    torch.cuda.synchronize()
    ms_off = e0.elapsed_time(e1) / k_off
    t_step = ms / 1e3 / steps
    nodes = w.nx * w.ny * w.nz
    bpn = 2 * 27 * (BYTES_PER_NODE[precision] // 18)
    achieved = info.n_fluid * bpn / t_step / 1e9
    q = 0.5 * w.u_ref ** 2 * w.area_ref
    out = {
        "metric": "D3Q27 MLUPS incl. per-step force + HBM GB/s % peak",
        "value": round(nodes / t_step / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms / steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32dev": "f32", "fp32sr": "f32",
                  "fp16dev": "f16 storage / f32 arithmetic"}[precision],
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "nz": w.nz, "tau": w.tau,
                   "storage": precision, "collision": collision, "layout": layout,
                   "schemes": list(ALL),
                   "fluid_nodes": int(info.n_fluid), "links": int(info.n_links),
                   "box_nodes": int(info.n_box), "general_strips": int(info.n_general),
                   "strips": int(info.n_strips), **w.meta},
        # one step = the main step kernel + the force-strip kernel; bytes are the
        # algorithmic 2 x 27 populations per fluid node over the whole step's time
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(w.name, precision, three_d=True)},
        "wall_s": round(wall, 3),
        "developed_steps": develop,
        "forces_off_ms_per_step": round(ms_off, 5),
        "force_cost_frac": round((ms / steps - ms_off) / ms_off, 4),
        "forces_finite": bool(np.isfinite(F).all()) if len(F) else None,
        "last_coefficients": {s: (F[-1, k] / q).tolist() for k, s in enumerate(ALL)}
        if len(F) else None,
    }
    del sim
    torch.cuda.empty_cache()
    if cpu:
        from oracle import d3q27 as D
        o = D.OracleSim3(w.mask, tau=w.tau, uin=w.uin, bc_z=w.bc_z, box=w.box,
                         collision=collision)
        t0 = time.perf_counter()
        o.step(1)
        o.forces()
        dt = time.perf_counter() - t0
        del o
        out["cpu_baseline"] = {"value": round(nodes / dt / 1e6, 3), "unit": "MLUPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"1 full-grid step of {w.nx}x{w.ny}x{w.nz} with A, B, "
                                         f"DRTT and SI forces ({dt:.1f} s, FP64, one thread)"}
    print(json.dumps(out), flush=True)


ALL = ("A", "B", "DRTT", "SI")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default=None, choices=sorted(BYTES_PER_NODE),
                    help="storage (default: fp32; fp32dev for the adjoint, the resolution "
                         "sweep and the sphere sweep; fp64 for the small-grid case; fp32sr, "
                         "binary32 populations rounded stochastically, for single 2-D "
                         "lattices only)")
    ap.add_argument("--workload", default="naca8192",
                    choices=["naca8192", "naca2048", "cyl200", "empty8192"],
                    help="empty8192: the 8192x4096 grid periodic in x and y without a body "
                         "(every node streams plainly: exactly 2 Q s bytes per node, the "
                         "counter calibration check)")
    ap.add_argument("--re", type=float, default=1e4)
    ap.add_argument("--aoa", type=float, default=4.0)
    ap.add_argument("--schemes", default="A,B,DRTT,SI,DRTT_POST")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "regularized", "kbc"])
    ap.add_argument("--pitch-rate", type=float, default=0.0,
                    help="turn the body at this rate (radians per step, counter-clockwise) "
                         "about its quarter chord (the centroid of a cylinder): the "
                         "moving-wall rule on every body link")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--from-rest", action="store_true",
                    help="start the timed workload from rest (default: the uniform inlet flow)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="report the timed step alone: no CPU baseline and no adjoint or "
                         "accuracy summaries (profiling runs)")
    ap.add_argument("--precision-study", action="store_true",
                    help="FP32 and FP16-deviation storage against FP64 on the NACA0012 "
                         "2048x1024 channel (AoA 0/4/8, Re 100/1000): force, coefficient "
                         "and velocity-field errors; one JSON line per case")
    ap.add_argument("--study-steps", type=int, default=20000)
    ap.add_argument("--sensitivity", action="store_true",
                    help="FP64 twins of the precision-study channel perturbed once by "
                         "binary32-sized noise: the spread of the window-mean coefficients")
    ap.add_argument("--twins", type=int, default=4)
    ap.add_argument("--perturb-every", type=int, default=0)
    ap.add_argument("--frozen", action="store_true")
    ap.add_argument("--adjoint-large", action="store_true",
                    help="adjoint on the 8192x4096 airfoil (chord 1024, AoA 4, Re 1e4): 200 "
                         "steps, checkpoint every 20, mean drag over the last 100")
    ap.add_argument("--adjoint", action="store_true",
                    help="adjoint workload: NACA0012 chord 256 in 1024x512, Re 500, 10000 "
                         "steps, mean drag over the last 2000, checkpoint every 500; "
                         "forward and backward MLUPS")
    ap.add_argument("--batch-accuracy", action="store_true",
                    help="per-instance force coefficients of the 256-instance batch in each "
                         "storage against the FP64 batch (--study-steps steps from rest, "
                         "window means over the last 2000)")
    ap.add_argument("--batched", action="store_true",
                    help="256 uneven cylinder/NACA0012 channels (64x32 to 512x256, Re 20 to "
                         "2000) stepped together; autotuned schedule; batched MLUPS beside "
                         "the instances stepped one by one and the FP64 batch")
    ap.add_argument("--seq-steps", type=int, default=50)
    ap.add_argument("--cp-cylinder", action="store_true",
                    help="time-averaged C_p around a cylinder at Re 100 (D = --cp-diameter, "
                         "channel 60D x 5D), binned by the angle from the front stagnation "
                         "point")
    ap.add_argument("--cp-diameter", type=int, default=15)
    ap.add_argument("--cp-window", type=float, default=40.0,
                    help="convective times averaged at the end of the --convective-times run")
    ap.add_argument("--resolution-sweep", action="store_true",
                    help="cylinder at Re 100 in a 60D x 5D channel for D in --diameters: "
                         "mean drag of A, B, DRTT and SI against points per diameter, with "
                         "Richardson extrapolation from the three finest grids")
    ap.add_argument("--diameters", default="10,15,20,30,40,60")
    ap.add_argument("--convective-times", type=float, default=150.0)
    ap.add_argument("--three-d", action="store_true",
                    help="the D3Q27 path on the 3-D NACA0012 (80 x 8 x 4 chords, --ppc nodes "
                         "per chord, periodic span)")
    ap.add_argument("--ppc", type=int, default=24)
    ap.add_argument("--remask", action="store_true",
                    help="cost of a mask change (a body moving through the grid) on the "
                         "2-D and 3-D benchmark airfoils")
    ap.add_argument("--slab", action="store_true",
                    help="one GPU's share of the benchmark airfoil in an 8-way x-slab "
                         "decomposition (1024 x 4096, periodic x for the halo)")
    ap.add_argument("--tile", default="auto", choices=["auto", "wide", "narrow"],
                    help="step-kernel tiles: 256 x 1 (wide), 64 x 4 (narrow), or the plan's rule")
    ap.add_argument("--layout", default="auto", choices=["auto", "rows", "planes"],
                    help="device layout of the state buffers")
    ap.add_argument("--small-grid", action="store_true",
                    help="the 200x80 cylinder: direct launches against captured graphs")
    ap.add_argument("--sphere-sweep", action="store_true",
                    help="3-D grid-requirement study: sphere drag against points per "
                         "diameter for A, B, DRTT and SI (--sphere-diameters, --re)")
    ap.add_argument("--sphere-diameters", default="8,12,16,20,24,32,40")
    ap.add_argument("--precision-study-3d", action="store_true",
                    help="FP64/FP32/FP32-dev/FP16-dev Cd and velocity errors on the sphere duct")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device-to-device copy of 1 GiB five times (the "
                         "known-size reference for the HBM byte counters)")
    args = ap.parse_args()
    explicit_precision = args.precision
    args.precision = args.precision or "fp32"

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the lattice is not decomposed across GPUs "
              "(it would shard into x-slabs with a three-population halo per cut).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        # The same copy timed: the practical ceiling of a kernel that reads and writes
        # each byte once (2 bytes of traffic per byte copied).
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 25, "ms_per_copy": round(ms, 4),
                          "read_plus_write_gbs": round(2 * n / (ms / 1e3) / 1e9, 1),
                          "frac_of_8tbs": round(2 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}),
              flush=True)
        return

    import workloads
    from paper_2210_10377_amd import Sim

    if args.sensitivity:
        sensitivity_study(args.study_steps, args.twins, args.perturb_every, args.frozen)
        return
    if args.precision_study:
        precision_study(args.study_steps)
        return
    if args.adjoint or args.adjoint_large:
        adjoint_bench(explicit_precision or "fp32dev", args.adjoint_large, args.tile)
        return
    if args.batch_accuracy:
        batch_accuracy(args.study_steps if args.study_steps != 20000 else 10000, 2000,
                       args.collision)
        return
    if args.batched:
        batched_bench(args.precision, args.steps, args.seq_steps, args.collision)
        return
    if args.precision_study_3d:
        precision_study3(16, args.convective_times if args.convective_times != 150.0 else 30.0,
                         args.re if args.re != 1e4 else 50.0)
        return
    if args.slab:
        slab_bench(args.precision, args.steps, args.warmup)
        return
    if args.remask:
        remask_bench(args.precision)
        return
    if args.small_grid:
        small_grid_bench(explicit_precision or "fp64",
                         args.steps if args.steps != 2000 else 5000)
        return
    if args.sphere_sweep:
        sphere_sweep([int(v) for v in args.sphere_diameters.split(",")],
                     args.convective_times if args.convective_times != 150.0 else 30.0,
                     explicit_precision or "fp32dev",
                     args.re if args.re != 1e4 else 50.0)
        return
    if args.three_d:
        three_d_bench(args.precision, args.steps if args.steps != 2000 else 500,
                      args.warmup if args.warmup != 200 else 50, args.ppc,
                      args.re if args.re != 1e4 else 200.0, not args.no_cpu_baseline,
                      args.collision if args.collision != "kbc" else "bgk", args.layout,
                      args.from_rest)
        return
    if args.cp_cylinder:
        cp_cylinder(args.cp_diameter, args.convective_times, args.cp_window, args.precision)
        return
    if args.resolution_sweep:
        resolution_sweep([int(v) for v in args.diameters.split(",")], args.convective_times,
                         explicit_precision or "fp32dev")
        return

    if args.workload == "naca8192":
        w = workloads.naca_8192x4096(aoa=args.aoa, re=args.re)
    elif args.workload == "naca2048":
        w = workloads.naca_2048x1024(aoa=args.aoa, re=args.re)
    elif args.workload == "empty8192":
        w = workloads.Workload("periodic_8192x4096_no_body", 8192, 4096,
                               np.zeros((4096, 8192), np.uint8), 0.6, np.zeros(4096), None,
                               0, 0.05, 1.0, bc_x=1, bc_y=1)
    else:
        w = workloads.cylinder_channel_200x80()
    schemes = tuple(s for s in args.schemes.split(",") if s)
    K, W = args.steps, args.warmup
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sim = Sim(w.mask, w.tau, w.uin, precision=args.precision, box=w.box, tile=args.tile, bc_x=w.bc_x,
              bc_y=w.bc_y, max_record=max(K, W, 1), rho_ref=1.0, u_ref=w.u_ref, l_ref=w.l_ref,
              device=dev, stream=stream, collision=args.collision, layout=args.layout)
    motion = None
    if args.pitch_rate:
        if "xq" in w.meta:
            xc, yc = float(w.meta["xq"]), float(w.meta["yq"])
        else:
            yc, xc = (float(v) for v in np.argwhere(w.mask).mean(axis=0))
        motion = (0.0, 0.0, args.pitch_rate, xc, yc)
        sim.set_body_motion(*motion)
    info = sim.info()
    if not args.from_rest:
        # Impulsive start: every node at the equilibrium of the inlet flow (rho = 1,
        # u = (u_in, 0)), so the body carries a physical force from the first step.
        sim.set_populations(uniform_flow_state(w))
    sim.step(W, schemes)
    sim.forces()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    sim.step(K, schemes)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    F = sim.forces()
    C = sim.coefficients(F)
    # The same step without force evaluation (no force strips, no reductions): the
    # per-step cost of the three estimators is the difference.
    k_off = min(K, 500)
    e0.record(stream)
    sim.step(k_off, ())
    e1.record(stream)
    torch.cuda.synchronize()
    ms_off = e0.elapsed_time(e1) / k_off

    t_step = ms / 1e3 / K
    nodes = w.nx * w.ny
    mlups = nodes / t_step / 1e6
    bytes_launch = info.n_fluid * BYTES_PER_NODE[args.precision]
    achieved = bytes_launch / t_step / 1e9
    traffic = measured_traffic(w.name, args.precision)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32dev": "f32", "fp32sr": "f32",
                  "fp16dev": "f16 storage / f32 arithmetic"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "tau": w.tau,
                   "storage": args.precision, "collision": args.collision,
                   "layout": args.layout, "tile": args.tile, "schemes": list(schemes),
                   "fluid_nodes": int(info.n_fluid), "links": int(info.n_links),
                   "box_nodes": int(info.n_box), **{k: v for k, v in w.meta.items()},
                   **({"body_motion": {"omega": motion[2], "xc": motion[3], "yc": motion[4]}}
                      if motion else {})},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "wall_s": round(wall, 3),
        "forces_off_ms_per_step": round(ms_off, 5),
        "force_cost_frac": round((ms / K - ms_off) / ms_off, 4),
    }
    if len(F):
        names = ("A", "B", "DRTT", "SI", "DRTT_POST")
        cols = [k for k, s in enumerate(names) if s in schemes]
        out["forces_finite"] = bool(np.all(np.isfinite(F[:, cols])))
        out["initial_state"] = "rest" if args.from_rest else "uniform inlet flow (impulsive start)"
        out["last_coefficients"] = {s: C[-1, k].tolist() for k, s in enumerate(names)
                                    if s in schemes}
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        if args.workload == "naca8192" and args.collision == "bgk" and not motion:
            # The other two parts of the metric, each on its own workload: the adjoint's
            # throughput (1024 x 512, 10,000 steps, checkpoint every 500) and the drag
            # and lift errors of the storage against FP64 (2048 x 1024, Re 1000).
            adj_prec = args.precision if args.precision in ("fp64", "fp32", "fp32dev") else "fp32dev"
            a = adjoint_bench(adj_prec, emit=False)
            out["adjoint"] = {k: a[k] for k in ("workload", "storage", "steps", "checkpoint_every",
                                                "forward_mlups", "backward_mlups",
                                                "fwd_plus_bwd_over_plain")}
            out["adjoint"]["backward_frac"] = a["roofline"]["backward_frac"]
            torch.cuda.empty_cache()
            extra = ["fp32sr"] if args.precision == "fp32" else []
            out["cd_rel_err_vs_fp64"] = accuracy_summary([args.precision] + extra)
            torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, args.collision, motion)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
