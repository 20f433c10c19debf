#!/usr/bin/env python3
"""Throughput of the fused D2Q9 step with per-step forces on one MI355X.

Workload (default): NACA0012 from the analytic 4-digit thickness law, chord 1024, angle
of attack 4 deg, in an 8192 x 4096 channel (33.5 M nodes) with no-slip walls, uniform
inlet 0.05 and zero-gradient outlet, Re 1e4 (tau_lb from nu = U c / Re), FP32 population
storage, forces by momentum exchange A and B and by DRTT at every step.  Synthetic input
(analytic geometry, flow started from rest).

One "step" is one lattice time step of the whole grid including the three force
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
BYTES_PER_NODE = {"fp64": 144, "fp32": 72, "fp16dev": 36}
CSRC = os.path.join(ROOT, "paper_2210_10377_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def kernel_hash() -> str:
    """sha256 over the library sources (kernel, launch layout and plan)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get(f"{workload}/{precision}")
    if not rec or rec.get("sources_sha256") != kernel_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(w, steps: int):
    """The oracle (plain FP64 C++, one thread) on a bounded sample of the same workload:
    `steps` full-grid time steps with all three forces."""
    import oracle
    o = oracle.OracleSim(w.mask, tau=w.tau, uin=w.uin, box=w.box)
    t0 = time.perf_counter()
    o.step(steps)
    o.forces()
    dt = time.perf_counter() - t0
    del o
    return {"value": w.nx * w.ny * steps / dt / 1e6, "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} full-grid steps of {w.nx}x{w.ny} with A, B and DRTT forces "
                      f"({dt:.1f} s, FP64, one thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="fp32", choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--workload", default="naca8192", choices=["naca8192", "naca2048", "cyl200"])
    ap.add_argument("--re", type=float, default=1e4)
    ap.add_argument("--aoa", type=float, default=4.0)
    ap.add_argument("--schemes", default="A,B,DRTT")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device-to-device copy of 1 GiB five times (the "
                         "known-size reference for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the lattice is not decomposed across GPUs "
              "(see the design notes for how it would shard).", file=sys.stderr)
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
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 5}), flush=True)
        return

    import workloads
    from paper_2210_10377_amd import Sim

    if args.workload == "naca8192":
        w = workloads.naca_8192x4096(aoa=args.aoa, re=args.re)
    elif args.workload == "naca2048":
        w = workloads.naca_2048x1024(aoa=args.aoa, re=args.re)
    else:
        w = workloads.cylinder_channel_200x80()
    schemes = tuple(s for s in args.schemes.split(",") if s)
    K, W = args.steps, args.warmup
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sim = Sim(w.mask, w.tau, w.uin, precision=args.precision, box=w.box,
              max_record=max(K, W, 1), rho_ref=1.0, u_ref=w.u_ref, l_ref=w.l_ref,
              device=dev, stream=stream)
    info = sim.info()
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
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16 storage / f32 arithmetic"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "tau": w.tau,
                   "storage": args.precision, "schemes": list(schemes),
                   "fluid_nodes": int(info.n_fluid), "links": int(info.n_links),
                   "box_nodes": int(info.n_box), **{k: v for k, v in w.meta.items()}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "wall_s": round(wall, 3),
    }
    if len(F):
        cols = [k for k, s in enumerate(("A", "B", "DRTT")) if s in schemes]
        out["forces_finite"] = bool(np.all(np.isfinite(F[:, cols])))
        out["last_coefficients"] = {s: C[-1, k].tolist() for k, s in enumerate(("A", "B", "DRTT"))
                                    if s in schemes}
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
