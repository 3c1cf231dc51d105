"""Throughput benchmark of the multi-scale semi-Lagrangian LBM step on one GPU.

A step is one pass of the whole hot path (criterion and switching every 20
steps, ghost fill, stream-and-collide of both velocity sets, band conversion)
over the workload's grid.  The default workload is the compressible slot jet:
1024 x 512 cells, thermal two-population model, FP32 storage, D2Q9 with D2Q16
where the local Mach number exceeds 0.4 (re-evaluated every 20 steps),
tau = 0.52, 20000 steps.  Inputs are synthetic and resident in HBM before the
timed region starts.

Prints one JSON line: MLUPS (million cell updates per second, each cell once
per step whatever its velocity set), the HBM roofline of the dominant kernel
(algorithmic bytes per launch / its HIP-event-timed average duration), and the
FP64 CPU oracle timed on a bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_2102_12559_amd import inputs
    if name == "jet":
        w = inputs.jet_c2()
        w["desc"] = ("slot jet 1024x512, slot 32 cells at Ma 0.6 (tanh edges 4 cells), athermal, "
                     "fp32, D2Q9 + D2Q36 where Ma > 0.4 (every 20 steps), tau 0.52, 20000 steps")
        return w
    if name == "jet-thermal-d2q16":
        # the thermal D2Q9/D2Q16 slot at Mach 1.2: diverges in the lattice frame
        w = inputs.jet_c2(ma=1.2, thermal=1, n_high=4, edge=0.0)
        w["desc"] = ("compressible slot jet 1024x512, slot 32 cells at Ma 1.2, thermal f+g, fp32, "
                     "D2Q9 + D2Q16 where Ma > 0.4 (every 20 steps), tau 0.52")
        return w
    if name.startswith("roofline"):
        # single velocity set on 8192^2 periodic cells, smooth random flow
        n = {"roofline-d2q9": 3, "roofline-d2q16": 4, "roofline-d2q36": 6}[name]
        N = 8192
        cfg = inputs.base_config(nx=N, ny=N, n_low=n, n_high=0, tau=0.6,
                                 store=inputs.STORE_FP32)
        rho, u, T = inputs.smooth_random_flow(N, N, umax=0.1, seed=0, modes=2)
        import numpy as np
        return dict(cfg=cfg, rho=rho, u=u, T=T, mask=np.zeros((1, N, N), np.uint8),
                    steps=100, desc=f"single D2Q{n*n} lattice 8192x8192 periodic fp32")
    if name == "vortex":
        w = inputs.vortex_c1()
        w["desc"] = "convected vortex 64x64, D2Q9 + D2Q16 disk, fp64"
        return w
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("msl_stream.hpp", "msl_device.hpp", "msl_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2102_12559_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(name, launches_cells):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, seconds_hint):
    """The FP64 oracle on the host cores: a bounded sample of the workload."""
    import numpy as np
    from oracle.oracle import Oracle
    cfg = dict(w["cfg"])
    cfg["store"] = 0
    o = Oracle(cfg)
    o.set_mask(w["mask"], convert=False)
    o.init(w["rho"], w["u"], w["T"])
    ncell = int(np.prod(o.shape))
    o.step(1)  # warm-up (first-touch of the arrays)
    steps, t0 = 0, time.time()
    while True:
        o.step(1)
        steps += 1
        if time.time() - t0 > seconds_hint:
            break
    dt = time.time() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=round(ncell * steps / dt / 1e6, 4), unit="MLUPS", cores=threads,
                kind="oracle",
                sample=f"{steps} steps of the full {cfg['nx']}x{cfg['ny']} grid from the "
                       f"initial state, FP64, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="jet")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported "
                                   "(the domain-decomposed multi-GPU step is a design only)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2102_12559_amd import msl

    w = workload(args.workload)
    steps = args.steps if args.steps is not None else w["steps"]
    cfg = w["cfg"]
    torch.cuda.set_device(0)
    s = msl.Solver(cfg, device="cuda:0")
    s.set_mask(w["mask"])
    s.init(w["rho"], w["u"], w["T"])
    s.step(args.warmup)
    torch.cuda.synchronize()
    s.profile(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = s.profile_read()
    s.profile(False)
    ncell = s.ncell
    value = ncell * steps / (ms / 1e3) / 1e6
    stable = True
    try:
        cons = s.conservation()
    except msl.MslError:
        stable, cons = False, None
    nhigh = int(s.get_mask().sum().item())

    # dominant kernel: the stream-collide class with the largest total time
    sc = {k: v for k, v in prof.items() if k.startswith("stream_collide") and v["launches"] > 0}
    dom = max(sc, key=lambda k: sc[k]["ms"])
    d = sc[dom]
    avg_ms = d["ms"] / d["launches"]
    bytes_per_launch = d["bytes"] / d["launches"]
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    store_name = {0: "f64", 1: "f32", 2: "fp16-dev", 3: "bf16-dev"}[cfg["store"]]
    out = {
        "metric": "MLUPS & % HBM roofline; learned/FP16 form vs plain at equal L2 err",
        "value": round(value, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg["store"] != 0 else "f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "grid": [cfg["nx"], cfg["ny"], cfg["nz"]],
                   "cells": ncell, "lattices": [cfg["n_low"] ** cfg["dim"],
                                                cfg["n_high"] ** cfg["dim"] if cfg["n_high"] else 0],
                   "storage": store_name, "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(args.workload, d),
            "bytes_per_launch": round(bytes_per_launch),
            "avg_launch_us": round(avg_ms * 1e3, 3),
        },
        "kernels_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
        "high_order_cells_end": nhigh,
        "stable": stable,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
