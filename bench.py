#!/usr/bin/env python3
"""Throughput of the unsplit MHD update on one MI355X.

Workload: the paper's performance problem (Sec. 4.2(i)): an ABC-field box
(Eq. 20, n = 1, A = B = C = 1, rho = p = 1, seeded uniform velocity noise of
amplitude 0.01) on a 128^3 periodic grid, VL + PLM(minmod) + Roe + CT,
Courant 1/2, gamma = 5/3.  One step = CFL reduction + full update
(mhd_advance), state resident in HBM.  Both FP64 and FP32 forms are timed;
the headline value is FP32 (the paper's 1.2e8 cell-updates/s on a P100 is the
FP32 number for this scheme and problem; 5.5e7 is its FP64 number).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PAPER_F32 = 1.2e8   # cell-updates/s, Tesla P100, VL+PLM+Roe, FP32 (paper Sec. 4.2(i))
PAPER_F64 = 5.5e7   # same, FP64
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def stage_bytes(stage: str, elem: int) -> float:
    """Algorithmic HBM bytes per cell of one stage launch (reads + writes of
    the arrays it touches, each element once)."""
    words = {
        "prim": 8 + 8,            # U(5) + B(3) in, W(8) out
        "flux_predict": 8 + 3 + 21,   # W(8) + normal B(3) in, F(3 x 7) out
        "flux_correct": 8 + 3 + 21,
        "emf_predict": 9 + 6 + 3,     # 3 x (mass, two EMFs) + v, Bc in, 3 edge EMFs out
        "emf_correct": 9 + 6 + 3,
        "half_step": 5 + 3 + 15 + 3 + 8 + 3,  # U, B, hydro F, E in; W, B out
        "final": 5 + 3 + 15 + 3 + 8,          # U, B, hydro F, E in; U, B out
    }[stage]
    return words * elem


def run_form(prec: str, n: int, steps: int, warmup: int, seed: int):
    import torch
    from paper_1804_03479_amd import inputs
    from paper_1804_03479_amd.mhd import Solver
    p = inputs.abc_problem(n, 0.01, seed=seed)
    s = Solver("vl", "plm", "roe", prec)
    W5 = torch.from_numpy(__import__("numpy").stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(__import__("numpy").stack([p["bx"], p["by"], p["bz"]]))
    lv = s.level_from_primitives(W5, B, p["dx"])
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        s.advance(lv, t_dev=t_dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        s.advance(lv, t_dev=t_dev)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    s.sync()
    cells = n ** 3
    stages = s.profile_step(lv, nrep=5)
    mx, _ = s.divb(lv)
    return dict(ms_per_step=ms / steps, value=cells * steps / (ms * 1e-3), stages=stages,
                max_divb_dx=mx * p["dx"], solver=s, level=lv)


def l1_vs_oracle(n: int, seed: int, nsteps: int, states: dict):
    """Relative L1 error (rho, e, B) of each GPU form after nsteps from the
    same initial state, against the FP64 oracle; also times the oracle."""
    import numpy as np
    import torch
    import oracle
    from paper_1804_03479_amd import inputs
    from paper_1804_03479_amd.mhd import Level, Solver
    p = inputs.abc_problem(n, 0.01, seed=seed)
    U, B = oracle.initial_state(p)
    dx = p["dx"]
    t0 = time.perf_counter()
    Uo, Bo = U, B
    for _ in range(nsteps):
        dt = oracle.cfl_dt(Uo, Bo, dx)
        Uo, Bo = oracle.step(Uo, Bo, dt, dx)
    t_cpu = time.perf_counter() - t0
    out = {}
    for prec in states:
        dtype = torch.float64 if prec == "f64" else torch.float32
        s = Solver("vl", "plm", "roe", prec)
        lv = Level(torch.from_numpy(U).to("cuda", dtype).contiguous(),
                   torch.from_numpy(B).to("cuda", dtype).contiguous(), dx)
        for _ in range(nsteps):
            s.advance(lv)
        torch.cuda.synchronize()
        Ug, Bg = lv.U.double().cpu().numpy(), lv.B.double().cpu().numpy()
        out[prec] = {
            "rho": float(np.abs(Ug[0] - Uo[0]).mean() / np.abs(Uo[0]).mean()),
            "e": float(np.abs(Ug[4] - Uo[4]).mean() / np.abs(Uo[4]).mean()),
            "B": float(np.abs(Bg - Bo).mean() / np.abs(Bo).mean()),
        }
        s.close()
    return out, t_cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle steps for the CPU baseline and L1 check")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    n = args.n
    cells = n ** 3
    forms = {}
    for prec in ("f64", "f32"):
        r = run_form(prec, n, args.steps, args.warmup, args.seed)
        forms[prec] = r

    head = forms["f32"]
    # roofline of the dominant stage kernel of the headline form
    stages = head["stages"]
    dom = max(stages, key=stages.get)
    elem = 4
    bytes_launch = stage_bytes(dom, elem) * cells
    achieved_gbs = bytes_launch / (stages[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "stage_ms": {k: round(v, 4) for k, v in stages.items()},
                "bytes_per_launch": bytes_launch}

    cpu = None
    l1 = None
    if not args.no_cpu:
        import oracle
        l1, t_cpu = l1_vs_oracle(n, args.seed, args.cpu_steps, forms)
        cpu = {"value": cells * args.cpu_steps / t_cpu, "unit": "cell-updates/s", "cores": oracle.get_threads(),
               "kind": "oracle", "sample": f"{n}^3 ABC box, VL+PLM+Roe FP64, {args.cpu_steps} steps incl. CFL"}

    line = {
        "metric": "cell-updates/s/GPU: FP64 vs FP32 vs MLP-flux at fixed L1 err; HBM GB/s",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": head["value"] / PAPER_F32,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"abc{n}_vl_plm_roe_ct", "cells": cells, "scheme": "VL+PLM(minmod)+Roe+CT",
                   "courant": 0.5, "noise": 0.01, "seed": args.seed},
        "forms": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                      "vs_paper": v["value"] / (PAPER_F32 if k == "f32" else PAPER_F64),
                      "max_divb_dx": v["max_divb_dx"],
                      "l1_vs_oracle": None if l1 is None else l1[k]} for k, v in forms.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    for v in forms.values():
        v["solver"].close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
