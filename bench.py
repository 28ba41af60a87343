#!/usr/bin/env python3
"""Throughput of the unsplit MHD update on one MI355X.

Headline workload (the precision-form configuration): the ABC-field box of
the paper's Sec. 4.1(v)/4.2 (Eq. 20 with n = 1, A = B = C = 1, rho = p = 1)
on a 128^3 periodic grid with seeded uniform velocity noise of amplitude 0.1,
CTU + PPM + HLLD + CT, Courant 1/2 (summed over directions), gamma = 5/3,
timed in FP64 and FP32 side by side.  One step = CFL reduction + full update
(mhd_advance), state resident in HBM.  The headline value is the FP32 form.

Also timed: the paper's own benchmark scheme (VL + PLM + Roe + CT, noise
0.01), for which the paper quotes 1.2e8 (FP32) and 5.5e7 (FP64)
cell-updates/s on one Tesla P100 (Sec. 4.2(i)).

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

# Algorithmic words per cell of each stage kernel: every array element the
# stage must read or write, counted once (neighbour re-reads excluded).
STAGE_WORDS = {
    "prim": 8 + 8,                        # U(5) + B(3) in, W(8) out
    "states": 8 + 3 + 42,                 # W, B in; QL, QR (2 x 3 x 7) out
    "flux_predict": 8 + 3 + 21,           # VL: W, B in, F out
    "flux_correct": 8 + 3 + 21,           # VL: Wh, Bh in, F out
    "emf_predict": 9 + 6 + 3,             # mass flux + 2 EMFs per face, v and Bc in; 3 edge EMFs out
    "emf_correct": 9 + 6 + 3,
    "half_step": 5 + 3 + 15 + 3 + 8 + 3,  # U, B, hydro F, E in; Wh, Bh out
    "final": 5 + 3 + 15 + 3 + 8,          # U, B, hydro F, E in; U, B out
}
CTU_WORDS = dict(STAGE_WORDS)
CTU_WORDS.update({
    "flux_predict": 42 + 3 + 21,          # QL, QR, B in; F1 out
    "flux_correct": 42 + 15 + 3 + 3 + 3 + 21,  # QL, QR, hydro F1, E, B, Bh in; F2 out
})

WORKLOADS = {
    "ctu": dict(scheme="ctu", recon="ppm", riemann="hlld", noise=0.1,
                name="abc{n}_ctu_ppm_hlld_ct", label="CTU+PPM+HLLD+CT"),
    "vl": dict(scheme="vl", recon="plm", riemann="roe", noise=0.01,
               name="abc{n}_vl_plm_roe_ct", label="VL+PLM(minmod)+Roe+CT"),
}


def run_form(wl: dict, prec: str, n: int, steps: int, warmup: int, seed: int, profile: bool):
    import numpy as np
    import torch
    from paper_1804_03479_amd import inputs
    from paper_1804_03479_amd.mhd import Solver
    p = inputs.abc_problem(n, wl["noise"], seed=seed)
    s = Solver(wl["scheme"], wl["recon"], wl["riemann"], prec)
    W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
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
    out = dict(ms_per_step=ms / steps, value=cells * steps / (ms * 1e-3))
    if profile:
        out["stages"] = s.profile_step(lv, nrep=5)
    mx, _ = s.divb(lv)
    out["max_divb_dx"] = mx * p["dx"]
    s.close()
    return out


def l1_vs_oracle(wl: dict, n: int, seed: int, nsteps: int, precs):
    """Relative L1 error (rho, e, B) of each GPU form after nsteps from the
    same initial state against the FP64 oracle; returns the oracle time too."""
    import numpy as np
    import torch
    import oracle
    from paper_1804_03479_amd import inputs
    from paper_1804_03479_amd.mhd import Level, Solver
    p = inputs.abc_problem(n, wl["noise"], seed=seed)
    U, B = oracle.initial_state(p)
    dx = p["dx"]
    kw = dict(scheme=oracle.CTU if wl["scheme"] == "ctu" else oracle.VL,
              recon=oracle.PPM if wl["recon"] == "ppm" else oracle.PLM,
              riemann={"roe": oracle.ROE, "hlle": oracle.HLLE, "hlld": oracle.HLLD}[wl["riemann"]])
    t0 = time.perf_counter()
    Uo, Bo = U, B
    for _ in range(nsteps):
        dt = oracle.cfl_dt(Uo, Bo, dx)
        Uo, Bo = oracle.step(Uo, Bo, dt, dx, **kw)
    t_cpu = time.perf_counter() - t0
    out = {}
    for prec in precs:
        dtype = torch.float64 if prec == "f64" else torch.float32
        s = Solver(wl["scheme"], wl["recon"], wl["riemann"], prec)
        lv = Level(torch.from_numpy(U).to("cuda", dtype).contiguous(),
                   torch.from_numpy(B).to("cuda", dtype).contiguous(), dx)
        for _ in range(nsteps):
            s.advance(lv)
        torch.cuda.synchronize()
        Ug, Bg = lv.U.double().cpu().numpy(), lv.B.double().cpu().numpy()
        out[prec] = {
            "steps": nsteps,
            "rho": float(np.abs(Ug[0] - Uo[0]).mean() / np.abs(Uo[0]).mean()),
            "e": float(np.abs(Ug[4] - Uo[4]).mean() / np.abs(Uo[4]).mean()),
            "B": float(np.abs(Bg - Bo).mean() / np.abs(Bo).mean()),
        }
        s.close()
    return out, t_cpu


def measured_traffic(workload: str, kernel: str):
    """Counter-measured HBM bytes per launch of a stage (profiles/hbm_traffic.json),
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for s in rec["sources"]:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if h.hexdigest() != rec["sources_sha256"] or rec["workload"] != workload:
        return None
    return rec["bytes_per_launch"].get(kernel)


def roofline_of(stages: dict, words: dict, elem: int, cells: int, workload: str) -> dict:
    dom = max(stages, key=stages.get)
    bytes_launch = words[dom] * elem * cells
    achieved = bytes_launch / (stages[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload, dom),
            "stage_ms": {k: round(v, 4) for k, v in stages.items()}, "bytes_per_launch": bytes_launch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle steps for the CPU baseline and L1 check")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB of a plain device-to-device copy run first (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["ctu", "vl"], default=None, help="time one workload only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calib_copy > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrate the HBM traffic counters of the MHD kernels
        nel = args.calib_copy * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    cells = n ** 3
    results = {}
    for key in (["ctu", "vl"] if args.only is None else [args.only]):
        wl = WORKLOADS[key]
        results[key] = {prec: run_form(wl, prec, n, args.steps, args.warmup, args.seed, profile=(prec == "f32"))
                        for prec in ("f64", "f32")}
    head_key = "ctu" if "ctu" in results else "vl"
    head = results[head_key]["f32"]
    words = CTU_WORDS if head_key == "ctu" else STAGE_WORDS
    roofline = roofline_of(head["stages"], words, 4, cells, WORKLOADS[head_key]["name"].format(n=n))

    cpu = None
    l1 = {}
    if not args.no_cpu:
        import oracle
        wl = WORKLOADS[head_key]
        l1[head_key], t_cpu = l1_vs_oracle(wl, n, args.seed, args.cpu_steps, ("f64", "f32"))
        cpu = {"value": cells * args.cpu_steps / t_cpu, "unit": "cell-updates/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"{n}^3 ABC box, {wl['label']} FP64, {args.cpu_steps} steps incl. CFL"}

    forms = {}
    for key, r in results.items():
        wl = WORKLOADS[key]
        for prec, v in r.items():
            e = {"workload": wl["name"].format(n=n), "value": v["value"], "ms_per_step": v["ms_per_step"],
                 "max_divb_dx": v["max_divb_dx"], "l1_vs_oracle": l1.get(key, {}).get(prec)}
            if key == "vl":
                e["vs_paper"] = v["value"] / (PAPER_F32 if prec == "f32" else PAPER_F64)
            forms[f"{key}_{prec}"] = e
        if key != head_key and "stages" in r["f32"]:
            forms[f"{key}_f32"]["stage_ms"] = {k: round(x, 4) for k, x in r["f32"]["stages"].items()}

    wl = WORKLOADS[head_key]
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
        "vs_baseline": None if head_key == "ctu" else head["value"] / PAPER_F32,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"].format(n=n), "cells": cells, "scheme": wl["label"], "courant": 0.5,
                   "noise": wl["noise"], "seed": args.seed},
        "forms": forms,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
