#!/usr/bin/env python3
"""Throughput of the unsplit MHD update on one MI355X.

Headline workload (the precision-form configuration): the ABC-field box of
the paper's Sec. 5.1(v)/4.2 (Eq. 20 with n = 1, A = B = C = 1, rho = p = 1)
on a 128^3 periodic grid with seeded uniform velocity noise of amplitude 0.1,
CTU + PPM + HLLD + CT, Courant 1/2 (summed over directions), gamma = 5/3,
timed in FP64 and FP32 side by side.  One step = CFL reduction + full update
(mhd_advance), state resident in HBM.  The headline value is the FP32 form.

Also timed, under "forms":
  * the FP32 form with double energy and low-beta double pressure recovery
    (f32_mixed), and the L1 distance of the FP32 and mixed forms from the
    FP64 form after --l1-steps steps;
  * the paper's own benchmark scheme (VL + PLM + Roe + CT, noise 0.01), for
    which the paper quotes 1.2e8 (FP32) and 5.5e7 (FP64) cell-updates/s on
    one Tesla P100 (Sec. 5.2(i));
  * the learned-flux form: a surrogate trained here on the GPU from captured
    interfaces, timed on the same box, with its L1 distance from the pure-HLLD
    run after --mlp-l1-steps steps (and the Roe run's, for scale), the HLLD
    fallback fraction and the MFMA rate of its flux stage;
  * the batched AMR form: the 128^3 root plus two refined levels of uneven
    group counts, shared dt, ghost refill, update and restriction of all
    levels replayed from one HIP graph, launch shapes autotuned per level.

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

PAPER_F32 = 1.2e8   # cell-updates/s, Tesla P100, VL+PLM+Roe, FP32 (paper Sec. 5.2(i))
PAPER_F64 = 5.5e7   # same, FP64
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK = 2500.0                          # TFLOP/s, dense BF16
MLP_FLOP_PER_FACE = 2 * (15 * 64 + 64 * 64 + 64 * 7)   # one 15-64-64-7 inference
# Vector ALU issue ceiling in wave64 instructions per second: the FP32 vector
# peak 157.3 TFLOP/s is 256 CUs x 2.4 GHz x 256 FLOP per clock, i.e. two
# 64-lane FMA instructions (128 FLOP each) per clock per CU; FP64 (78.6
# TFLOP/s) one.  Every counted VALU instruction takes one such slot.
VALU_PEAK_WAVE_INSTR = {4: 157.3e12 / 128.0, 8: 78.6e12 / 128.0}

# The words that define a cell update (Sec. 5.2 counts cell updates): the
# 5 conserved values and 3 face fields of a cell read once and written once.
CELL_UPDATE_WORDS = 16

# Scratch words per cell of each stage kernel: every array element the stage
# reads or writes, intermediates included, counted once (neighbour re-reads
# excluded).  Implementation traffic of the stage split, not algorithmic.
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


def abc_level(s, n: int, noise: float, seed: int):
    import numpy as np
    import torch
    from paper_1804_03479_amd import inputs
    p = inputs.abc_problem(n, noise, seed=seed)
    W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
    return s.level_from_primitives(W5, B, p["dx"]), p["dx"]


def run_form(wl: dict, prec: str, n: int, steps: int, warmup: int, seed: int, profile: bool,
             riemann: str | None = None, setup=None):
    import torch
    from paper_1804_03479_amd.mhd import Solver
    s = Solver(wl["scheme"], wl["recon"], riemann or wl["riemann"], prec)
    if setup is not None:
        setup(s)
    lv, dx = abc_level(s, n, wl["noise"], seed)
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        s.advance(lv, t_dev=t_dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    s.fallback_count()
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
    if (riemann or wl["riemann"]) in ("roe", "mlp"):
        out["fallback_faces_per_step"] = s.fallback_count() / steps
    if profile:
        out["stages"] = s.profile_step(lv, nrep=5)
    mx, _ = s.divb(lv)
    out["max_divb_dx"] = mx * dx
    s.close()
    return out


def l1_gpu_pair(wl: dict, n: int, seed: int, nsteps: int, ref: tuple, test: tuple, setup=None):
    """Relative L1 (rho, e, B) of form `test` against form `ref` (each a
    (prec, riemann) pair) after nsteps in lockstep on the GPU, both taking the
    reference's time step."""
    import numpy as np
    import torch
    from paper_1804_03479_amd.mhd import Solver
    a = Solver(wl["scheme"], wl["recon"], ref[1], ref[0])
    b = Solver(wl["scheme"], wl["recon"], test[1], test[0])
    if setup is not None:
        setup(b)
    la, dx = abc_level(a, n, wl["noise"], seed)
    lb, _ = abc_level(b, n, wl["noise"], seed)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    b.fallback_count()
    for _ in range(nsteps):
        a.cfl_dt_device(la, dt)
        a.step_devdt(la, dt)
        b.step_devdt(lb, dt)
    torch.cuda.synchronize()
    nfb = b.fallback_count()
    Ua, Ub = la.U.double().cpu().numpy(), lb.U.double().cpu().numpy()
    if lb.E64 is not None:
        Ub[4] = lb.E64.cpu().numpy()
    Ba, Bb = la.B.double().cpu().numpy(), lb.B.double().cpu().numpy()
    mx, _ = b.divb(lb)
    out = {"steps": nsteps, "vs": f"{ref[1]} {ref[0]}",
           "rho": float(np.abs(Ub[0] - Ua[0]).mean() / np.abs(Ua[0]).mean()),
           "e": float(np.abs(Ub[4] - Ua[4]).mean() / np.abs(Ua[4]).mean()),
           "B": float(np.abs(Bb - Ba).mean() / np.abs(Ba).mean()),
           "M": float(np.abs(Ub[1:4] - Ua[1:4]).mean() / np.abs(Ua[1:4]).mean()),
           "max_divb_dx": mx * dx, "fallback_faces": nfb}
    a.close()
    b.close()
    return out


def train_surrogate(n_capture: int, seed: int, n_samples: int, epochs: int):
    """Interface samples from CTU+PPM+HLLD runs of the ABC box, then Adam on
    the GPU (the library's own forward/backward kernels); returns weights."""
    import time as _t
    import torch
    from paper_1804_03479_amd import surrogate
    from paper_1804_03479_amd.mhd import MlpOps, Solver
    t0 = _t.perf_counter()
    # interfaces of 8 steps spread over a 500-step run (early, noisy flow and
    # the smoother flow of later times), another noise realisation than the
    # measured runs
    at = [0, 1, 100, 101, 250, 251, 450, 451]
    stride = max(1, (6 * n_capture ** 3 * len(at)) // (2 * n_samples))
    samples = surrogate.capture(n=n_capture, steps=452, noise=0.1, seed=seed + 1, stride=stride,
                                cap=2 * n_samples, capture_at=at)
    # strong (near-threshold) faces: a noise-0.3 run once compressions have
    # formed (its first steps carry velocity jumps only)
    strong = surrogate.capture(n=n_capture, steps=121, noise=0.3, seed=seed + 2, stride=2,
                               cap=n_samples, capture_at=[20, 40, 80, 120])
    samples = torch.cat([samples, strong])
    del strong
    s = Solver("ctu", "ppm", "mlp", "f32")
    ops = MlpOps(s)
    X, T, info = surrogate.training_set(ops, samples, n_samples, seed=seed)
    cls = info.pop("cls")
    params, hist = surrogate.train(ops, X, T, epochs=epochs, batch=4096, lr0=3e-3, seed=seed, cls=cls)
    torch.cuda.synchronize()
    s.close()
    return params, {"samples": n_samples, "captured": int(samples.shape[0]), "epochs": epochs,
                    "val_loss": hist[-1]["val_loss"], "val_loss_smooth": hist[-1].get("val_loss_smooth"),
                    "val_loss_strong": hist[-1].get("val_loss_strong"),
                    "val_loss_first_epoch": hist[0]["val_loss"],
                    "seconds": round(_t.perf_counter() - t0, 2), "mix": info}


def run_amr(n_root: int, counts, steps: int, warmup: int, seed: int, tune: bool):
    """Root + refined levels, shared dt, ghost refill, update, correction,
    restriction, all levels of a step replayed from one HIP graph; then the
    same hierarchy sub-cycled (level l: 2^l steps per root step)."""
    import gc
    import torch
    from paper_1804_03479_amd import autotune
    from paper_1804_03479_amd.amr import Hierarchy
    tuned = None
    if tune:
        h = Hierarchy(n_root, counts, prec="f32", seed=seed)
        tuned = autotune.tune(h, reps=3)
        h.close()
        del h
        gc.collect()
        torch.cuda.empty_cache()
    h = Hierarchy(n_root, counts, prec="f32", seed=seed)
    if tuned:
        h.set_launch(tuned["shapes"])
    st = h.stream
    cells = h.cells_per_level()

    def timed(fn, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(k):
            fn()
        e1.record(st)
        st.synchronize()
        return e0.elapsed_time(e1) / k

    for _ in range(warmup):
        h.step()
    ms_eager = timed(h.step, steps)
    g = h.capture()
    for _ in range(warmup):
        h.replay(g)
    ms_graph = timed(lambda: h.replay(g), steps)
    per_level = [autotune.time_level(h, lvl, reps=3) for lvl in range(len(h.levels))]
    divb = []
    for sv, lv in zip(h.solvers, h.levels):
        mx, _ = sv.divb(lv)
        divb.append(mx * lv.dx)
    h.close()
    del h
    gc.collect()
    torch.cuda.empty_cache()
    # sub-cycled: level l takes 2^l steps of dt_0 / 2^l per root step
    hs = Hierarchy(n_root, counts, prec="f32", seed=seed, subcycle=True)
    if tuned:
        hs.set_launch(tuned["shapes"])
    st = hs.stream
    for _ in range(warmup):
        hs.step()
    gs = hs.capture()
    for _ in range(warmup):
        hs.replay(gs)
    ms_sub = timed(lambda: hs.replay(gs), steps)
    upd = hs.updates_per_step()
    hs.close()
    return {"counts": list(counts), "cells_per_level": cells, "ms_per_step_graph": ms_graph,
            "ms_per_step_eager": ms_eager, "value": sum(cells) / (ms_graph * 1e-3),
            "per_level_ms": per_level,
            "per_level_value": [c / (t * 1e-3) for c, t in zip(cells, per_level)],
            "launch_shapes": None if not tuned else [list(x) for x in tuned["shapes"]],
            "autotune": None if not tuned else [
                {"shape_fields": ["blocks_per_cu", "threads", "batch", "lds_tiles"],
                 "table": [list(c) + [round(ms, 4)] for c, ms in zip(cands, mss)]}
                for cands, mss in zip(tuned["candidates"], tuned["ms"])],
            "max_divb_dx_listed": divb,
            "subcycled": {"updates_per_root_step": upd, "ms_per_root_step_graph": ms_sub,
                          "value": sum(upd) / (ms_sub * 1e-3)}}


def run_amr_criterion(n_root: int, steps: int, warmup: int, fraction: float = 0.187, t_cross: float = 1.3,
                      capacity: int = 2048):
    """The n = 2 ABC relaxation problem evolved on the root to t = 1.3 L/C_s
    (current sheets formed), then regridded by |curl B| dx / |B| > thr with
    thr chosen so that level 1 covers about `fraction` of the root (the
    paper's 18.7 % at that time); the same threshold lists level 2 from
    level 1.  Times the hierarchy from one HIP graph, shared dt and
    sub-cycled."""
    import math
    import numpy as np
    import torch
    from paper_1804_03479_amd import inputs
    from paper_1804_03479_amd.amr import Hierarchy
    from paper_1804_03479_amd.mhd import Solver
    p = inputs.abc_relaxation_problem(n_root)
    s = Solver("ctu", "ppm", "hlld", "f32")
    W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
    lv = s.level_from_primitives(W5, B, p["dx"])
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    t_stop = t_cross / math.sqrt(5.0 / 3.0)
    evolve = 0
    while float(t.item()) < t_stop:
        for _ in range(100):
            s.advance(lv, t_dev=t)
        evolve += 100
    torch.cuda.synchronize()
    # threshold for the wanted level-1 coverage (bisection on the device count)
    cand = (2 * n_root // 16) ** 3
    out = torch.zeros((cand, 3), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    wanted = torch.zeros(1, dtype=torch.int32, device="cuda")
    lo, hi = 0.0, 4.0
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        s.regrid_flag(lv, mid, 1, 16, out, cnt, wanted)
        if int(wanted.item()) > fraction * cand:
            lo = mid
        else:
            hi = mid
    thr = hi
    res = {"evolved_root_steps": evolve, "t_over_tcross": float(t.item()) * math.sqrt(5.0 / 3.0), "threshold": thr}
    for sub in (False, True):
        h = Hierarchy(n_root, [0, 0], prec="f32", subcycle=sub, capacity=capacity, problem=p)
        h.reset_root(lv.U, lv.B)
        h.regrid(thr)
        res["wanted"] = h.check_regrid()
        counts = h.group_counts()
        st = h.stream
        for _ in range(warmup):
            h.step()
        g = h.capture()
        for _ in range(warmup):
            h.replay(g)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            h.replay(g)
        e1.record(st)
        st.synchronize()
        ms = e0.elapsed_time(e1) / steps
        upd = h.updates_per_step()
        key = "subcycled" if sub else "shared"
        res[key] = {"ms_per_root_step_graph": ms, "updates_per_root_step": upd, "value": sum(upd) / (ms * 1e-3)}
        res["groups_per_level"] = counts
        res["volume_fraction_per_level"] = [c * 16 ** 3 / int(np.prod(x.shape))
                                            for c, x in zip(counts, h.levels[1:])]
        h.close()
        del h
        torch.cuda.empty_cache()
    s.close()
    return res


def run_c4(n_root: int, count: int, steps: int, warmup: int, seed: int, params, drift_root: int = 64,
           drift_count: int = 7, drift_steps: int = 100, oracle_steps: int = 0):
    """Full stack: FP32 CTU+PPM with the learned flux (HLLD fallback) on an
    AMR hierarchy (n_root^3 ABC root, noise 0.3, one refined level of
    `count` groups), `steps` root steps replayed from one HIP graph; energy
    budget and fallback fraction over the run.  Then the L1 drift of the same
    stack against the FP64 HLLD hierarchy at drift_root^3 + one level after
    drift_steps steps (root data, which holds the restricted fine data), and,
    with oracle_steps > 0, the drift of both against the oracle's two-level
    step after that many steps (each GPU hierarchy takes the oracle's dt)."""
    import numpy as np
    import torch
    from paper_1804_03479_amd.amr import Hierarchy
    from paper_1804_03479_amd.mhd import MlpOps
    h = Hierarchy(n_root, [count], "ctu", "ppm", "mlp", "f32", noise=0.3, seed=seed)
    for sv in h.solvers:
        MlpOps(sv).set_weights(params)
    st = h.stream
    e_start = h.s.sums(h.levels[0])
    fb0 = sum(sv.fallback_count() for sv in h.solvers)
    for _ in range(warmup):
        h.step()
    g = h.capture()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        h.replay(g)
    e1.record(st)
    st.synchronize()
    ms = e0.elapsed_time(e1) / steps
    total_steps = warmup + 1 + steps
    e_end = h.s.sums(h.levels[0])
    fb = sum(sv.fallback_count() for sv in h.solvers) - fb0
    cells = h.cells_per_level()
    mx = max(sv.divb(lv)[0] * lv.dx for sv, lv in zip(h.solvers, h.levels))
    h.close()
    del h
    torch.cuda.empty_cache()
    out = {"n_root": n_root, "groups": count, "cells_per_level": cells, "noise": 0.3, "steps": total_steps,
           "timed_steps": steps, "ms_per_step_graph": ms, "value": sum(cells) / (ms * 1e-3),
           "algorithmic_GBps": sum(cells) / (ms * 1e-3) * 64 / 1e9,
           "fallback_fraction": fb / (6.0 * sum(cells) * total_steps),
           "energy": {"E_T": [e_start[4], e_end[4]], "U_B": [e_start[5], e_end[5]], "U_V": [e_start[6], e_end[6]]},
           "E_T_drift": abs(e_end[4] - e_start[4]) / abs(e_start[4]), "max_divb_dx": mx}
    # drift of the stack against the FP64 HLLD hierarchy (same steps, same time)
    ref = Hierarchy(drift_root, [drift_count], "ctu", "ppm", "hlld", "f64", noise=0.3, seed=seed)
    run = Hierarchy(drift_root, [drift_count], "ctu", "ppm", "mlp", "f32", noise=0.3, seed=seed)
    for sv in run.solvers:
        MlpOps(sv).set_weights(params)
    for _ in range(drift_steps):
        ref.step()
        ref.stream.synchronize()
        run.step(dt_max=float(ref.dts[0].item()))
    run.stream.synchronize()
    Ur, Br = ref.levels[0].U.cpu().numpy(), ref.levels[0].B.cpu().numpy()
    Ug, Bg = run.levels[0].U.double().cpu().numpy(), run.levels[0].B.double().cpu().numpy()
    rel = lambda a, b: float(np.abs(a - b).mean() / np.abs(b).mean())   # noqa: E731
    out["l1_drift_vs_f64_hlld"] = {"root": drift_root, "groups": drift_count, "steps": drift_steps,
                                   "rho": rel(Ug[0], Ur[0]), "e": rel(Ug[4], Ur[4]), "B": rel(Bg, Br)}
    ref.close()
    run.close()
    if oracle_steps > 0:
        import oracle
        from oracle import amr as oamr
        from paper_1804_03479_amd import inputs
        ref = Hierarchy(drift_root, [drift_count], "ctu", "ppm", "hlld", "f64", noise=0.3, seed=seed)
        run = Hierarchy(drift_root, [drift_count], "ctu", "ppm", "mlp", "f32", noise=0.3, seed=seed)
        for sv in run.solvers:
            MlpOps(sv).set_weights(params)
        p = inputs.abc_problem(drift_root, 0.3, seed=seed)
        Uc, Bc = oracle.initial_state(p)
        g = ref.groups[0]
        Uf, Bf = oamr.initial_fine(Uc, Bc, g)
        t0 = time.perf_counter()
        for k in range(oracle_steps):
            Uc, Bc, Uf, Bf, dt = oamr.two_level_step(Uc, Bc, Uf, Bf, g, p["dx"])
            ref.step(dt_max=dt)
            run.step(dt_max=dt)
            if (k + 1) % 10 == 0:
                print(f"c4 oracle drift: step {k + 1} of {oracle_steps}", file=sys.stderr, flush=True)
        t_or = time.perf_counter() - t0
        ref.stream.synchronize()
        run.stream.synchronize()
        U64, B64 = ref.levels[0].U.cpu().numpy(), ref.levels[0].B.cpu().numpy()
        Ug, Bg = run.levels[0].U.double().cpu().numpy(), run.levels[0].B.double().cpu().numpy()
        out["l1_drift_vs_oracle"] = {
            "root": drift_root, "groups": drift_count, "steps": oracle_steps, "oracle_s": round(t_or, 1),
            "mlp_f32_stack": {"rho": rel(Ug[0], Uc[0]), "e": rel(Ug[4], Uc[4]), "B": rel(Bg, Bc)},
            "hlld_f64_hierarchy": {"rho": rel(U64[0], Uc[0]), "e": rel(U64[4], Uc[4]), "B": rel(B64, Bc)}}
        ref.close()
        run.close()
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
        E64 = torch.from_numpy(U[4].copy()).to("cuda") if prec == "f32_mixed" else None
        lv = Level(torch.from_numpy(U).to("cuda", dtype).contiguous(),
                   torch.from_numpy(B).to("cuda", dtype).contiguous(), dx, E64=E64)
        for _ in range(nsteps):
            s.advance(lv)
        torch.cuda.synchronize()
        Ug, Bg = lv.U.double().cpu().numpy(), lv.B.double().cpu().numpy()
        if E64 is not None:
            Ug[4] = E64.cpu().numpy()
        out[prec] = {
            "steps": nsteps,
            "rho": float(np.abs(Ug[0] - Uo[0]).mean() / np.abs(Uo[0]).mean()),
            "e": float(np.abs(Ug[4] - Uo[4]).mean() / np.abs(Uo[4]).mean()),
            "B": float(np.abs(Bg - Bo).mean() / np.abs(Bo).mean()),
        }
        s.close()
    return out, t_cpu


def l1_vs_oracle_run(wl: dict, n: int, seed: int, nsteps: int, precs, log_every: int = 20):
    """The FP64 oracle run for nsteps CFL steps on the host, then each GPU form
    stepped with the oracle's own dt sequence (so both sit at the same times);
    relative L1 (rho, e, B) of each form against the oracle and its max |div B|."""
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
    Uo, Bo, dts = U, B, []
    for k in range(nsteps):
        dt = oracle.cfl_dt(Uo, Bo, dx)
        dts.append(dt)
        Uo, Bo = oracle.step(Uo, Bo, dt, dx, **kw)
        if log_every and (k + 1) % log_every == 0:
            print(f"oracle step {k + 1}/{nsteps} ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    t_cpu = time.perf_counter() - t0
    out = {"steps": nsteps, "t": float(sum(dts)), "oracle_seconds": round(t_cpu, 1),
           "oracle_threads": oracle.get_threads()}
    for prec in precs:
        dtype = torch.float64 if prec == "f64" else torch.float32
        s = Solver(wl["scheme"], wl["recon"], wl["riemann"], prec)
        E64 = torch.from_numpy(U[4].copy()).to("cuda") if prec == "f32_mixed" else None
        lv = Level(torch.from_numpy(U).to("cuda", dtype).contiguous(),
                   torch.from_numpy(B).to("cuda", dtype).contiguous(), dx, E64=E64)
        for dt in dts:
            s.step(lv, dt)
        torch.cuda.synchronize()
        mx, _ = s.divb(lv)
        Ug, Bg = lv.U.double().cpu().numpy(), lv.B.double().cpu().numpy()
        if E64 is not None:
            Ug[4] = E64.cpu().numpy()
        out[prec] = {
            "rho": float(np.abs(Ug[0] - Uo[0]).mean() / np.abs(Uo[0]).mean()),
            "e": float(np.abs(Ug[4] - Uo[4]).mean() / np.abs(Uo[4]).mean()),
            "B": float(np.abs(Bg - Bo).mean() / np.abs(Bo).mean()),
            "max_divb_dx": mx * dx,
        }
        s.close()
    out["oracle_max_divb_dx"] = float(np.abs(oracle.divb(Bo, dx)).max() * dx)
    return out


def counter_record(name: str, workload: str, prec: str):
    """A committed counter summary (profiles/<name>.json) of this workload and
    precision, or None when the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for s in rec["sources"]:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if h.hexdigest() != rec["sources_sha256"] or rec["workload"] != workload or rec.get("prec") != prec:
        return None
    return rec


def roofline_of(stages: dict, step_ms: float, words: dict, elem: int, cells: int, workload: str, prec: str) -> dict:
    """HBM roofline of the dominant stage kernel (live hipEvent times on the
    library's stream): algorithmic bytes = 16 words per cell update x cells
    per launch; beside it the whole step at the same bytes, the stage's
    scratch traffic, the counter-measured traffic and the VALU issue rate."""
    dom = max(stages, key=stages.get)
    alg = CELL_UPDATE_WORDS * elem * cells
    achieved = alg / (stages[dom] * 1e-3) / 1e9
    step_rate = alg / (step_ms * 1e-3) / 1e9
    scratch = words[dom] * elem * cells
    hbm = counter_record("hbm_traffic", workload, prec)
    valu = counter_record("valu_counters", workload, prec)
    out = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if hbm is None else hbm["bytes_per_launch"].get(dom),
           "algorithmic_bytes_per_launch": alg,
           "step": {"achieved": round(step_rate, 1), "frac": round(step_rate / HBM_PEAK_GBS, 4),
                    "ms": round(step_ms, 4)},
           "scratch": {"words_per_cell": words[dom], "bytes_per_launch": scratch,
                       "achieved": round(scratch / (stages[dom] * 1e-3) / 1e9, 1)},
           "stage_ms": {k: round(v, 4) for k, v in stages.items()}}
    if valu is not None:
        peak = VALU_PEAK_WAVE_INSTR[elem]
        per = {}
        for k, n_instr in valu["wave_instructions_per_launch"].items():
            if k in stages:
                r = n_instr / (stages[k] * 1e-3)
                per[k] = {"wave_instructions": n_instr, "rate": round(r, 0), "frac": round(r / peak, 4)}
        out["valu"] = {"kernel": dom, "frac": per.get(dom, {}).get("frac"), "peak_wave_instr_per_s": peak,
                       "step_frac": round(sum(v["wave_instructions"] for v in per.values()) / (step_ms * 1e-3) / peak, 4),
                       "per_stage": per, "summary": valu.get("summary")}
    else:
        out["valu"] = None
    return out


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
    ap.add_argument("--oracle-l1-steps", type=int, default=0,
                    help="also run the FP64 oracle this many steps on the headline workload and report the "
                         "L1 of every precision form against it (200: the precision form's full length, "
                         "about 2 minutes on 16 host cores)")
    ap.add_argument("--only", choices=["ctu", "vl", "mlp", "amr"], default=None, help="time one workload only")
    ap.add_argument("--l1-steps", type=int, default=200,
                    help="steps of the FP32 / mixed forms against the FP64 form (precision form)")
    ap.add_argument("--mlp-l1-steps", type=int, default=500, help="steps of the MLP form against pure HLLD")
    ap.add_argument("--mlp-samples", type=int, default=10_000_000)
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--amr-counts", default="511,1024",
                    help="patch groups (16^3 cells) of each refined level; also runs 7,64")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--c4-steps", type=int, default=1000,
                    help="root steps of the full-stack form (AMR + learned flux, FP32); 0 skips it")
    ap.add_argument("--c4-oracle-steps", type=int, default=0,
                    help="steps of the full stack's drift against the oracle's two-level step at 64^3 + 7 "
                         "groups (the oracle takes about 3 s per step on 16 host cores)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line, print one line with cell-updates/s of the CTU form "
                         "over grid sizes 32^3 .. 512^3 (FP32) and .. 384^3 (FP64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
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
    if args.sweep:
        sweep = {}
        for prec, sizes in (("f32", (32, 64, 96, 128, 192, 256, 384, 512)), ("f64", (32, 64, 96, 128, 192, 256, 384))):
            for key in ("ctu", "vl"):
                for n_ in sizes:
                    steps = max(5, min(args.steps, int(3e8 / n_ ** 3)))
                    r = run_form(WORKLOADS[key], prec, n_, steps, args.warmup, args.seed, profile=False)
                    sweep[f"{key}_{prec}_{n_}"] = {"n": n_, "steps": steps, "value": r["value"],
                                                   "ms_per_step": r["ms_per_step"]}
                    print(f"sweep {key} {prec} {n_}^3: {r['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)
        print(json.dumps({"metric": "cell-updates/s/GPU", "unit": "cell-updates/s", "sweep": sweep,
                          "config": {"workloads": {k: WORKLOADS[k]["label"] for k in ("ctu", "vl")}}}))
        return
    n = args.n
    cells = n ** 3
    todo = ["ctu", "vl", "mlp", "amr"] if args.only is None else [args.only]
    results = {}
    forms = {}
    if "ctu" in todo:
        precs = ("f64", "f32", "f32_mixed")
        results["ctu"] = {prec: run_form(WORKLOADS["ctu"], prec, n, args.steps, args.warmup, args.seed,
                                         profile=(prec == "f32")) for prec in precs}
    if "vl" in todo:
        results["vl"] = {prec: run_form(WORKLOADS["vl"], prec, n, args.steps, args.warmup, args.seed,
                                        profile=(prec == "f32")) for prec in ("f64", "f32")}
    head_key = "ctu" if "ctu" in results else ("vl" if "vl" in results else None)

    cpu = None
    l1 = {}
    if not args.no_cpu and head_key is not None:
        import oracle
        wl = WORKLOADS[head_key]
        precs = ("f64", "f32", "f32_mixed") if head_key == "ctu" else ("f64", "f32")
        l1[head_key], t_cpu = l1_vs_oracle(wl, n, args.seed, args.cpu_steps, precs)
        cpu = {"value": cells * args.cpu_steps / t_cpu, "unit": "cell-updates/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"{n}^3 ABC box, {wl['label']} FP64, {args.cpu_steps} steps incl. CFL"}
        # the same oracle on one core (one step incl. CFL) and the host CPU
        from paper_1804_03479_amd import inputs
        p = inputs.abc_problem(n, wl["noise"], seed=args.seed)
        U, B = oracle.initial_state(p)
        threads = oracle.get_threads()
        oracle.set_threads(1)
        t0 = time.perf_counter()
        dt = oracle.cfl_dt(U, B, p["dx"])
        oracle.step(U, B, dt, p["dx"], scheme=oracle.CTU if wl["scheme"] == "ctu" else oracle.VL,
                    recon=oracle.PPM if wl["recon"] == "ppm" else oracle.PLM,
                    riemann={"roe": oracle.ROE, "hlle": oracle.HLLE, "hlld": oracle.HLLD}[wl["riemann"]])
        cpu["value_1_core"] = cells / (time.perf_counter() - t0)
        oracle.set_threads(threads)
        try:
            cpu["cpu_model"] = next(line.split(":", 1)[1].strip() for line in open("/proc/cpuinfo")
                                    if line.startswith("model name"))
        except (OSError, StopIteration):
            cpu["cpu_model"] = None

    for key, r in results.items():
        wl = WORKLOADS[key]
        for prec, v in r.items():
            e = {"workload": wl["name"].format(n=n), "value": v["value"], "ms_per_step": v["ms_per_step"],
                 "max_divb_dx": v["max_divb_dx"], "l1_vs_oracle": l1.get(key, {}).get(prec)}
            if "fallback_faces_per_step" in v:
                e["fallback_faces_per_step"] = v["fallback_faces_per_step"]
            if key == "vl":
                e["vs_paper"] = v["value"] / (PAPER_F32 if prec == "f32" else PAPER_F64)
            if key == "ctu" and prec != "f64" and args.l1_steps > 0:
                e["l1_vs_f64_form"] = l1_gpu_pair(wl, n, args.seed, args.l1_steps, ("f64", "hlld"), (prec, "hlld"))
            forms[f"{key}_{prec}"] = e
        if key != head_key and "stages" in r["f32"]:
            forms[f"{key}_f32"]["stage_ms"] = {k: round(x, 4) for k, x in r["f32"]["stages"].items()}

    if "ctu" in results:
        # the reconstruction stage on LDS tiles (a launch-shape option): same
        # bits, timed beside the per-cell form
        wl = WORKLOADS["ctu"]
        tiles = {}
        for prec in ("f32", "f64"):
            r = run_form(wl, prec, n, args.steps, args.warmup, args.seed, profile=True,
                         setup=lambda s: s.set_launch(tiles=1))
            base = results["ctu"][prec]
            tiles[prec] = {"ms_per_step": round(r["ms_per_step"], 4), "states_ms": round(r["stages"]["states"], 4),
                           "per_cell_states_ms": round(base["stages"]["states"], 4) if "stages" in base else None,
                           "step_vs_per_cell": round(base["ms_per_step"] / r["ms_per_step"], 4)}
        forms["ctu_lds_tiles"] = {"workload": wl["name"].format(n=n), "tile": [16, 4, 4], **tiles}

    if args.oracle_l1_steps > 0 and head_key is not None:
        precs = ("f64", "f32", "f32_mixed") if head_key == "ctu" else ("f64", "f32")
        forms[f"{head_key}_l1_vs_oracle_full"] = l1_vs_oracle_run(WORKLOADS[head_key], n, args.seed,
                                                                   args.oracle_l1_steps, precs)

    if "mlp" in todo:
        from paper_1804_03479_amd.mhd import MlpOps
        params, tinfo = train_surrogate(n, args.seed, args.mlp_samples, args.mlp_epochs)
        setup = lambda s: MlpOps(s).set_weights(params)  # noqa: E731
        wl = WORKLOADS["ctu"]
        r = run_form(wl, "f32", n, args.steps, args.warmup, args.seed, profile=True, riemann="mlp", setup=setup)
        e = {"workload": f"abc{n}_ctu_ppm_mlp_hlld_fallback_ct", "value": r["value"], "ms_per_step": r["ms_per_step"],
             "max_divb_dx": r["max_divb_dx"], "fallback_faces_per_step": r["fallback_faces_per_step"],
             "fallback_fraction": r["fallback_faces_per_step"] / (6 * cells), "training": tinfo,
             "stage_ms": {k: round(x, 4) for k, x in r["stages"].items()}}
        if args.mlp_l1_steps > 0:
            e["l1_vs_hlld"] = l1_gpu_pair(wl, n, args.seed, args.mlp_l1_steps, ("f32", "hlld"), ("f32", "mlp"),
                                          setup=setup)
            e["l1_roe_vs_hlld"] = l1_gpu_pair(wl, n, args.seed, args.mlp_l1_steps, ("f32", "hlld"), ("f32", "roe"))
        if "ctu" in results:
            e["speed_vs_hlld_f32"] = r["value"] / results["ctu"]["f32"]["value"]
        # the network's MFMA work in the predictor flux stage: 3 faces per cell
        t_flux = r["stages"]["flux_predict"] * 1e-3
        flops = 3 * cells * MLP_FLOP_PER_FACE
        e["mfma"] = {"kernel": "flux_predict", "achieved": round(flops / t_flux / 1e12, 2), "peak": MFMA_BF16_PEAK,
                     "unit": "TFLOP/s", "frac": round(flops / t_flux / 1e12 / MFMA_BF16_PEAK, 5),
                     "flop_per_face": MLP_FLOP_PER_FACE}
        forms["ctu_f32_mlp"] = e
        if args.c4_steps > 0:
            r = run_c4(2 * n, 511, args.c4_steps, args.warmup, args.seed, params,
                       oracle_steps=args.c4_oracle_steps)
            r["workload"] = f"abc{2 * n}_root_plus_1_level_ctu_ppm_mlp_hlld_fallback_ct_f32"
            forms["c4_full_stack"] = r

    if "amr" in todo:
        counts = [int(x) for x in args.amr_counts.split(",")]
        for cs in (counts, [7, 64]):
            r = run_amr(n, cs, args.steps, args.warmup, args.seed, tune=not args.no_tune)
            r["workload"] = f"abc{n}_root_plus_{len(cs)}_levels_ctu_ppm_hlld_ct_f32"
            forms["amr_f32_" + "_".join(map(str, cs))] = r
        r = run_amr_criterion(n, args.steps, args.warmup)
        r["workload"] = f"abc_n2_{n}_root_plus_2_levels_criterion_lists_ctu_ppm_hlld_ct_f32"
        forms["amr_f32_criterion"] = r

    if head_key is None:
        print(json.dumps({"forms": forms}))
        return
    head = results[head_key]["f32"]
    words = CTU_WORDS if head_key == "ctu" else STAGE_WORDS
    roofline = roofline_of(head["stages"], head["ms_per_step"], words, 4, cells,
                           WORKLOADS[head_key]["name"].format(n=n), "f32")
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
