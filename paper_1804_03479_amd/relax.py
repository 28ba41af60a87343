"""The ABC relaxation run of paper Sec. 5.1(v) on one GPU.

The n = 2 ABC field with the eigenmode of Eqs. 21-23 and a diagonal drift
(inputs.abc_relaxation_problem) is advanced with the CTU + PPM + HLLD + CT
update on a uniform periodic grid; at sample times the run records the
volume totals of the library (total energy E_T, magnetic energy U_B, flow
energy U_V, double-precision reductions on the device) and, from a copy of
the face field, the magnetic helicity H = int A.B dV and the share of U_B in
the Fourier shells |k| L / 2 pi = 1, sqrt 2, 2.  Expected from the paper:
E_T constant, U_B falling to about half of U_B(0) (the n = 1 ABC state
carries half the energy of the n = 2 one at equal helicity,
H = U_B L / (pi n)), H nearly constant, and a relaxed state dominated by
the n = 1 shell with the ABC pattern of Eq. 24.

The analysis (FFT helicity, spectra) runs on the host with numpy: it is
diagnostics of the run, not part of the update.

    python -m paper_1804_03479_amd.relax --n 64 --t-end 31
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import inputs
from .mhd import Solver


def cell_centred(B: np.ndarray) -> np.ndarray:
    """(3, n, n, n) face field -> cell-centred field (mean of the two faces)."""
    out = np.empty_like(B)
    for a in range(3):
        ax = 2 - a                      # B[a] is [z][y][x]: component a steps along axis 2 - a
        out[a] = 0.5 * (B[a] + np.roll(B[a], -1, axis=ax))
    return out


def _wavevectors(n: int, L: float):
    k = 2.0 * math.pi * np.fft.fftfreq(n, d=L / n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    return kx, ky, kz


def helicity(Bc: np.ndarray, L: float = 1.0) -> float:
    """int A.B dV over the periodic box, A in the Coulomb gauge
    (A_k = i k x B_k / |k|^2), from the cell-centred field Bc."""
    n = Bc.shape[1]
    Bk = np.fft.fftn(Bc, axes=(1, 2, 3))
    kx, ky, kz = _wavevectors(n, L)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[0, 0, 0] = 1.0
    cx = ky * Bk[2] - kz * Bk[1]
    cy = kz * Bk[0] - kx * Bk[2]
    cz = kx * Bk[1] - ky * Bk[0]
    Ak = [1j * c / k2 for c in (cx, cy, cz)]
    for a in Ak:
        a[0, 0, 0] = 0.0
    s = sum(np.vdot(Bk[m], Ak[m]) for m in range(3)).real      # sum_k conj(B_k) . A_k
    dV = (L / n) ** 3
    return float(s / n ** 3 * dV)


def shell_fractions(Bc: np.ndarray, L: float = 1.0, shells=(1.0, math.sqrt(2.0), 2.0)):
    """Share of sum |B_k|^2 in each shell |k| L / 2 pi = s (within 1e-6)."""
    n = Bc.shape[1]
    Bk = np.fft.fftn(Bc, axes=(1, 2, 3))
    kx, ky, kz = _wavevectors(n, L)
    kn = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2) * L / (2.0 * math.pi)
    p = (np.abs(Bk) ** 2).sum(0)
    tot = p.sum()
    return {f"{s:.4f}": float(p[np.abs(kn - s) < 1e-6].sum() / tot) for s in shells}


def abc1_amplitudes(Bc: np.ndarray, L: float = 1.0):
    """Amplitudes (A, B, C) of an n = 1 ABC pattern (Eq. 20 form, any
    phases): A from the z-modes of Bx and By, B from the x-modes of By and
    Bz, C from the y-modes of Bz and Bx."""
    n = Bc.shape[1]
    Bk = np.fft.fftn(Bc, axes=(1, 2, 3)) / n ** 3
    # array axes: [component][z][y][x]; the mode k = 1 along one axis
    zmode = lambda m: abs(Bk[m][1, 0, 0])      # noqa: E731
    ymode = lambda m: abs(Bk[m][0, 1, 0])      # noqa: E731
    xmode = lambda m: abs(Bk[m][0, 0, 1])      # noqa: E731
    return (zmode(0) + zmode(1), xmode(1) + xmode(2), ymode(2) + ymode(0))


def run(n: int = 64, prec: str = "f32", t_end: float = 31.0, samples: int = 62, gamma: float = 5.0 / 3.0,
        scheme=("ctu", "ppm", "hlld"), perturb: bool = True, drift: bool = True, noise: float = 1e-3,
        seed: int = 0, log=None) -> dict:
    """Advance the relaxation problem to t_end sound-crossing times L / C_s;
    returns the sampled diagnostics (times in units of L / C_s)."""
    p = inputs.abc_relaxation_problem(n, gamma=gamma, perturb=perturb, drift=drift, noise=noise, seed=seed)
    cs = math.sqrt(gamma)                     # rho0 = P0 = 1
    t_cross = 1.0 / cs
    s = Solver(*scheme, prec, gamma=gamma)
    W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
    lv = s.level_from_primitives(W5, B, p["dx"])
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    rows = []

    def sample(steps):
        torch.cuda.synchronize()
        sums = s.sums(lv)
        Bc = cell_centred(lv.B.double().cpu().numpy())
        mx, _ = s.divb(lv)
        row = {"t": float(t.item()) / t_cross, "steps": steps, "E_T": sums[4], "U_B": sums[5], "U_V": sums[6],
               "H": helicity(Bc), "shells": shell_fractions(Bc), "max_divb_dx": mx * p["dx"]}
        rows.append(row)
        if log:
            log(f"t = {row['t']:.2f} L/Cs  steps {steps}  U_B {row['U_B']:.4f}  U_V {row['U_V']:.4f}  "
                f"H {row['H']:.5f}  shells {row['shells']}")
        return Bc

    sample(0)
    steps = 0
    dt0 = s.cfl_dt(lv)
    every = t_end * t_cross / samples
    t0 = time.perf_counter()
    while float(t.item()) < t_end * t_cross:
        chunk = max(1, int(every / dt0))
        for _ in range(chunk):
            s.advance(lv, t_dev=t)
        steps += chunk
        Bc = sample(steps)
        dt0 = s.cfl_dt(lv)
    wall = time.perf_counter() - t0
    amps = abc1_amplitudes(Bc)
    first, last = rows[0], rows[-1]
    s.close()
    return {
        "n": n, "prec": prec, "scheme": "+".join(scheme), "noise": noise, "seed": seed, "t_end": last["t"],
        "steps": steps,
        "seconds": round(wall, 2), "cell_updates_per_s": n ** 3 * steps / wall,
        "E_T_drift": max(abs(r["E_T"] - first["E_T"]) for r in rows) / first["E_T"],
        "U_B_end_over_start": last["U_B"] / first["U_B"],
        "U_V_max_over_U_B0": max(r["U_V"] for r in rows) / first["U_B"],
        "H_end_over_start": last["H"] / first["H"],
        "H_min_over_start": min(r["H"] for r in rows) / first["H"],
        "shells_start": first["shells"], "shells_end": last["shells"],
        "abc1_amplitudes_end": [float(a) for a in amps],
        "abc1_sum_sq_end": float(sum(a * a for a in amps)),
        "max_divb_dx": max(r["max_divb_dx"] for r in rows),
        "series": rows,
    }


def run_amr(n_root: int = 64, levels: int = 2, threshold: float = 1.43, t_end: float = 31.0, samples: int = 31,
            regrid_every: int = 8, prec: str = "f32", capacity: int = 4096, noise: float = 1e-3, seed: int = 0,
            gamma: float = 5.0 / 3.0, log=None) -> dict:
    """The relaxation run on an AMR hierarchy (the paper's configuration:
    a root grid plus refined levels following the current sheets): sub-cycled
    levels regridded every regrid_every root steps by |curl B| dh / |B| >
    threshold on each parent level (R28's calibrated constant by default).
    Diagnostics from the root, which holds the restricted finer data."""
    import math as _m
    from .amr import Hierarchy
    p = inputs.abc_relaxation_problem(n_root, gamma=gamma, noise=noise, seed=seed)
    t_cross = 1.0 / _m.sqrt(gamma)
    h = Hierarchy(n_root, [0] * levels, "ctu", "ppm", "hlld", prec, subcycle=True, capacity=capacity, problem=p)
    h.regrid(threshold)
    h.check_regrid()
    rows = []

    def sample(t, steps):
        sums = h.s.sums(h.levels[0])
        Bc = cell_centred(h.levels[0].B.double().cpu().numpy())
        row = {"t": t / t_cross, "root_steps": steps, "E_T": sums[4], "U_B": sums[5], "U_V": sums[6],
               "H": helicity(Bc), "shells": shell_fractions(Bc), "groups": h.group_counts()}
        rows.append(row)
        if log:
            log(f"t = {row['t']:.2f} L/Cs  root steps {steps}  U_B {row['U_B']:.4f}  H {row['H']:.5f}  "
                f"groups {row['groups']}")
        return Bc

    sample(0.0, 0)
    t, steps = 0.0, 0
    t0 = time.perf_counter()
    for k in range(1, samples + 1):
        stop = t_end * t_cross * k / samples
        while t < stop * (1.0 - 1e-12):
            if steps and steps % regrid_every == 0:
                h.regrid(threshold)
                h.check_regrid()
            h.step(dt_max=stop - t)
            h.stream.synchronize()
            t += float(h.dts[0].item())
            steps += 1
        Bc = sample(t, steps)
    wall = time.perf_counter() - t0
    divb = [h.solvers[i].divb(lv)[0] * lv.dx for i, lv in enumerate(h.levels)]
    h.close()
    first, last = rows[0], rows[-1]
    amps = abc1_amplitudes(Bc)
    return {"n_root": n_root, "levels": levels, "threshold": threshold, "prec": prec, "noise": noise,
            "t_end": last["t"], "root_steps": steps, "seconds": round(wall, 2),
            "E_T_drift": max(abs(r["E_T"] - first["E_T"]) for r in rows) / first["E_T"],
            "U_B_end_over_start": last["U_B"] / first["U_B"], "H_end_over_start": last["H"] / first["H"],
            "shells_end": last["shells"], "abc1_amplitudes_end": [float(a) for a in amps],
            "abc1_sum_sq_end": float(sum(a * a for a in amps)),
            "max_groups": [max(r["groups"][i] for r in rows) for i in range(levels)],
            "max_divb_dx": divb, "series": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--prec", default="f32")
    ap.add_argument("--t-end", type=float, default=31.0)
    ap.add_argument("--samples", type=int, default=62)
    ap.add_argument("--noise", type=float, default=1e-3, help="velocity noise in units of C_s")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--series", action="store_true", help="include the sampled time series")
    ap.add_argument("--amr-levels", type=int, default=0, help="run on an AMR hierarchy with this many levels")
    ap.add_argument("--threshold", type=float, default=1.43)
    args = ap.parse_args()
    import sys
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    if args.amr_levels:
        r = run_amr(args.n, args.amr_levels, args.threshold, args.t_end, args.samples, prec=args.prec,
                    noise=args.noise, seed=args.seed, log=log)
    else:
        r = run(args.n, args.prec, args.t_end, args.samples, noise=args.noise, seed=args.seed, log=log)
    if not args.series:
        r.pop("series")
    print(json.dumps(r))


if __name__ == "__main__":
    main()
