"""The Orszag-Tang vortex with AMR against uniform grids (paper
Sec. 5.1(iii)), on one GPU.

The 2D vortex (inputs.orszag_tang) runs on periodic slabs uniform along z:
an AMR hierarchy (root n^2, `levels` refined levels regridded every few root
steps by the criterion |J|/|B| > C / dh(k), i.e. |curl B| dh / |B| > C on
the parent level; C = 3.2 in the paper) with sub-cycled levels, a uniform
grid at the finest level's resolution, and a uniform grid at the root's.
At t_end (0.5 L / C_s in the paper) all three are compared on the root
grid: the uniform fine run averaged onto root cells (cells: volume means;
faces: area means) is the reference, and the AMR root holds the restricted
finest data wherever it is refined.  Reported: relative L1 differences of
gas and magnetic pressure from the reference (over the whole grid and over
the root cells under the finest level), the fraction of root cells
whose AMR / reference pressure ratios lie within 5 %, and the volume
fraction of each refined level (the paper's figures: 24.0 %, 8.5 %, 3.3 %
with 3 levels on a 256^2 root).

    python -m paper_1804_03479_amd.orszag_tang --n 128 --levels 2
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import inputs
from .amr import Hierarchy
from .mhd import Solver

GAMMA = 5.0 / 3.0


def _uniform(n: int, t_end: float, prec: str, scheme):
    p = inputs.orszag_tang(n, nz=4)
    s = Solver(*scheme, prec)
    W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
    lv = s.level_from_primitives(W5, B, p["dx"])
    t, steps = 0.0, 0
    while t < t_end * (1.0 - 1e-12):
        dt = min(s.cfl_dt(lv), t_end - t)
        s.step(lv, dt)
        t += dt
        steps += 1
    torch.cuda.synchronize()
    U, Bf = lv.U[:, 0].double().cpu().numpy(), lv.B[:, 0].double().cpu().numpy()
    s.close()
    return U, Bf, steps


def onto(U, B, r):
    """(5, ny, nx) cells and (3, ny, nx) faces of a z-uniform slab averaged
    onto a grid r times coarser in x and y."""
    ny, nx = U.shape[1:]
    Uc = U.reshape(5, ny // r, r, nx // r, r).mean(axis=(2, 4))
    bx = B[0][:, ::r].reshape(ny // r, r, nx // r).mean(axis=1)          # x-faces at coarse x
    by = B[1][::r, :].reshape(ny // r, nx // r, r).mean(axis=2)          # y-faces at coarse y
    bz = B[2].reshape(ny // r, r, nx // r, r).mean(axis=(1, 3))
    return Uc, np.stack([bx, by, bz])


def pressures(U, B):
    bx = 0.5 * (B[0] + np.roll(B[0], -1, axis=1))
    by = 0.5 * (B[1] + np.roll(B[1], -1, axis=0))
    pm = 0.5 * (bx * bx + by * by + B[2] * B[2])
    pg = (GAMMA - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0] - pm)
    return pg, pm


def compare(a, ref, mask=None):
    if mask is not None:
        a, ref = a[mask], ref[mask]
    l1 = float(np.abs(a - ref).sum() / np.abs(ref).sum())
    within = float(np.mean(np.abs(a / ref - 1.0) <= 0.05))
    return l1, within


def run(n: int = 64, levels: int = 2, threshold: float = 3.2, t_end: float = 0.5, regrid_every: int = 4,
        prec: str = "f64", capacity: int = 1024, scheme=("ctu", "ppm", "roe")) -> dict:
    r = 1 << levels
    t0 = time.perf_counter()
    Uf, Bf, steps_fine = _uniform(n * r, t_end, prec, scheme)
    t_fine = time.perf_counter() - t0
    Uc, Bc, steps_coarse = _uniform(n, t_end, prec, scheme)
    h = Hierarchy(n, [0] * levels, *scheme, prec=prec, subcycle=True, capacity=capacity,
                  problem=inputs.orszag_tang(n, nz=16))
    h.regrid(threshold)
    h.check_regrid()
    t0 = time.perf_counter()
    steps_amr, counts = h.run(t_end, threshold, regrid_every)
    t_amr = time.perf_counter() - t0
    final = h.group_counts()
    # root cells under the finest level's groups (z-uniform: one xy map)
    finest = h.levels[-1].groups[:final[-1]].cpu().numpy() if final[-1] else np.zeros((0, 3), np.int32)
    covered = np.zeros((n, n), bool)
    for (gx, gy, _) in finest:
        covered[gy // r:(gy + 16) // r, gx // r:(gx + 16) // r] = True
    Ua = h.levels[0].U[:, 0].double().cpu().numpy()
    Ba = h.levels[0].B[:, 0].double().cpu().numpy()
    divb = [h.solvers[i].divb(lv)[0] * lv.dx for i, lv in enumerate(h.levels)]
    cells_lvl = [int(np.prod(lv.shape)) for lv in h.levels]
    frac = [c * 16 ** 3 / cells_lvl[i + 1] for i, c in enumerate(final)]
    h.close()
    ref = onto(Uf, Bf, r)
    pg_ref, pm_ref = pressures(*ref)
    out = {"n_root": n, "levels": levels, "threshold": threshold, "t_end": t_end, "prec": prec,
           "scheme": "+".join(scheme), "steps": {"fine_uniform": steps_fine, "coarse_uniform": steps_coarse,
                                                 "amr_root": steps_amr},
           "seconds": {"fine_uniform": round(t_fine, 2), "amr": round(t_amr, 2)},
           "volume_fraction_per_level": frac, "groups_per_level": final,
           "max_divb_dx": divb, "finest_root_fraction": float(covered.mean())}
    for name, (U, B) in (("amr", (Ua, Ba)), ("coarse_uniform", (Uc, Bc))):
        pg, pm = pressures(U, B)
        lg, wg = compare(pg, pg_ref)
        lm, wm = compare(pm, pm_ref)
        out[name] = {"l1_gas_pressure": lg, "l1_magnetic_pressure": lm,
                     "within_5pct_gas": wg, "within_5pct_magnetic": wm}
        if covered.any():
            out[name]["finest_region_l1_gas_pressure"] = compare(pg, pg_ref, covered)[0]
            out[name]["finest_region_l1_magnetic_pressure"] = compare(pm, pm_ref, covered)[0]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--threshold", type=float, default=3.2)
    ap.add_argument("--t-end", type=float, default=0.5)
    ap.add_argument("--regrid-every", type=int, default=4)
    ap.add_argument("--prec", default="f64")
    args = ap.parse_args()
    print(json.dumps(run(args.n, args.levels, args.threshold, args.t_end, args.regrid_every, args.prec)))


if __name__ == "__main__":
    main()
