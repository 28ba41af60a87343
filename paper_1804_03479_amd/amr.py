"""A level hierarchy of dense periodic grids with patch-group work lists.

Each level l holds a dense (n 2^l)^3 grid in HBM; only the listed patch groups
of a refined level are updated, and the cells around them are ghosts refilled
from the coarser level before each update (paper Sec. 3.3).

Shared time step (subcycle=False), one step of every level:

  dt = min over levels of the CFL step          (mhd_cfl_dt_min, on device)
  for each level, coarse to fine:
      refill the ghost halos from the parent    (mhd_prolong, list mode)
  for each level: update the listed groups      (mhd_step_devdt)
  for each level, fine to coarse:
      correct the parent at the coarse-fine interface with the level's
      fluxes and EMFs                           (mhd_correct)
      restrict the level onto its parent        (mhd_restrict)

Sub-cycled (subcycle=True; Sec. 3.3's update of level l: update l, evolve
l + 1 until it reaches l's time, correct l, here with a refinement ratio of
2 in time): dt_0 = min over l of 2^l times level l's CFL step, dt_l =
dt_{l-1} / 2, and

  advance(l):
      keep level l's state at the start of its step   (copy, levels with children)
      update level l by dt_l
      for the two sub-steps s = 0, 1 of level l + 1:
          refill l + 1's ghosts from l at time fraction s/2
              (old + s/2 (new - old); mhd_prolong_time)
          advance(l + 1)
          add half of l + 1's final fluxes and EMFs to its registers
              (mhd_accumulate_registers)
      correct l with the time-mean registers (mhd_correct, fine_registers)
      restrict l + 1 onto l

Group lists are chosen with a seeded generator and are octree-consistent:
every group of level l + 1 lies inside a group of level l.  With a list
capacity, regrid() replaces them by the refinement criterion (Sec. 3.3,
refinement / derefinement): for each refined level, coarse to fine, the
candidate groups where |curl B| dx / |B| exceeds a threshold on the parent
level (inside the parent's groups) become the new list (mhd_regrid_flag),
and the created groups take the parent's data (mhd_prolong_new_groups); the
lists live in fixed (capacity, 3) buffers with a device count, so a
captured step stays valid across regrids.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs
from .mhd import Level, Solver, check_group_origins


def nested_groups(n_root: int, counts, edge: int = 16, seed: int = 0):
    """Seeded group origins (cells of each level) for levels 1..len(counts).

    Level-1 groups are distinct random groups of the (2 n_root)^3 level;
    each deeper level draws distinct groups among the 8 children of the
    previous level's groups.  Counts above the available children are capped.
    """
    rng = np.random.default_rng(seed)
    out = []
    n1 = 2 * n_root
    g1 = n1 // edge
    cand = np.stack(np.meshgrid(np.arange(g1), np.arange(g1), np.arange(g1), indexing="ij"), -1).reshape(-1, 3)
    pick = cand[rng.choice(len(cand), min(counts[0], len(cand)), replace=False)]
    out.append(pick * edge)
    for c in counts[1:]:
        parents = out[-1] // edge           # group indices of the previous level
        kids = (2 * parents[:, None, :] + np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
                ).reshape(-1, 3)
        pick = kids[rng.choice(len(kids), min(c, len(kids)), replace=False)]
        out.append(pick * edge)
    return [g.astype(np.int32) for g in out]


class Hierarchy:
    """Root level plus refined levels, one libmhd context per level (each level
    keeps its own launch shape and scratch), all on one stream."""

    def __init__(self, n_root: int, counts, scheme="ctu", recon="ppm", riemann="hlld", prec="f32",
                 noise: float = 0.1, seed: int = 0, edge: int = 16, stream: torch.cuda.Stream | None = None,
                 correct: bool = True, subcycle: bool = False, capacity: int | None = None,
                 problem: inputs.Problem | None = None):
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.correct = correct
        self.subcycle = subcycle
        self.groups = nested_groups(n_root, counts, edge, seed)
        with torch.cuda.stream(self.stream):
            self.solvers = [Solver(scheme, recon, riemann, prec, stream=self.stream)
                            for _ in range(len(self.groups) + 1)]
            s0 = self.solvers[0]
            p = problem if problem is not None else inputs.abc_problem(n_root, noise, seed=seed)
            W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
            B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
            root = s0.level_from_primitives(W5, B, p["dx"])
            self.levels = [root]
            for lvl, g in enumerate(self.groups, start=1):
                shape = tuple(x << lvl for x in root.shape)
                U = torch.empty((5,) + shape, dtype=s0.dtype, device="cuda")
                Bf = torch.empty((3,) + shape, dtype=s0.dtype, device="cuda")
                fine = Level(U, Bf, p["dx"] / (1 << lvl))
                self.solvers[lvl].prolong(self.levels[-1], fine)     # whole level, initial data
                if capacity is None:
                    fine.group_edge = edge
                    fine.set_groups(torch.from_numpy(g).cuda())
                else:
                    # at most every candidate group of the level
                    cap = min(capacity, int(np.prod(shape)) // edge ** 3)
                    if len(g) > cap:
                        raise ValueError("initial group list longer than the capacity")
                    check_group_origins(g, shape, edge)
                    buf = torch.zeros((cap, 3), dtype=torch.int32, device="cuda")
                    buf[:len(g)] = torch.from_numpy(g).cuda()
                    fine.group_edge = edge
                    # rows past the device count are unused padding
                    fine.set_groups(buf, validate=False)
                    fine.n_groups_dev = torch.tensor([len(g)], dtype=torch.int32, device="cuda")
                fine.group_edge = edge
                self.levels.append(fine)
            self.capacity = capacity
            self.edge = edge
            if capacity is not None:
                # regridding: the new list, its count, and the number each level wanted
                self._new = torch.zeros((capacity, 3), dtype=torch.int32, device="cuda")
                self._count = torch.zeros(1, dtype=torch.int32, device="cuda")
                self._wanted = torch.zeros(len(self.levels), dtype=torch.int32, device="cuda")
            # per-level steps (all equal without sub-cycling); dt is the root's
            self.dts = torch.zeros(len(self.levels), dtype=torch.float64, device="cuda")
            self.dt = self.dts[:1]
            # a level's state at the start of its step, for its children's ghosts
            self.old = []
            if subcycle:
                for lv in self.levels[:-1]:
                    self.old.append(Level(torch.empty_like(lv.U), torch.empty_like(lv.B), lv.dx))
        self.stream.synchronize()

    @property
    def s(self):
        return self.solvers[0]

    def group_counts(self):
        """Listed groups of each refined level (a host sync with a capacity)."""
        if self.capacity is None:
            return [len(g) for g in self.groups]
        return [int(lv.n_groups_dev.item()) for lv in self.levels[1:]]

    def cells_per_level(self):
        out = [int(np.prod(self.levels[0].shape))]
        for n, lv in zip(self.group_counts(), self.levels[1:]):
            out.append(n * lv.group_edge ** 3)
        return out

    def regrid(self, threshold: float, buffer: int = 1):
        """Refinement / derefinement of every refined level from the criterion
        |curl B| dx / |B| > threshold on its parent (asynchronous); then
        check_regrid() reports whether every list fitted its capacity."""
        if self.capacity is None:
            raise RuntimeError("regrid needs a Hierarchy built with a list capacity")
        with torch.cuda.stream(self.stream):
            for lvl in range(1, len(self.levels)):
                s, coarse, fine = self.solvers[lvl], self.levels[lvl - 1], self.levels[lvl]
                cap = fine.groups.shape[0]
                buf = self._new[:cap]
                s.regrid_flag(coarse, threshold, buffer, self.edge, buf, self._count, self._wanted[lvl - 1:lvl])
                # the list was written by the library's regridding kernels
                new = Level(fine.U, fine.B, fine.dx, groups=buf, group_edge=self.edge, validate_groups=False)
                new.n_groups_dev = self._count
                s.prolong_new_groups(coarse, new, fine)
                fine.groups.copy_(buf)
                fine.n_groups_dev.copy_(self._count)

    def run(self, t_end: float, threshold: float | None = None, regrid_every: int = 0, buffer: int = 1):
        """Root steps to t_end (the last one shortened), regridding every
        regrid_every root steps; returns (steps, per-regrid group counts)."""
        t, steps, counts = 0.0, 0, []
        while t < t_end * (1.0 - 1e-12):
            if threshold is not None and regrid_every and steps and steps % regrid_every == 0:
                self.regrid(threshold, buffer)
                self.check_regrid()
                counts.append(self.group_counts())
            self.step(dt_max=t_end - t)
            self.stream.synchronize()
            t += float(self.dts[0].item())
            steps += 1
        return steps, counts

    def reset_root(self, U: torch.Tensor, B: torch.Tensor):
        """Replace the root state (conserved U, face B of the root's shape and
        dtype), refill every finer level from it by whole-level prolongation
        and empty the group lists (capacity mode; regrid() lists them again)."""
        if self.capacity is None:
            raise RuntimeError("reset_root needs a Hierarchy built with a list capacity")
        with torch.cuda.stream(self.stream):
            self.levels[0].U.copy_(U)
            self.levels[0].B.copy_(B)
            for lvl in range(1, len(self.levels)):
                fine = self.levels[lvl]
                whole = Level(fine.U, fine.B, fine.dx)
                self.solvers[lvl].prolong(self.levels[lvl - 1], whole)
                fine.n_groups_dev.zero_()

    def check_regrid(self):
        """Groups each level wanted at the last regrid; raises if one did not fit."""
        self.stream.synchronize()
        wanted = self._wanted[:len(self.levels) - 1].cpu().tolist()
        caps = [lv.groups.shape[0] for lv in self.levels[1:]]
        if any(w > c for w, c in zip(wanted, caps)):
            raise RuntimeError(f"regrid wanted {wanted} groups per level, capacities {caps}")
        return wanted

    def updates_per_step(self):
        """Cell updates of each level in one root step (2^l sub-steps on level l
        when sub-cycling)."""
        return [c << (l if self.subcycle else 0) for l, c in enumerate(self.cells_per_level())]

    def set_launch(self, shapes):
        """Launch shape of each level: blocks per CU of the persistent launches
        (0 = one item per thread), or a (blocks_per_cu, threads, batch[,
        tiles]) tuple."""
        for s, b in zip(self.solvers, shapes):
            s.set_launch(*(tuple(b) if isinstance(b, (tuple, list)) else (int(b),)))

    def shared_dt(self, dt_max: float = float("inf")):
        """Device steps of all levels: the shared CFL minimum, or with
        sub-cycling dt_0 = min_l 2^l dt_cfl(l) and dt_l = dt_0 / 2^l; dt_0 is
        at most dt_max."""
        with torch.cuda.stream(self.stream):
            d0 = self.dts[:1]
            d0.fill_(float(dt_max))
            for lvl, (s, lv) in enumerate(zip(self.solvers, self.levels)):
                s.cfl_dt_min(lv, d0, scale=float(1 << lvl) if self.subcycle else 1.0)
            for lvl in range(1, len(self.levels)):
                self.s.dt_subdivide(self.dts[lvl - 1:lvl], 2 if self.subcycle else 1, self.dts[lvl:lvl + 1])

    def update_level(self, lvl: int):
        """Ghost refill from the parent (refined levels) and the update of level lvl."""
        s, lv = self.solvers[lvl], self.levels[lvl]
        if lvl > 0:
            s.prolong(self.levels[lvl - 1], lv, halo=4)
        s.step_devdt(lv, self.dts[lvl:lvl + 1])

    def _close_level(self, lvl: int, registers: bool):
        """Correction of level lvl - 1 by level lvl, then the restriction."""
        if self.correct:
            self.solvers[lvl - 1].correct(self.levels[lvl - 1], self.solvers[lvl], self.levels[lvl],
                                          self.dts[lvl - 1:lvl], fine_registers=registers)
        self.solvers[lvl].restrict(self.levels[lvl], self.levels[lvl - 1])

    def _advance(self, lvl: int):
        s, lv = self.solvers[lvl], self.levels[lvl]
        last = lvl == len(self.levels) - 1
        if not last:
            old = self.old[lvl]
            old.U.copy_(lv.U)
            old.B.copy_(lv.B)
        s.step_devdt(lv, self.dts[lvl:lvl + 1])
        if last:
            return
        child, cs = self.levels[lvl + 1], self.solvers[lvl + 1]
        for sub in range(2):
            cs.prolong(lv, child, halo=4, coarse_old=self.old[lvl], alpha=0.5 * sub)
            self._advance(lvl + 1)
            if self.correct:
                cs.accumulate_registers(child, 0.5, reset=sub == 0)
        self._close_level(lvl + 1, registers=True)

    def step(self, dt_max: float = float("inf")):
        """One root step of all levels (asynchronous on self.stream)."""
        with torch.cuda.stream(self.stream):
            self.shared_dt(dt_max)
            if self.subcycle:
                self._advance(0)
                return
            for lvl in range(1, len(self.levels)):
                self.solvers[lvl].prolong(self.levels[lvl - 1], self.levels[lvl], halo=4)
            for lvl in range(len(self.levels)):
                self.solvers[lvl].step_devdt(self.levels[lvl], self.dts[lvl:lvl + 1])
            for lvl in range(len(self.levels) - 1, 0, -1):
                self._close_level(lvl, registers=False)

    def capture(self):
        """Capture one step() into a HIP graph (torch.cuda.CUDAGraph); returns it.
        Replay it with replay(), which launches it on the hierarchy's stream."""
        self.step()                       # allocations and first-use set-up happen eagerly
        self.stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            self.step()
        return g

    def replay(self, g):
        """One replay of a captured step, ordered on the hierarchy's stream
        (CUDAGraph.replay launches on the current stream)."""
        with torch.cuda.stream(self.stream):
            g.replay()

    def close(self):
        for s in self.solvers:
            s.close()
