"""A level hierarchy of dense periodic grids with patch-group work lists.

Each level l holds a dense (n 2^l)^3 grid in HBM; only the listed patch groups
of a refined level are updated, and the cells around them are ghosts refilled
from the coarser level before each update (paper Sec. 3.3).  One step of the
hierarchy (shared time step, no sub-cycling):

  dt = min over levels of the CFL step          (mhd_cfl_dt_min, on device)
  for each level, coarse to fine:
      refill the ghost halos from the parent    (mhd_prolong, list mode)
      update the listed groups                  (mhd_step_devdt)
  for each level, fine to coarse:
      correct the parent at the coarse-fine interface with the level's
      fluxes and EMFs                           (mhd_correct)
      restrict the level onto its parent        (mhd_restrict)

Group lists are chosen with a seeded generator and are octree-consistent:
every group of level l + 1 lies inside a group of level l.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs
from .mhd import Level, Solver


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
                 correct: bool = True):
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.correct = correct
        self.groups = nested_groups(n_root, counts, edge, seed)
        with torch.cuda.stream(self.stream):
            self.solvers = [Solver(scheme, recon, riemann, prec, stream=self.stream)
                            for _ in range(len(self.groups) + 1)]
            s0 = self.solvers[0]
            p = inputs.abc_problem(n_root, noise, seed=seed)
            W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
            B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
            root = s0.level_from_primitives(W5, B, p["dx"])
            self.levels = [root]
            for lvl, g in enumerate(self.groups, start=1):
                n = n_root << lvl
                U = torch.empty((5, n, n, n), dtype=s0.dtype, device="cuda")
                Bf = torch.empty((3, n, n, n), dtype=s0.dtype, device="cuda")
                fine = Level(U, Bf, p["dx"] / (1 << lvl))
                self.solvers[lvl].prolong(self.levels[-1], fine)     # whole level, initial data
                fine.set_groups(torch.from_numpy(g).cuda())
                fine.group_edge = edge
                self.levels.append(fine)
            self.dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.stream.synchronize()

    @property
    def s(self):
        return self.solvers[0]

    def cells_per_level(self):
        out = [int(np.prod(self.levels[0].shape))]
        for g, lv in zip(self.groups, self.levels[1:]):
            out.append(len(g) * lv.group_edge ** 3)
        return out

    def set_launch(self, shapes):
        """Blocks per CU of each level's persistent launches (0 = one item per thread)."""
        for s, b in zip(self.solvers, shapes):
            s.set_launch(int(b))

    def shared_dt(self):
        with torch.cuda.stream(self.stream):
            self.dt.fill_(float("inf"))
            for s, lv in zip(self.solvers, self.levels):
                s.cfl_dt_min(lv, self.dt)

    def update_level(self, lvl: int):
        """Ghost refill from the parent (refined levels) and the update of level lvl."""
        s, lv = self.solvers[lvl], self.levels[lvl]
        if lvl > 0:
            s.prolong(self.levels[lvl - 1], lv, halo=4)
        s.step_devdt(lv, self.dt)

    def step(self):
        """One shared-dt step of all levels (asynchronous on self.stream)."""
        with torch.cuda.stream(self.stream):
            self.shared_dt()
            for lvl in range(len(self.levels)):
                self.update_level(lvl)
            for lvl in range(len(self.levels) - 1, 0, -1):
                if self.correct:
                    self.solvers[lvl - 1].correct(self.levels[lvl - 1], self.solvers[lvl], self.levels[lvl], self.dt)
                self.solvers[lvl].restrict(self.levels[lvl], self.levels[lvl - 1])

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
