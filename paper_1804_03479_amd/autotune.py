"""Launch-shape autotuner of the batched level update.

A level's stage kernels have four launch parameters (mhd_set_launch):
blocks per CU of the persistent grid that walks the level's work items (the
cells of its listed patch groups and their halos) with a grid-wide stride,
threads per block, for a group list the batch of groups that runs through
the middle stages together (so that a batch's intermediates can stay in the
caches between stages; paper Sec. 4 sends patch groups to the GPU in
batches), and for CTU with PPM whether the reconstruction stage runs on LDS
tiles.  The tuner times each candidate shape on the level itself (ghost
refill plus update, HIP events, median of a few reps) and keeps the fastest
of the first three parameters' grid; then, for CTU with PPM, it times the
winner with LDS tiles and keeps that if faster.  Results are cached in a
JSON file keyed by device, method, precision, level shape and group count.
Shapes with the same tile choice give bit-identical results; LDS tiles agree
with the per-cell form to rounding.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

BLOCKS_PER_CU = (0, 2, 8)
THREADS = (128, 256, 512)
BATCHES = (16, 32, 64, 128, 256, 512, 1024, 2048, 4096)
# the former one-parameter sweep (blocks per CU at 256 threads, whole list)
CANDIDATES = (0, 1, 2, 4, 8, 16)


def shape(c):
    """(blocks_per_cu, threads, batch, tiles) of a candidate given as an int
    or a tuple."""
    if isinstance(c, (tuple, list)):
        b, t, n, k = (tuple(c) + (0, 0, 0))[:4]
        return int(b), int(t), int(n), int(k)
    return int(c), 0, 0, 0


def tiles_apply(h, lvl: int) -> bool:
    """Does the LDS-tile option change level lvl's update (CTU with PPM)?"""
    c = h.solvers[lvl].cfg
    return c.scheme == 1 and c.recon == 1


def level_candidates(n_groups: int):
    """Shapes swept on a level with n_groups listed groups (0: whole grid):
    blocks per CU x threads per block x batch (the whole list, and every
    batch of 16 .. 4096 groups smaller than the list), per-cell
    reconstruction."""
    batches = (0,) + tuple(b for b in BATCHES if b < n_groups)
    return [(b, t, n, 0) for b, t, n in itertools.product(BLOCKS_PER_CU, THREADS, batches)]


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_1804_03479_amd", "autotune.json")


def n_listed(h, lvl: int) -> int:
    lv = h.levels[lvl]
    return 0 if lv.groups is None else int(lv.groups.shape[0])


def level_key(h, lvl: int) -> str:
    s, lv = h.solvers[lvl], h.levels[lvl]
    dev = torch.cuda.get_device_properties(0)
    arch = getattr(dev, "gcnArchName", dev.name)
    c = s.cfg
    return f"{arch}|s{c.scheme}r{c.recon}f{c.riemann}p{c.prec}|{'x'.join(map(str, lv.shape))}|g{n_listed(h, lvl)}"


def time_level(h, lvl: int, reps: int = 5, inner: int = 3) -> float:
    """Median milliseconds of one ghost refill + update of level lvl."""
    st = h.stream
    times = []
    h.shared_dt()
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(inner):
            h.update_level(lvl)
        e1.record(st)
        st.synchronize()
        times.append(e0.elapsed_time(e1) / inner)
    times = sorted(times[1:])
    return times[len(times) // 2]


def tune(h, candidates=None, reps: int = 5, cache: str | None = None, use_cache: bool = False,
         try_tiles: bool = True):
    """Pick each level's launch shape; sets it on the hierarchy and returns
    {"shapes": [(blocks_per_cu, threads, batch, tiles) per level],
    "candidates": [[shape...] per level], "ms": [[ms per candidate] per
    level], "keys": [...]}.  candidates: None (level_candidates of each
    level) or one list of shapes (ints: blocks per CU at the default threads
    and batch) for every level.  try_tiles: also time the best shape with
    LDS tiles where that option applies (it is then the last candidate).

    The timing runs advance the levels' state (it is a real update); tune
    before the measured run, not inside it."""
    path = cache or default_cache_path()
    store = {}
    if os.path.exists(path):
        try:
            store = json.load(open(path))
        except (OSError, ValueError):
            store = {}
    shapes, table, cands, keys = [], [], [], []
    for lvl in range(len(h.levels)):
        cl = [shape(c) for c in (candidates if candidates is not None else level_candidates(n_listed(h, lvl)))]
        key = level_key(h, lvl) + "|" + ",".join("%d/%d/%d/%d" % c for c in cl) + ("|t" if try_tiles else "")
        keys.append(key)
        if use_cache and key in store:
            shapes.append(tuple(store[key]["shape"]))
            table.append(store[key]["ms"])
            cands.append([tuple(c) for c in store[key]["candidates"]])
            continue
        ms = []
        for c in cl:
            h.solvers[lvl].set_launch(*c)
            ms.append(time_level(h, lvl, reps))
        best = cl[min(range(len(ms)), key=ms.__getitem__)]
        if try_tiles and tiles_apply(h, lvl) and best[3] == 0:
            tiled = best[:3] + (1,)
            h.solvers[lvl].set_launch(*tiled)
            cl = cl + [tiled]
            ms.append(time_level(h, lvl, reps))
            best = cl[min(range(len(ms)), key=ms.__getitem__)]
        shapes.append(best)
        table.append(ms)
        cands.append(cl)
        store[key] = {"shape": list(best), "candidates": [list(c) for c in cl], "ms": ms}
    h.set_launch(shapes)
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return {"shapes": shapes, "candidates": cands, "ms": table, "keys": keys}
