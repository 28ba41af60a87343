"""Launch-shape autotuner of the batched level update.

Each level's stage kernels are persistent: a grid of at most
blocks_per_cu x CUs blocks walks the level's work items (the cells of its
listed patch groups and their halos) with a grid-wide stride, so one launch
covers any number of groups.  The shape decides how many groups one sweep of
the grid holds (blocks x 256 threads / 16^3 cells per group) and how much of
the chip a small level occupies.  The tuner times each candidate on the
level itself (ghost refill plus update, HIP events, median of a few reps)
and keeps the fastest; results are cached in a JSON file keyed by device,
method, precision, level shape and group count.
"""
from __future__ import annotations

import json
import os

import torch

CANDIDATES = (0, 1, 2, 4, 8, 16)


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_1804_03479_amd", "autotune.json")


def level_key(h, lvl: int) -> str:
    s, lv = h.solvers[lvl], h.levels[lvl]
    dev = torch.cuda.get_device_properties(0)
    arch = getattr(dev, "gcnArchName", dev.name)
    n = 0 if lv.groups is None else int(lv.groups.shape[0])
    c = s.cfg
    return f"{arch}|s{c.scheme}r{c.recon}f{c.riemann}p{c.prec}|{'x'.join(map(str, lv.shape))}|g{n}"


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


def tune(h, candidates=CANDIDATES, reps: int = 5, cache: str | None = None, use_cache: bool = False):
    """Pick each level's blocks_per_cu; sets it on the hierarchy and returns
    {"shapes": [...], "ms": [[candidate ms...] per level], "keys": [...]}.

    The timing runs advance the levels' state (it is a real update); tune
    before the measured run, not inside it."""
    path = cache or default_cache_path()
    store = {}
    if os.path.exists(path):
        try:
            store = json.load(open(path))
        except (OSError, ValueError):
            store = {}
    shapes, table, keys = [], [], []
    for lvl in range(len(h.levels)):
        key = level_key(h, lvl)
        keys.append(key)
        if use_cache and key in store:
            shapes.append(int(store[key]["blocks_per_cu"]))
            table.append(store[key]["ms"])
            continue
        ms = []
        for b in candidates:
            h.solvers[lvl].set_launch(b)
            ms.append(time_level(h, lvl, reps))
        best = candidates[min(range(len(ms)), key=ms.__getitem__)]
        shapes.append(int(best))
        table.append(ms)
        store[key] = {"blocks_per_cu": int(best), "candidates": list(candidates), "ms": ms}
    h.set_launch(shapes)
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return {"shapes": shapes, "candidates": list(candidates), "ms": table, "keys": keys}
