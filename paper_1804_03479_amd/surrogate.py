"""Training driver of the learned interface flux.

Every arithmetic step (capture, feature normalisation, forward, backward,
Adam) runs in libmhd's kernels; this module only chooses samples (seeded
index selection) and the learning-rate schedule.

Recipe: capture (wl, wr, bn, HLLD flux) from CTU+PPM+HLLD runs of the ABC
box (at several times of a run, so that the decaying flow of late times is
represented as well as the noisy start; a run with stronger velocity noise
supplies faces with strong jumps), drop samples whose normalised jump is
below 1e-4 (their targets are float round-off) and faces beyond the fallback
thresholds (HLLD takes those at run time), classify the rest by the
relative jump max(|dp|/p_min, |drho|/rho_min): "smooth" up to `strong_lo`
(0.1), "strong" between it and the fallback threshold, draw a seeded 3:1
smooth:strong mix (with replacement when a class is short), split 90/10 by a
seeded permutation, and train with MSE + Adam (0.9, 0.999), batch 4096,
learning rate decaying to 1e-5 on a cosine; the validation loss is reported
per class.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import inputs
from .mhd import MlpOps, Solver


def init_params(nparam: int, seed: int = 0) -> torch.Tensor:
    """Glorot-uniform weights, zero biases, in the packed layout."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for shape in [(15, 64), (64,), (64, 64), (64,), (64, 7), (7,)]:
        if len(shape) == 2:
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append((torch.rand(shape, generator=g, dtype=torch.float64) * 2 - 1) * lim)
        else:
            parts.append(torch.zeros(shape, dtype=torch.float64))
    p = torch.cat([x.reshape(-1) for x in parts]).to(torch.float32)
    assert p.numel() == nparam
    return p.cuda()


def capture(n: int = 64, steps: int = 10, noise: float = 0.1, seed: int = 0, stride: int = 1,
            cap: int = 1_000_000, prec: str = "f32", capture_at=None) -> torch.Tensor:
    """Run CTU+PPM+HLLD on an n^3 ABC box for `steps` steps, capturing the
    interfaces of the steps listed in capture_at (default: all of them);
    returns samples (m, 22)."""
    s = Solver("ctu", "ppm", "hlld", prec)
    ops = MlpOps(s)
    p = inputs.abc_problem(n, noise, seed=seed)
    W5 = torch.from_numpy(np.stack([p["rho"], p["vx"], p["vy"], p["vz"], p["p"]]))
    B = torch.from_numpy(np.stack([p["bx"], p["by"], p["bz"]]))
    lv = s.level_from_primitives(W5, B, p["dx"])
    buf = torch.empty((cap, 22), dtype=torch.float32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    when = set(range(steps)) if capture_at is None else set(capture_at)
    on = False
    for k in range(steps):
        if (k in when) != on:
            on = k in when
            if on:
                ops.set_capture(buf, count, stride)
            else:
                ops.set_capture(None)
        s.advance(lv)
    ops.set_capture(None)
    torch.cuda.synchronize()
    m = min(int(count.item()), cap)
    out = buf[:m].clone()
    s.close()
    return out


def relative_jump(samples: torch.Tensor) -> np.ndarray:
    """max(|p_R - p_L| / min(p), |rho_R - rho_L| / min(rho)) of captured samples
    (sample selection only; the fallback decision itself is the kernels')."""
    S = samples[:, [0, 4, 7, 11]].double().cpu().numpy()
    rl, pl, rr, pr = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    return np.maximum(np.abs(pr - pl) / np.minimum(pl, pr), np.abs(rr - rl) / np.minimum(rl, rr))


def training_set(ops: MlpOps, samples: torch.Tensor, n_total: int, seed: int = 0, smooth_frac: float = 0.75,
                 strong_lo: float = 0.1):
    """Seeded 3:1 mix of smooth (relative jump <= strong_lo) and strong (above
    it, below the fallback thresholds) captured samples -> (X, T, info);
    info["cls"] is the class of each row (0 smooth, 1 strong) on the device."""
    X, T, flags = ops.prepare(samples)
    fl = flags.cpu().numpy()
    usable = ((fl & 2) == 0) & ((fl & 1) == 0)   # float-resolvable targets, network faces only
    strong = relative_jump(samples) > strong_lo
    rng = np.random.default_rng(seed)
    idx_s, idx_k = np.flatnonzero(usable & ~strong), np.flatnonzero(usable & strong)
    n_s = int(round(n_total * smooth_frac)) if len(idx_k) else n_total
    n_k = n_total - n_s
    pick, cls = [], []
    if len(idx_s):
        pick.append(rng.choice(idx_s, n_s, replace=n_s > len(idx_s)))
        cls.append(np.zeros(n_s, np.int8))
    if n_k and len(idx_k):
        pick.append(rng.choice(idx_k, n_k, replace=n_k > len(idx_k)))
        cls.append(np.ones(n_k, np.int8))
    order = rng.permutation(sum(len(p) for p in pick))
    sel = np.concatenate(pick)[order]
    lab = np.concatenate(cls)[order]
    sel_t = torch.from_numpy(sel).cuda()
    return X[sel_t].contiguous(), T[sel_t].contiguous(), {
        "smooth": int(n_s), "strong": int(n_k), "strong_lo": strong_lo,
        "available_smooth": int(len(idx_s)), "available_strong": int(len(idx_k)),
        "fallback_faces_dropped": int(((fl & 1) != 0).sum()), "cls": torch.from_numpy(lab).cuda()}


def train(ops: MlpOps, X: torch.Tensor, T: torch.Tensor, epochs: int = 5, batch: int = 4096, lr0: float = 1e-3,
          lr1: float = 1e-5, seed: int = 0, params: torch.Tensor | None = None, cls: torch.Tensor | None = None):
    """Adam on the MSE of normalised fluxes; returns (params, history).  With
    cls (the class of each row) the validation loss is also given per class."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = torch.from_numpy(rng.permutation(n)).cuda()
    n_val = max(1, n // 10)
    val, tr = perm[:n_val], perm[n_val:]
    Xv, Tv = X[val].contiguous(), T[val].contiguous()
    cv = None if cls is None else cls[val]
    if params is None:
        params = init_params(ops.nparam, seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    g = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    nb = max(1, (len(tr) + batch - 1) // batch)
    total = epochs * nb
    step = 0
    hist = []
    for ep in range(epochs):
        order = tr[torch.from_numpy(rng.permutation(len(tr))).cuda()]
        for b in range(nb):
            ib = order[b * batch:(b + 1) * batch]
            if len(ib) == 0:
                continue
            step += 1
            lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * (step - 1) / max(1, total - 1)))
            ops.train_step(params, m, v, g, step, X[ib].contiguous(), T[ib].contiguous(), lr, loss)
        Yv = ops.forward(params, Xv)
        err = ((Yv - Tv) ** 2).mean(dim=1)
        h = {"epoch": ep + 1, "train_loss": float(loss.item()), "val_loss": float(err.mean().item())}
        if cv is not None:
            for k, name in ((0, "val_loss_smooth"), (1, "val_loss_strong")):
                sel = cv == k
                h[name] = float(err[sel].mean().item()) if bool(sel.any()) else None
        hist.append(h)
    return params, hist
