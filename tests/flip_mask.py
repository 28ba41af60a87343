"""Cells where the method itself cannot be held to a per-cell FP32 bar.

The update has discontinuous decisions: PPM's extremum test, the upwind
choice of the corner EMF by the sign of the face mass flux, Roe's HLLE
fallback.  Where such a decision's argument lies within float rounding of
its switch, a float run may take the other branch and move nearby cells
by a slope-sized amount, far above float round-off.  These cells are found
with the oracle alone: it is run again from the same state perturbed at
random by a few float ulps (relative eps per value, seeded); a cell whose
result moves by more than the parity bar under such a perturbation sits
next to a decision within float rounding of its switch (elsewhere the
update is Lipschitz and moves by about eps).  The union over a few seeds
is the excluded set; parity tests hold the per-cell bar everywhere else
and bound the excluded fraction."""
from __future__ import annotations

import numpy as np

import oracle


def flow_scales(U, B, gamma=5.0 / 3.0):
    """Per-component scales of a conserved state: max |rho|, the momentum
    scale max(rho) * max(fast speed) for the three momenta (their own
    magnitude can be far below it), max |e|, and max |B| for the field."""
    W = oracle.cons_to_prim(U, B, gamma)
    cf = np.sqrt((gamma * W[4] + (W[5:8] ** 2).sum(axis=0)) / W[0]).max()
    rho = np.abs(U[0]).max()
    return np.array([rho, rho * cf, rho * cf, rho * cf, np.abs(U[4]).max()]), np.abs(B).max()


def sensitive_mask(run, U, B, bar=1e-5, eps=3e-6, seeds=(101, 102, 103)):
    """run(U, B) -> (U1, B1) with the oracle.  Returns boolean masks (of U's
    and B's shapes) of the values that move by more than bar (relative to
    flow_scales of the unperturbed result) when the input is perturbed by
    relative eps, each seed's noise applied with both signs (a decision whose
    margin is below the change the noise makes in its argument flips under
    one of the two)."""
    U0, B0 = run(U, B)
    su, sb = flow_scales(U0, B0)
    mu = np.zeros(U.shape, bool)
    mb = np.zeros(B.shape, bool)
    for sd in seeds:
        rng = np.random.default_rng(sd)
        nu = eps * rng.uniform(-1, 1, U.shape)
        nb = eps * rng.uniform(-1, 1, B.shape)
        for sgn in (1.0, -1.0):
            U1, B1 = run(U * (1 + sgn * nu), B * (1 + sgn * nb))
            mu |= np.abs(U1 - U0) > bar * su[:, None, None, None]
            mb |= np.abs(B1 - B0) > bar * sb
    return mu, mb, su, sb


def check_outside(Ug, Bg, Uo, Bo, mu, mb, su, sb, bar=1e-5, max_frac=0.02, what=""):
    """Per-value bar outside the masks; the masked fraction bounded.  Returns
    (worst ratio outside, masked fraction) for reporting."""
    ru = np.abs(Ug - Uo) / (bar * su[:, None, None, None])
    rb = np.abs(Bg - Bo) / (bar * sb)
    worst = max(float(ru[~mu].max(initial=0.0)), float(rb[~mb].max(initial=0.0)))
    frac = (mu.sum() + mb.sum()) / (mu.size + mb.size)
    print(f"\n{what}: worst |gpu - oracle| / bar outside the flip set {worst:.3f}; "
          f"flip set {int(mu.sum())} + {int(mb.sum())} values ({100 * frac:.3f} %); "
          f"worst inside {max(float(ru.max()), float(rb.max())):.1f} x bar")
    assert worst <= 1.0, (what, worst)
    assert frac <= max_frac, (what, frac)
    return worst, frac


def level_flip_masks(run, levels, masks, bar=1e-12, eps=1e-14, seeds=(201, 202)):
    """The same test for a hierarchy in double precision.  run(levels) ->
    levels, each a (U, B) pair; masks[l] = (cell mask, [face masks]) of the
    values of level l that count.  Each seed's relative noise eps (about 45
    double ulps, well above the rounding by which two implementations of the
    step differ) is applied to every level with both signs; a value that
    moves by more than bar times its component's largest magnitude over the
    counted values sits next to a decision within that noise of its switch.
    Returns (reference levels, per level (U mask, B mask) of such values)."""
    ref = run(levels)
    out = [(np.zeros(U.shape, bool), np.zeros(B.shape, bool)) for U, B in ref]
    for sd in seeds:
        rng = np.random.default_rng(sd)
        noise = [(eps * rng.uniform(-1, 1, U.shape), eps * rng.uniform(-1, 1, B.shape)) for U, B in levels]
        for sgn in (1.0, -1.0):
            per = run([(U * (1 + sgn * nu), B * (1 + sgn * nb)) for (U, B), (nu, nb) in zip(levels, noise)])
            for (Ur, Br), (Up, Bp), (cm, fm), (mu, mb) in zip(ref, per, masks, out):
                for c in range(Ur.shape[0]):
                    s = np.abs(Ur[c][cm]).max()
                    mu[c] |= cm & (np.abs(np.nan_to_num(Up[c] - Ur[c])) > bar * s)
                for a in range(3):
                    s = np.abs(Br[a][fm[a]]).max()
                    mb[a] |= fm[a] & (np.abs(np.nan_to_num(Bp[a] - Br[a])) > bar * s)
    return ref, out
