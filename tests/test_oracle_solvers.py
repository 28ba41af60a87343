"""Pins of the oracle's Riemann solvers and PPM reconstruction against what
mathematics fixes, beyond consistency:

* HLLE (Sec. 3.2 names it): for mirrored states its two Davis bounds are
  -S and +S, and the HLL flux reduces to the Rusanov flux
  (F_L + F_R)/2 - S (U_R - U_L)/2, computed here from the textbook fast
  speed and conserved variables; outside both bounds it is the upwind
  physical flux.  A flipped sign or a wrong bound of the dissipative term
  fails.
* The hydrodynamic limit (B = 0) of every solver inside the full VL
  update converges to the exact Riemann solution (textbook construction,
  tests/exact_riemann.py) on Sod's problem and on the strong double
  rarefaction 1-2-0-3 of Einfeldt et al.; HLLE keeps density and pressure
  positive in the near-vacuum rarefaction, where Roe's linearisation fails
  and falls back to HLLE.
* PPM (Colella & Woodward 1984, the reading of Sec. 3.2's PPM): the edge
  values of cell averages of any cubic equal the cubic's point values
  where the limiters are inactive; at a local extremum the parabola is
  flat; for any data the limited parabola is monotone inside the cell.
"""
import math

import numpy as np
import pytest

import exact_riemann as er

orc = pytest.importorskip("oracle")

ROE, HLLE, HLLD = 0, 1, 2
G = 5.0 / 3.0


# ---------------------------------------------------------------- exact solver
def test_exact_solver_textbook_star_states():
    # star pressure and velocity of the classic tests as tabulated in
    # textbooks (four to six digits)
    p, u = er.star_state((1, 0, 1), (0.125, 0, 0.1), 1.4)
    assert abs(p - 0.30313) <= 5e-6 and abs(u - 0.92745) <= 5e-6
    p, u = er.star_state((1, -2, 0.4), (1, 2, 0.4), 1.4)
    assert abs(p - 0.00189) < 5e-6 and abs(u) < 1e-14
    p, u = er.star_state((1, 0, 1000), (1, 0, 0.01), 1.4)
    assert abs(p - 460.894) <= 5e-4 and abs(u - 19.5975) <= 5e-5


@pytest.mark.parametrize("left, right", [((1, 0, 1), (0.125, 0, 0.1)), ((1, -2, 0.4), (1, 2, 0.4)),
                                         ((1, 0.3, 2.0), (0.6, -0.8, 0.7)), ((0.8, 1.5, 0.5), (1.1, 0.2, 3.0))])
def test_exact_solver_jump_conditions(left, right):
    """Independent of any tabulated value: across a shock the mass, momentum
    and energy fluxes in the shock frame agree (Rankine-Hugoniot); through a
    fan the entropy and the outgoing Riemann invariant are constant; pressure
    and velocity are continuous across the contact."""
    g = 1.4
    s = np.linspace(-6, 6, 24001)
    rho, u, p = er.sample(left, right, g, s)
    ps, us = er.star_state(left, right, g)
    i = np.searchsorted(s, us)
    assert abs(p[i - 1] - ps) < 1e-12 * ps and abs(p[i + 1] - ps) < 1e-12 * ps
    assert abs(u[i - 1] - us) < 1e-12 and abs(u[i + 1] - us) < 1e-12
    for side, k in ((left, slice(0, i)), (right, slice(i, None))):
        r, v, q = rho[k], u[k], p[k]
        ent = q / r ** g
        jump = np.flatnonzero(np.abs(np.diff(r)) > 1e-3 * r.max())
        if side[2] < ps:          # shock: one jump, satisfying Rankine-Hugoniot
            a0, a1 = jump[0], jump[0] + 1
            (r0, v0, q0), (r1, v1, q1) = (r[a0], v[a0], q[a0]), (r[a1], v[a1], q[a1])
            S = (r1 * v1 - r0 * v0) / (r1 - r0)            # mass conservation fixes the speed
            m = r0 * (v0 - S)
            assert abs(m * (v1 - v0) + (q1 - q0)) < 1e-9 * q1          # momentum
            h0 = g / (g - 1) * q0 / r0 + 0.5 * (v0 - S) ** 2
            h1 = g / (g - 1) * q1 / r1 + 0.5 * (v1 - S) ** 2
            assert abs(h1 - h0) < 1e-9 * h1                               # energy
        else:                     # rarefaction: isentropic, invariant constant
            assert np.allclose(ent, side[2] / side[0] ** g, rtol=1e-10)
            a = np.sqrt(g * q / r)
            inv = v + 2 * a / (g - 1) if side is left else v - 2 * a / (g - 1)
            assert np.allclose(inv, inv[0], rtol=0, atol=1e-10)


# ---------------------------------------------------------------- HLLE
def textbook_fast(w, bn):
    rho, p = w[0], w[4]
    a2 = G * p / rho
    b2 = (bn * bn + w[5] ** 2 + w[6] ** 2) / rho
    return math.sqrt(0.5 * (a2 + b2 + math.sqrt((a2 + b2) ** 2 - 4 * a2 * bn * bn / rho)))


def conserved(w, bn):
    rho, vn, v1, v2, p, b1, b2 = w
    e = p / (G - 1) + 0.5 * rho * (vn * vn + v1 * v1 + v2 * v2) + 0.5 * (bn * bn + b1 * b1 + b2 * b2)
    return np.array([rho, rho * vn, rho * v1, rho * v2, e, b1, b2])


def test_hlle_mirrored_states_give_rusanov_flux():
    rng = np.random.default_rng(31)
    for _ in range(200):
        rho, p, vn = rng.uniform(0.3, 3), rng.uniform(0.2, 3), rng.uniform(-1, 1)
        bt, th1, th2 = rng.uniform(0, 1.5), rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)
        bn = rng.uniform(-1.5, 1.5)
        wl = np.array([rho, vn, rng.uniform(-1, 1), rng.uniform(-1, 1), p, bt * math.cos(th1), bt * math.sin(th1)])
        wr = np.array([rho, -vn, rng.uniform(-1, 1), rng.uniform(-1, 1), p, bt * math.cos(th2), bt * math.sin(th2)])
        S = abs(vn) + textbook_fast(wl, bn)
        assert abs(S - (abs(vn) + textbook_fast(wr, bn))) < 1e-14 * S
        rus = 0.5 * (orc.phys_flux(wl, bn) + orc.phys_flux(wr, bn)) - 0.5 * S * (conserved(wr, bn) - conserved(wl, bn))
        f, _ = orc.riemann(HLLE, wl, wr, bn)
        assert np.allclose(f, rus, rtol=0, atol=1e-13 * (1 + np.abs(rus).max()))


def test_hlle_supersonic_faces_take_the_upwind_flux():
    rng = np.random.default_rng(32)
    for _ in range(100):
        wl = np.array([rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1),
                       rng.uniform(0.1, 0.5), rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)])
        wr = wl * (1 + 0.2 * rng.uniform(-1, 1, 7))
        bn = rng.uniform(-0.3, 0.3)
        shift = 1.5 * max(textbook_fast(wl, bn), textbook_fast(wr, bn)) + 1.0
        for sgn in (1, -1):
            a, b = wl.copy(), wr.copy()
            a[1] += sgn * shift
            b[1] += sgn * shift
            f, _ = orc.riemann(HLLE, a, b, bn)
            up = orc.phys_flux(a if sgn > 0 else b, bn)
            assert np.array_equal(f, up)


# ---------------------------------------------------------------- hydro limit
def pencil_run(left, right, gamma, per_unit, t_end, recon, solver):
    """Periodic pencil [0, 2) x 4 x 4 cells, B = 0: state `left` on [0.5, 1.5),
    `right` elsewhere; VL update to t_end.  Returns cell centres, the final
    primitives and the minima of rho and p over every step."""
    nx = 2 * per_unit
    dx = 1.0 / per_unit
    xc = (np.arange(nx) + 0.5) * dx
    inside = (xc >= 0.5) & (xc < 1.5)
    W5 = np.zeros((5, 4, 4, nx))
    for m, (a, b) in enumerate(zip(left, right)):
        val = np.where(inside, a, b)
        W5[(0, 1, 4)[m]] = val[None, None, :]
    B = np.zeros((3, 4, 4, nx))
    U = orc.prim_to_cons(W5, B, gamma)
    t, mins, nfb = 0.0, [np.inf, np.inf], 0
    while t < t_end * (1 - 1e-14):
        dt = min(orc.cfl_dt(U, B, dx, gamma, 0.5), t_end - t)
        U, B, fb = orc.step(U, B, dt, dx, scheme=orc.VL, recon=recon, riemann=solver, gamma=gamma,
                            return_fallbacks=True)
        nfb += fb
        t += dt
        W = orc.cons_to_prim(U, B, gamma)
        mins = [min(mins[0], W[0].min()), min(mins[1], W[4].min())]
    W = orc.cons_to_prim(U, B, gamma)
    return xc, W, mins, nfb


def window_l1(left, right, gamma, xc, W, t):
    """L1 of (rho, u, p) against the exact solution of the discontinuity at
    x = 1.5, over [1, 2) (the other discontinuity's waves stay below 1)."""
    sel = xc >= 1.0
    ex = er.sample(left, right, gamma, (xc[sel] - 1.5) / t)
    got = np.stack([W[0, 0, 0, sel], W[1, 0, 0, sel], W[4, 0, 0, sel]])
    assert np.allclose(W[:, :, :, sel], W[:, :1, :1, sel], rtol=0, atol=1e-12)   # uniform across
    return np.abs(got - ex).mean(axis=1)


SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
DOUBLE_RAREFACTION = ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4))


@pytest.mark.parametrize("solver", [ROE, HLLE, HLLD])
def test_hydro_limit_converges_to_exact_sod(solver):
    errs = []
    for per_unit in (64, 128, 256):
        xc, W, mins, _ = pencil_run(*SOD, 1.4, per_unit, 0.15, orc.PLM, solver)
        errs.append(window_l1(*SOD, 1.4, xc, W, 0.15))
    errs = np.array(errs)
    # first order at the discontinuities: at least 1.5x per doubling
    assert np.all(errs[1] < errs[0] / 1.5) and np.all(errs[2] < errs[1] / 1.5), errs
    assert errs[2][0] < 4e-3, errs


@pytest.mark.parametrize("recon", [2, 0])   # first order, PLM
def test_hlle_double_rarefaction_positive_and_converging(recon):
    errs = []
    for per_unit in (64, 128, 256):
        xc, W, mins, _ = pencil_run(*DOUBLE_RAREFACTION, 1.4, per_unit, 0.15, recon, HLLE)
        assert mins[0] > 0 and mins[1] > 0
        errs.append(window_l1(*DOUBLE_RAREFACTION, 1.4, xc, W, 0.15))
    errs = np.array(errs)
    assert np.all(errs[2] < errs[0] / 1.8), errs


def test_roe_falls_back_to_hlle_in_the_double_rarefaction():
    xc, W, mins, nfb = pencil_run(*DOUBLE_RAREFACTION, 1.4, 64, 0.15, 2, ROE)
    assert nfb > 0
    assert mins[0] > 0 and mins[1] > 0


# ---------------------------------------------------------------- PPM
def cubic_averages(c, x0, h=1.0):
    """Averages of c0 + c1 x + c2 x^2 + c3 x^3 over [x0 + i h, x0 + (i+1) h], i = 0..4."""
    P = np.polynomial.polynomial.Polynomial(c).integ()
    e = x0 + h * np.arange(6)
    return np.diff(P(e)) / h


def test_ppm_edges_exact_for_cubics():
    rng = np.random.default_rng(33)
    n = 0
    for _ in range(400):
        c = rng.uniform(-1, 1, 4) * np.array([1, 1, 0.05, 0.01])
        c[1] = 2.0 + abs(c[1])                    # monotone, limiters inactive
        x0 = rng.uniform(-2, 2)
        q = cubic_averages(c, x0)
        lo, hi = orc.ppm_edges(q)
        P = np.polynomial.polynomial.Polynomial(c)
        assert abs(lo - P(x0 + 2)) < 1e-13 * (1 + abs(lo)), (lo, P(x0 + 2))
        assert abs(hi - P(x0 + 3)) < 1e-13 * (1 + abs(hi)), (hi, P(x0 + 3))
        n += 1
    assert n == 400


def test_ppm_flat_at_extrema_and_monotone_parabola():
    rng = np.random.default_rng(34)
    flat = 0
    for _ in range(4000):
        q = rng.uniform(0, 1, 5)
        lo, hi = orc.ppm_edges(q)
        c = q[2]
        if (c - q[1]) * (q[3] - c) <= 0:          # local extremum of the averages
            assert lo == c and hi == c
            flat += 1
            continue
        # the parabola with edge values lo, hi and average c
        d, a6 = hi - lo, 6 * (c - 0.5 * (lo + hi))
        s0, s1 = d + a6, d - a6                   # its slopes at the two edges
        assert s0 * s1 >= -1e-12 * (1 + d * d + a6 * a6), (q, lo, hi)
        assert min(q[1], q[2]) - 1e-12 <= lo <= max(q[1], q[2]) + 1e-12
        assert min(q[2], q[3]) - 1e-12 <= hi <= max(q[2], q[3]) + 1e-12
    assert flat > 500
