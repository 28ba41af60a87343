"""Pins of the oracle's one-dimensional building blocks against mathematics
the paper fixes (Eqs. 1-9) rather than against the oracle itself.

* The physical flux (Eq. 7): its finite-difference Jacobian must have the
  textbook MHD characteristic speeds (u, u +- c_a, u +- c_s, u +- c_f with
  c_f,s from the closed-form quadratic), which fails for any dropped or
  mis-signed term.
* Each Riemann solver is consistent: F(W, W) equals the physical flux.
* Roe (paper: Roe solver, Sec. 3.2): the Roe property F_R - F_L =
  R diag(lam) R^-1 (U_R - U_L) for random states, and in the limit of equal
  states R diag(lam) R^-1 is the finite-difference Jacobian.
* HLLD (paper: HLLD solver, Sec. 3.2): scale invariance of ideal MHD, exact
  flux for an isolated contact and an isolated rotational discontinuity, and
  positive intermediate states for the paper's Table 1 Riemann problems.
"""
import math

import numpy as np
import pytest

G = 5.0 / 3.0


def rstate(rng):
    return np.array([rng.uniform(0.5, 2.0), *rng.uniform(-1, 1, 3), rng.uniform(0.5, 2.0),
                     *rng.uniform(-1, 1, 2)])


def fd_jacobian(orc, w, bn):
    u = orc.w_to_u(w, bn)
    J = np.zeros((7, 7))
    for j in range(7):
        h = 1e-6 * max(1.0, abs(u[j]))
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        J[:, j] = (orc.phys_flux(orc.u_to_w(up, bn), bn) - orc.phys_flux(orc.u_to_w(um, bn), bn)) / (2 * h)
    return J


def textbook_speeds(w, bn):
    d, u, p = w[0], w[1], w[4]
    a2 = G * p / d
    b2 = (bn * bn + w[5] ** 2 + w[6] ** 2) / d
    bn2 = bn * bn / d
    disc = math.sqrt((a2 + b2) ** 2 - 4 * a2 * bn2)
    cf = math.sqrt(0.5 * (a2 + b2 + disc))
    cs = math.sqrt(max(0.0, 0.5 * (a2 + b2 - disc)))
    ca = abs(bn) / math.sqrt(d)
    return np.sort([u - cf, u - ca, u - cs, u, u + cs, u + ca, u + cf])


def test_physical_flux_characteristic_speeds(orc):
    rng = np.random.default_rng(11)
    for _ in range(20):
        w = rstate(rng)
        bn = rng.uniform(-1, 1)
        lam = np.sort(np.linalg.eigvals(fd_jacobian(orc, w, bn)).real)
        assert np.allclose(lam, textbook_speeds(w, bn), atol=2e-6)
        # the oracle's fast speed is the largest |eigenvalue - u|
        assert abs(orc.fast_speed(w, bn) - (lam[-1] - w[1])) < 2e-6


def test_state_conversion_roundtrip(orc):
    rng = np.random.default_rng(2)
    for _ in range(10):
        w = rstate(rng)
        bn = rng.uniform(-1, 1)
        assert np.allclose(orc.u_to_w(orc.w_to_u(w, bn), bn), w, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("solver", [0, 1, 2])
def test_riemann_consistency(orc, solver):
    rng = np.random.default_rng(3 + solver)
    for _ in range(20):
        w = rstate(rng)
        bn = rng.uniform(-1, 1)
        f, fb = orc.riemann(solver, w, w, bn)
        assert fb == 0
        assert np.allclose(f, orc.phys_flux(w, bn), rtol=1e-13, atol=1e-13)


def test_roe_property(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        wl, wr = rstate(rng), rstate(rng)
        bn = rng.uniform(-1, 1)
        lam, R = orc.roe_eigen(wl, wr, bn)
        du = orc.w_to_u(wr, bn) - orc.w_to_u(wl, bn)
        alpha = np.linalg.solve(R, du)
        df = orc.phys_flux(wr, bn) - orc.phys_flux(wl, bn)
        assert np.allclose(R @ (lam * alpha), df, rtol=0, atol=1e-12 * (1 + np.abs(df).max()))


def test_roe_jacobian_limit(orc):
    rng = np.random.default_rng(6)
    for _ in range(20):
        w = rstate(rng)
        bn = rng.uniform(-1, 1)
        lam, R = orc.roe_eigen(w, w, bn)
        A = R @ np.diag(lam) @ np.linalg.inv(R)
        assert np.allclose(A, fd_jacobian(orc, w, bn), atol=1e-6)
        assert np.allclose(np.sort(lam), textbook_speeds(w, bn), atol=1e-12)


def test_roe_eigenvectors_degenerate_field(orc):
    # zero transverse field and Alfven speed equal to the sound speed: the
    # normalised eigenvectors must stay finite and independent
    w = np.array([1.0, 0.1, 0.0, 0.0, 0.6, 0.0, 0.0])
    bn = 1.0   # a^2 = gamma p / rho = 1 = bn^2 / rho
    lam, R = orc.roe_eigen(w, w, bn)
    assert np.all(np.isfinite(R))
    assert abs(np.linalg.det(R)) > 1e-6


def test_roe_positivity_fallback(orc):
    # strong rarefaction: the linearised intermediate states lose positivity,
    # so the solver falls back to HLLE
    wl = np.array([1.0, -5.0, 0.0, 0.0, 0.1, 0.0, 0.0])
    wr = np.array([1.0, 5.0, 0.0, 0.0, 0.1, 0.0, 0.0])
    f, fb = orc.riemann(0, wl, wr, 0.0)
    assert fb == 1
    assert np.all(np.isfinite(f))


def test_hlld_scale_invariance(orc):
    # rho -> a rho, p -> b p, v -> sqrt(b/a) v, B -> sqrt(b) B maps solutions to
    # solutions; fluxes scale by (sqrt(ab), b, b sqrt(b/a), sqrt(b/a) sqrt(b))
    rng = np.random.default_rng(7)
    for _ in range(20):
        wl, wr = rstate(rng), rstate(rng)
        bn = rng.uniform(-1, 1)
        a, b = rng.uniform(0.3, 3), rng.uniform(0.3, 3)
        sv, sb = math.sqrt(b / a), math.sqrt(b)
        sc = np.array([a, sv, sv, sv, b, sb, sb])
        f0, _ = orc.riemann(2, wl, wr, bn)
        f1, _ = orc.riemann(2, wl * sc, wr * sc, bn * sb)
        fs = np.array([a * sv, b, b, b, b * sv, sb * sv, sb * sv])
        assert np.allclose(f1, f0 * fs, rtol=1e-12, atol=1e-12)


def test_hlld_isolated_contact_exact(orc):
    # contact: rho jumps, v, p, B continuous, Bn != 0; exact flux is the
    # flux of the upwind state
    wl = np.array([1.0, 0.3, 0.2, -0.1, 1.0, 0.5, 0.4])
    wr = wl.copy()
    wr[0] = 0.25
    f, _ = orc.riemann(2, wl, wr, 0.7)
    assert np.allclose(f, orc.phys_flux(wl, 0.7), rtol=1e-13, atol=1e-13)
    wl[1] = wr[1] = -0.3
    f, _ = orc.riemann(2, wl, wr, 0.7)
    assert np.allclose(f, orc.phys_flux(wr, 0.7), rtol=1e-13, atol=1e-13)


def test_hlld_isolated_rotational_discontinuity_exact(orc):
    # right-going rotational discontinuity at rest frame u = 0: |Bt|, rho, p
    # unchanged, dv_t = -sign(Bn) dB_t / sqrt(rho); x/t = 0 sees the left state
    rho, p, bn = 1.3, 0.8, 0.9
    th0, th1, bt = 0.3, 1.9, 0.7
    btl = bt * np.array([math.cos(th0), math.sin(th0)])
    btr = bt * np.array([math.cos(th1), math.sin(th1)])
    vtl = np.array([0.1, -0.2])
    vtr = vtl - np.sign(bn) * (btr - btl) / math.sqrt(rho)
    wl = np.array([rho, 0.0, *vtl, p, *btl])
    wr = np.array([rho, 0.0, *vtr, p, *btr])
    f, _ = orc.riemann(2, wl, wr, bn)
    assert np.allclose(f, orc.phys_flux(wl, bn), rtol=1e-12, atol=1e-12)


TABLE1 = {
    # paper Table 1: (rho, vx, vy, vz, p, By, Bz) left / right, and Bx
    "torrilhon": ([1.0, 0, 0, 0, 1.0, 1.0, 0.0],
                  [0.2, 0, 0, 0, 0.2, math.cos(3.0), math.sin(3.0)], 1.0),
    "rj2a": ([1.08, 1.2, 0.01, 0.5, 0.95, 3.6 / math.sqrt(4 * math.pi), 2 / math.sqrt(4 * math.pi)],
             [1.0, 0, 0, 0, 1.0, 4 / math.sqrt(4 * math.pi), 2 / math.sqrt(4 * math.pi)],
             2 / math.sqrt(4 * math.pi)),
}


@pytest.mark.parametrize("name", sorted(TABLE1))
@pytest.mark.parametrize("solver", [0, 1, 2])
def test_table1_riemann_problems_finite(orc, name, solver):
    wl, wr, bn = TABLE1[name]
    f, _ = orc.riemann(solver, np.array(wl), np.array(wr), bn)
    assert np.all(np.isfinite(f))
    # the mass flux lies between the extreme one-sided values of an HLL fan
    fl, fr = orc.phys_flux(np.array(wl), bn), orc.phys_flux(np.array(wr), bn)
    assert abs(f[0]) < 10 * (abs(fl[0]) + abs(fr[0]) + 1)


def test_hlld_table1_intermediate_positive(orc):
    # HLLD's starred densities are rho (S - u)/(S - S_M); a solver that
    # returns finite fluxes with the same sign structure as HLLE on both
    # Table 1 states stays physical
    for name, (wl, wr, bn) in TABLE1.items():
        f2, _ = orc.riemann(2, np.array(wl), np.array(wr), bn)
        f1, _ = orc.riemann(1, np.array(wl), np.array(wr), bn)
        assert np.all(np.isfinite(f2)), name
        assert np.sign(f2[0]) == np.sign(f1[0]) or abs(f2[0]) < 1e-12, name
