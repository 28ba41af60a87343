"""Grid-level pins of the oracle against what the paper fixes:

* Eq. 10 telescopes: totals of mass, momentum and energy are unchanged to
  round-off on a periodic box (Sec. 5.1(v): total energy constant to machine
  precision).
* Eq. 13 + Eq. 16: the discrete divergence is unchanged by a step, for any
  initial face field, so a solenoidal field stays solenoidal to round-off.
* Sec. 5.1(i): linear slow, Alfven and fast waves along the diagonal converge
  at second order.
* Sec. 5.1(v) closed forms: magnetic energy of the ABC field; a force-free
  ABC field with zero velocity stays static up to truncation error; the
  Galilean-boosted ABC field is an exact moving solution; the A = B = C field
  is invariant under the cyclic permutation of axes.
* CFL time step on a uniform state equals the closed form built from the
  eigenvalues of the finite-difference flux Jacobian.
"""
import math

import numpy as np
import pytest

from linear_wave import wave_setup
from paper_1804_03479_amd import inputs

G = 5.0 / 3.0


def run_to(orc, U, B, dx, T, **kw):
    t = 0.0
    while t < T - 1e-14:
        dt = min(orc.cfl_dt(U, B, dx), T - t)
        U, B = orc.step(U, B, dt, dx, **kw)
        t += dt
    return U, B


@pytest.mark.parametrize("solver", [0, 1, 2])
def test_conservation_and_divergence(orc, solver):
    p = inputs.smooth_problem(12, 10, 9, seed=4)
    U, B = orc.initial_state(p)
    dx = p["dx"]
    s0 = orc.sums(U, B, dx)
    for _ in range(5):
        dt = orc.cfl_dt(U, B, dx)
        U, B = orc.step(U, B, dt, dx, riemann=solver)
    s1 = orc.sums(U, B, dx)
    assert np.all(np.abs(s1[:5] - s0[:5]) <= 1e-13 * (1 + np.abs(s0[:5])))
    assert np.abs(orc.divb(B, dx)).max() * dx < 1e-13


def test_divergence_unchanged_for_any_face_field(orc):
    rng = np.random.default_rng(9)
    p = inputs.smooth_problem(8, 9, 10, seed=1)
    U, B = orc.initial_state(p)
    B = B + 0.01 * rng.standard_normal(B.shape)   # not solenoidal
    dx = p["dx"]
    d0 = orc.divb(B, dx)
    U1, B1 = orc.step(U, B, 0.2 * orc.cfl_dt(U, B, dx), dx)
    assert np.abs(orc.divb(B1, dx) - d0).max() * dx < 1e-13


def test_cfl_uniform_state_closed_form(orc):
    from test_oracle_units import fd_jacobian
    n = 4
    w = dict(rho=1.3, v=(0.2, -0.3, 0.1), p=0.7, b=(0.5, -0.8, 0.3))
    shape = (n, n, n)
    W5 = np.stack([np.full(shape, w["rho"])] + [np.full(shape, v) for v in w["v"]] + [np.full(shape, w["p"])])
    B = np.stack([np.full(shape, b) for b in w["b"]])
    U = orc.prim_to_cons(W5, B)
    dx = 0.25
    s = 0.0
    for a in range(3):
        t1, t2 = (a + 1) % 3, (a + 2) % 3
        w1 = np.array([w["rho"], w["v"][a], w["v"][t1], w["v"][t2], w["p"], w["b"][t1], w["b"][t2]])
        lam = np.linalg.eigvals(fd_jacobian(orc, w1, w["b"][a])).real
        s += np.abs(lam).max()
    assert abs(orc.cfl_dt(U, B, dx) - 0.5 * dx / s) < 1e-6 * 0.5 * dx / s


def test_abc_magnetic_energy_closed_form(orc):
    # U_B = (A^2 + B^2 + C^2) L^3 / 2 (Sec. 5.1(v)), times the square of the
    # face-average factor sinc(k dx / 2) of Eq. 14
    n = 16
    A, Bc, C = 1.0, 0.7, 1.3
    p = inputs.abc_problem(n, 0.0, A=A, B=Bc, C=C)
    U, B = orc.initial_state(p)
    k = 2 * math.pi
    s = math.sin(k / n / 2) / (k / n / 2)
    sums = orc.sums(U, B, p["dx"])
    assert abs(sums[5] - 0.5 * (A * A + Bc * Bc + C * C) * s * s) < 1e-13
    assert abs(sums[0] - 1.0) < 1e-13
    assert np.abs(orc.divb(B, p["dx"])).max() == 0.0


def cyclic(state_cells, state_faces):
    """(x, y, z) -> (y, z, x) relabelling of a state: new(x,y,z) = P old(z,x,y)."""
    T = lambda a: np.transpose(a, (2, 0, 1))
    U = state_cells
    B = state_faces
    Un = np.stack([T(U[0]), T(U[2]), T(U[3]), T(U[1]), T(U[4])])
    Bn = np.stack([T(B[1]), T(B[2]), T(B[0])])
    return Un, Bn


def test_abc_cyclic_symmetry(orc):
    n = 12
    p = inputs.abc_problem(n, 0.0, drift=(0.05, 0.05, 0.05))
    U, B = orc.initial_state(p)
    Uc, Bc = cyclic(U, B)
    assert np.abs(Uc - U).max() < 1e-15 and np.abs(Bc - B).max() < 1e-15
    dx = p["dx"]
    for _ in range(4):
        U, B = orc.step(U, B, orc.cfl_dt(U, B, dx), dx)
    Uc, Bc = cyclic(U, B)
    assert np.abs(Bc - B).max() <= 1e-13 * np.abs(B).max()
    for m in range(5):
        assert np.abs(Uc[m] - U[m]).max() <= 1e-13 * max(np.abs(U[m]).max(), 1.0)


def boosted_abc_error(orc, n, V0=0.1, T=0.05):
    p = inputs.abc_problem(n, 0.0, drift=(V0, V0, V0))
    U, B = orc.initial_state(p)
    U, B = run_to(orc, U, B, p["dx"], T)
    d = 1.0 / n
    k = 2 * math.pi
    s = math.sin(k * d / 2) / (k * d / 2)
    c = (np.arange(n) + 0.5) * d
    X, Y, Z = c[None, None, :] - V0 * T, c[None, :, None] - V0 * T, c[:, None, None] - V0 * T
    full = (n, n, n)
    exact = np.stack([np.broadcast_to(s * (np.sin(k * Z) + np.cos(k * Y)), full),
                      np.broadcast_to(s * (np.sin(k * X) + np.cos(k * Z)), full),
                      np.broadcast_to(s * (np.sin(k * Y) + np.cos(k * X)), full)])
    return np.abs(B - exact).mean()


def test_boosted_abc_converges(orc):
    e16, e32 = boosted_abc_error(orc, 16), boosted_abc_error(orc, 32)
    assert e32 < e16 / 3.0


def static_abc_vmax(orc, n, T=0.05):
    p = inputs.abc_problem(n, 0.0)
    U, B = orc.initial_state(p)
    U, B = run_to(orc, U, B, p["dx"], T)
    W = orc.cons_to_prim(U, B)
    return np.abs(W[1:4]).mean(), np.abs(W[1:4]).max()


def test_static_abc_stays_static(orc):
    m16, x16 = static_abc_vmax(orc, 16)
    m32, x32 = static_abc_vmax(orc, 32)
    # truncation-level motion that falls with resolution (mean ~ second
    # order; the maximum sits on limiter-clipped extrema)
    assert m32 < m16 / 3.0
    assert x32 < x16 / 2.5
    assert x32 < 0.05


def linear_wave_l1(orc, n, wave, recon):
    W5, B, T, dx = wave_setup(n, wave)
    U = orc.prim_to_cons(W5, B)
    W0 = orc.cons_to_prim(U, B)
    U, B = run_to(orc, U, B, dx, T, recon=recon)
    return np.abs(orc.cons_to_prim(U, B) - W0).mean(axis=(1, 2, 3)).sum()


@pytest.mark.parametrize("wave", ["fast", "alfven", "slow"])
def test_linear_wave_second_order_unlimited(orc, wave):
    # central slopes isolate the integrator's order from limiter clipping
    e8 = linear_wave_l1(orc, 8, wave, 3)
    e16 = linear_wave_l1(orc, 16, wave, 3)
    assert e16 < e8 / 3.5


def vl_ppm_wave_l1(orc, n, wave, solver):
    W5, B, T, dx = wave_setup(n, wave)
    U = orc.prim_to_cons(W5, B)
    W0 = orc.cons_to_prim(U, B)
    U, B = run_to(orc, U, B, dx, T, scheme=0, recon=1, riemann=solver)
    return np.abs(orc.cons_to_prim(U, B) - W0).mean(axis=(1, 2, 3)).sum()


@pytest.mark.parametrize("wave", ["fast", "alfven", "slow"])
def test_vl_ppm_linear_wave_converges(orc, wave):
    # VL with limited PPM edges (Sec. 3.2 pairs either integrator with
    # either reconstruction); measured 2.6 - 3.1 at 16 -> 32 (HLLD), the
    # limiter clipping the extrema as with minmod
    e16 = vl_ppm_wave_l1(orc, 16, wave, 2)
    e32 = vl_ppm_wave_l1(orc, 32, wave, 2)
    assert e32 < e16 / 2.5, (e16, e32)


def test_vl_ppm_conservation_divergence_and_boosted_abc(orc):
    p = inputs.smooth_problem(12, 10, 9, seed=4)
    U, B = orc.initial_state(p)
    dx = p["dx"]
    s0 = orc.sums(U, B, dx)
    for _ in range(5):
        U, B = orc.step(U, B, orc.cfl_dt(U, B, dx), dx, scheme=0, recon=1, riemann=2)
    s1 = orc.sums(U, B, dx)
    assert np.all(np.abs(s1[:5] - s0[:5]) <= 1e-13 * (1 + np.abs(s0[:5])))
    assert np.abs(orc.divb(B, dx)).max() * dx < 1e-13

    def err(n, V0=0.1, T=0.05):
        q = inputs.abc_problem(n, 0.0, drift=(V0, V0, V0))
        U, B = orc.initial_state(q)
        U, B = run_to(orc, U, B, q["dx"], T, scheme=0, recon=1, riemann=2)
        d = 1.0 / n
        k = 2 * math.pi
        s = math.sin(k * d / 2) / (k * d / 2)
        c = (np.arange(n) + 0.5) * d
        X, Y, Z = c[None, None, :] - V0 * T, c[None, :, None] - V0 * T, c[:, None, None] - V0 * T
        full = (n, n, n)
        exact = np.stack([np.broadcast_to(s * (np.sin(k * Z) + np.cos(k * Y)), full),
                          np.broadcast_to(s * (np.sin(k * X) + np.cos(k * Z)), full),
                          np.broadcast_to(s * (np.sin(k * Y) + np.cos(k * X)), full)])
        return np.abs(B - exact).mean()
    assert err(32) < err(16) / 3.0


@pytest.mark.parametrize("wave", ["fast", "alfven", "slow"])
def test_linear_wave_minmod_converges(orc, wave):
    e16 = linear_wave_l1(orc, 16, wave, 0)
    e32 = linear_wave_l1(orc, 32, wave, 0)
    assert e32 < e16 / 2.5


def test_thread_count_independence(orc):
    p = inputs.abc_problem(10, 0.05, seed=3)
    U, B = orc.initial_state(p)
    dt = orc.cfl_dt(U, B, p["dx"])
    n0 = orc.get_threads()
    try:
        orc.set_threads(1)
        a = orc.step(U, B, dt, p["dx"])
        orc.set_threads(4)
        b = orc.step(U, B, dt, p["dx"])
    finally:
        orc.set_threads(n0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- CTU
def ctu_wave_l1(orc, n, wave, recon, solver):
    W5, B, T, dx = wave_setup(n, wave)
    U = orc.prim_to_cons(W5, B)
    W0 = orc.cons_to_prim(U, B)
    U, B = run_to(orc, U, B, dx, T, scheme=1, recon=recon, riemann=solver)
    return np.abs(orc.cons_to_prim(U, B) - W0).mean(axis=(1, 2, 3)).sum()


@pytest.mark.parametrize("solver", [0, 2])
def test_ctu_conservation_and_divergence(orc, solver):
    p = inputs.smooth_problem(12, 10, 9, seed=4)
    U, B = orc.initial_state(p)
    dx = p["dx"]
    s0 = orc.sums(U, B, dx)
    for _ in range(5):
        U, B = orc.step(U, B, orc.cfl_dt(U, B, dx), dx, scheme=1, recon=1, riemann=solver)
    s1 = orc.sums(U, B, dx)
    assert np.all(np.abs(s1[:5] - s0[:5]) <= 1e-13 * (1 + np.abs(s0[:5])))
    assert np.abs(orc.divb(B, dx)).max() * dx < 1e-13


def test_ctu_divergence_unchanged_for_any_face_field(orc):
    rng = np.random.default_rng(10)
    p = inputs.smooth_problem(8, 9, 10, seed=2)
    U, B = orc.initial_state(p)
    B = B + 0.01 * rng.standard_normal(B.shape)
    dx = p["dx"]
    d0 = orc.divb(B, dx)
    _, B1 = orc.step(U, B, 0.2 * orc.cfl_dt(U, B, dx), dx, scheme=1, recon=1, riemann=2)
    assert np.abs(orc.divb(B1, dx) - d0).max() * dx < 1e-13


@pytest.mark.parametrize("wave, solver", [("fast", 2), ("alfven", 2), ("slow", 2), ("slow", 0)])
def test_ctu_linear_wave_second_order_unlimited(orc, wave, solver):
    # Unlimited fourth-order PPM edges isolate the integrator's order (the
    # transverse corrections of CTU step 5 included).  At 16 -> 32 cells each
    # first-order inconsistency of the CTU states shows (measured ratios):
    # corrected states converted back with the time-n normal field instead of
    # the half-step one (Alfven 3.2, 2.4 at 32 -> 64); no momentum and energy
    # div B source in the transverse correction (slow 2.9 HLLD, 2.4 Roe);
    # HLLD with waves moving away from an edge left untraced (1D slow wave
    # 2.0).  With all three: 4.1 - 4.7.
    e16 = ctu_wave_l1(orc, 16, wave, 4, solver)
    e32 = ctu_wave_l1(orc, 32, wave, 4, solver)
    assert e32 < e16 / 3.8, (e16, e32)


@pytest.mark.parametrize("wave", ["fast", "alfven", "slow"])
def test_ctu_ppm_hlld_linear_wave_converges(orc, wave):
    e16 = ctu_wave_l1(orc, 16, wave, 1, 2)
    e32 = ctu_wave_l1(orc, 32, wave, 1, 2)
    assert e32 < e16 / 2.8


def test_ctu_plm_roe_linear_wave_converges(orc):
    # the paper's linear-wave combination: CTU + PLM + Roe (Sec. 5.1(i))
    e16 = ctu_wave_l1(orc, 16, "fast", 0, 0)
    e32 = ctu_wave_l1(orc, 32, "fast", 0, 0)
    assert e32 < e16 / 2.5


def test_ctu_boosted_abc_converges(orc):
    def err(n, V0=0.1, T=0.05):
        p = inputs.abc_problem(n, 0.0, drift=(V0, V0, V0))
        U, B = orc.initial_state(p)
        U, B = run_to(orc, U, B, p["dx"], T, scheme=1, recon=1, riemann=2)
        d = 1.0 / n
        k = 2 * math.pi
        s = math.sin(k * d / 2) / (k * d / 2)
        c = (np.arange(n) + 0.5) * d
        X, Y, Z = c[None, None, :] - V0 * T, c[None, :, None] - V0 * T, c[:, None, None] - V0 * T
        full = (n, n, n)
        exact = np.stack([np.broadcast_to(s * (np.sin(k * Z) + np.cos(k * Y)), full),
                          np.broadcast_to(s * (np.sin(k * X) + np.cos(k * Z)), full),
                          np.broadcast_to(s * (np.sin(k * Y) + np.cos(k * X)), full)])
        return np.abs(B - exact).mean()
    assert err(32) < err(16) / 4.0


def test_ctu_abc_cyclic_symmetry(orc):
    p = inputs.abc_problem(12, 0.0, drift=(0.05, 0.05, 0.05))
    U, B = orc.initial_state(p)
    dx = p["dx"]
    for _ in range(3):
        U, B = orc.step(U, B, orc.cfl_dt(U, B, dx), dx, scheme=1, recon=1, riemann=2)
    Uc, Bc = cyclic(U, B)
    assert np.abs(Bc - B).max() <= 1e-13 * np.abs(B).max()
    for m in range(5):
        assert np.abs(Uc[m] - U[m]).max() <= 1e-13 * max(np.abs(U[m]).max(), 1.0)
