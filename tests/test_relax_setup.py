"""Pins of the ABC relaxation set-up (paper Sec. 5.1(v)) and of its
diagnostics against the closed forms the paper states: U_B = (A^2 + B^2 +
C^2) L^3 / 2 and H = U_B L / (pi n) for an ABC field of n periods; the
eigenmode of Eqs. 21-23 is divergence-free with wave vectors of length
sqrt 2 (2 pi / L); its face values are exact face averages (checked by
quadrature); the drift has magnitude C_s / (8 sqrt gamma) along the
diagonal."""
import math

import numpy as np
import pytest

import oracle
from paper_1804_03479_amd import inputs, relax


@pytest.mark.parametrize("mode", [1, 2])
def test_helicity_and_energy_of_abc_fields(mode):
    n = 128
    A, B, C = 0.33, 0.85, 0.80
    bx, by, bz = inputs.abc_face_field(n, A, B, C, mode=mode)
    Bc = relax.cell_centred(np.stack([bx, by, bz]))
    UB = 0.5 * (Bc ** 2).sum() / n ** 3
    assert UB == pytest.approx((A * A + B * B + C * C) / 2, rel=2e-3)
    H = relax.helicity(Bc)
    assert H > 0                                      # right-handed, like the paper's field
    assert H == pytest.approx(UB / (math.pi * mode), rel=2e-3)
    fr = relax.shell_fractions(Bc)
    assert fr["%.4f" % float(mode)] > 1 - 1e-12
    if mode == 1:
        amps = relax.abc1_amplitudes(Bc)
        assert np.allclose(amps, (A, B, C), rtol=2e-3)


def test_eigenmode_is_solenoidal_with_sqrt2_wavevectors():
    n = 32
    d = inputs.eigenmode_face_field(n)
    B = np.stack(d)
    assert np.abs(oracle.divb(B, 1.0 / n)).max() / n < 1e-15 * 100
    fr = relax.shell_fractions(relax.cell_centred(B))
    assert fr["%.4f" % math.sqrt(2.0)] > 1 - 1e-12


def test_eigenmode_face_values_are_face_averages():
    n = 16
    bx, by, bz = inputs.eigenmode_face_field(n)
    h = 1.0 / n
    xg, wg = np.polynomial.legendre.leggauss(8)

    def point(a, x, y, z):
        v = 0.0
        for ca, sa, kv in inputs.EIGENMODE[a]:
            ph = 2 * math.pi * (kv[0] * x + kv[1] * y + kv[2] * z)
            v += ca * math.cos(ph) + sa * math.sin(ph)
        return 1e-2 * v

    rng = np.random.default_rng(0)
    for _ in range(5):
        i, j, k = rng.integers(0, n, 3)
        for a, arr in enumerate((bx, by, bz)):
            lo = [i * h, j * h, k * h]
            s = 0.0
            for u, wu in zip(xg, wg):
                for v, wv in zip(xg, wg):
                    c = list(lo)
                    b_, c_ = (a + 1) % 3, (a + 2) % 3
                    c[b_] = lo[b_] + 0.5 * h * (u + 1)
                    c[c_] = lo[c_] + 0.5 * h * (v + 1)
                    s += 0.25 * wu * wv * point(a, *c)
            assert arr[k, j, i] == pytest.approx(s, abs=1e-14)


def test_relaxation_problem_matches_the_stated_set_up():
    gam = 5.0 / 3.0
    p = inputs.abc_relaxation_problem(32, noise=0.0)
    v = np.array([p["vx"][0, 0, 0], p["vy"][0, 0, 0], p["vz"][0, 0, 0]])
    q = inputs.abc_relaxation_problem(32, noise=1e-3, seed=1)
    dv = np.stack([q["vx"], q["vy"], q["vz"]]) - v[:, None, None, None]
    assert 0.9e-3 * math.sqrt(gam) < np.abs(dv).max() <= 1e-3 * math.sqrt(gam)
    assert np.allclose(v, v[0]) and v[0] > 0
    assert np.linalg.norm(v) == pytest.approx(math.sqrt(gam) / (8 * math.sqrt(gam)), rel=1e-14)
    U, B = oracle.initial_state(p)
    assert np.abs(oracle.divb(B, p["dx"])).max() * p["dx"] < 1e-14
    base = np.stack(inputs.abc_face_field(32, 1.0, 1.0, 1.0, mode=2))
    dB = B - base
    assert 0.005 < np.abs(dB).max() < 0.3          # a percent-level perturbation
