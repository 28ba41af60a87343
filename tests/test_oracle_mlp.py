"""Pins of the surrogate-flux reference (an addition, not the paper's):

* backward() equals central finite differences of the FP64 loss;
* the features and targets are invariant under the ideal-MHD scaling map,
  checked against the HLLD oracle itself (scaled states give identical
  normalised HLLD fluxes), so a network of these features can represent HLLD;
* the numpy physical flux equals the C oracle's, and the target (HLLD minus
  the central flux) vanishes for equal states;
* Adam reduces the loss on a fixed batch; the fallback test flags jumps.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def sample_states(rng, n, jump=0.1):
    base = np.stack([rng.uniform(0.5, 2, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n),
                     rng.uniform(0.5, 2, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)], axis=1)
    pert = 1.0 + jump * rng.uniform(-1, 1, (n, 7))
    return base, base * pert, rng.uniform(-1, 1, n)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1) + 0.01 * rng.standard_normal(mlp.NPARAM)
    X = rng.standard_normal((32, mlp.NIN))
    T = rng.standard_normal((32, mlp.NOUT))
    _, g = mlp.mse_grad(theta, X, T)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    for i in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.mse(tp, X, T) - mlp.mse(tm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_gelu_derivative():
    x = np.linspace(-4, 4, 101)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_prime(x), fd, atol=1e-8)
    assert abs(mlp.gelu(np.array([0.0]))[0]) == 0.0
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


def test_normalisation_matches_hlld_scaling(orc):
    rng = np.random.default_rng(3)
    wl, wr, bn = sample_states(rng, 20, jump=0.5)
    X = mlp.features(wl, wr, bn)
    for _ in range(3):
        a, b = rng.uniform(0.3, 3), rng.uniform(0.3, 3)
        sc = np.array([a, math.sqrt(b / a), math.sqrt(b / a), math.sqrt(b / a), b, math.sqrt(b), math.sqrt(b)])
        X2 = mlp.features(wl * sc, wr * sc, bn * math.sqrt(b))
        assert np.allclose(X2, X, rtol=1e-14, atol=1e-14)
        for n in range(5):
            f1, _ = orc.riemann(orc.HLLD, wl[n], wr[n], bn[n])
            f2, _ = orc.riemann(orc.HLLD, wl[n] * sc, wr[n] * sc, bn[n] * math.sqrt(b))
            t1 = mlp.targets(wl[n], wr[n], bn[n], f1)[0]
            t2 = mlp.targets(wl[n] * sc, wr[n] * sc, bn[n] * math.sqrt(b), f2)[0]
            assert np.allclose(t1, t2, rtol=1e-12, atol=1e-12)


def test_features_are_a_lossless_reparameterisation():
    """The two states come back from the features and the scales rho0, p0:
    w = (mean -/+ s unit / 2) * scale, with mean rho = mean p = 1."""
    rng = np.random.default_rng(10)
    wl, wr, bn = sample_states(rng, 30, jump=0.3)
    x = mlp.features(wl, wr, bn)
    rho0, p0 = 0.5 * (wl[:, 0] + wr[:, 0]), 0.5 * (wl[:, 4] + wr[:, 4])
    v0, b0 = np.sqrt(p0 / rho0), np.sqrt(p0)
    sc = np.stack([rho0, v0, v0, v0, p0, b0, b0], axis=1)
    mean = np.stack([x[:, 0], x[:, 1], x[:, 2], x[:, 3], np.ones(30), x[:, 5], x[:, 6]], axis=1)
    half = 0.5 * x[:, 4:5] * x[:, 7:14]
    assert np.allclose((mean - half) * sc, wl, rtol=1e-13, atol=1e-13)
    assert np.allclose((mean + half) * sc, wr, rtol=1e-13, atol=1e-13)
    assert np.allclose(x[:, 14] * b0, bn, rtol=1e-13, atol=1e-13)
    assert np.allclose(x[:, 0], 1.0, rtol=1e-15)
    # equal states: zero jump and zero unit vector
    x0 = mlp.features(wl[:1], wl[:1], bn[:1])
    assert x0[0, 4] == 0.0 and np.all(x0[0, 7:14] == 0.0)


def test_physical_flux_matches_c_oracle_and_consistency(orc):
    """Eq. 7 in numpy equals the C oracle's flux, and the target of a face
    with equal states is zero (a consistent Riemann flux is F(w) there)."""
    rng = np.random.default_rng(9)
    wl, wr, bn = sample_states(rng, 12, jump=0.4)
    F = mlp.physical_flux(wl, bn)
    for n in range(12):
        assert np.allclose(F[n], orc.phys_flux(wl[n], bn[n]), rtol=1e-14, atol=1e-14)
        f, _ = orc.riemann(orc.HLLD, wl[n], wl[n], bn[n])
        assert np.abs(mlp.targets(wl[n], wl[n], bn[n], f)).max() <= 1e-13
    # a zero network reproduces the central flux
    theta = np.zeros(mlp.NPARAM)
    assert np.allclose(mlp.surrogate_flux(theta, wl, wr, bn), mlp.central_flux(wl, wr, bn), rtol=0, atol=0)


def test_adam_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((256, mlp.NIN))
    T = np.tanh(X[:, :mlp.NOUT]) * 0.5
    theta = mlp.init_params(2)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.mse(theta, X, T)
    for t in range(1, 201):
        _, g = mlp.mse_grad(theta, X, T)
        theta, m, v = mlp.adam(theta, m, v, g, t, 3e-3)
    assert mlp.mse(theta, X, T) < 0.2 * l0


def test_fallback_flags_strong_jumps():
    wl = np.array([[1.0, 0, 0, 0, 1.0, 0, 0]] * 4)
    wr = wl.copy()
    wr[1, 4] = 1.35   # pressure jump 35 %
    wr[2, 0] = 0.7    # density jump 43 %
    wr[3, 4] = 1.25   # 25 %: smooth
    assert list(mlp.fallback(wl, wr)) == [False, True, True, False]


def test_bf16_rounding():
    # bfloat16 keeps 7 mantissa bits: spacing 2^-7 just above 1
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -8, -3.14159])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # halfway, ties to the even mantissa 0
    assert r[2] == 1.0                      # below halfway
    assert r[3] == 1.0 + 2 ** -6            # halfway between mantissas 1 and 2: to 2
    assert r[4] == -3.140625
