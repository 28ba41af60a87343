"""Pins of the Orszag-Tang set-up (paper Sec. 5.1(iii), Eq. 18): the sound
speed is one with the default rho0, P0; the field is divergence-free on the
slab (exact face averages); velocity and field follow Eq. 18 at cell
centres / face centres (up to the face-average factor)."""
import math

import numpy as np

import oracle
from paper_1804_03479_amd import inputs


def test_orszag_tang_set_up():
    n = 32
    p = inputs.orszag_tang(n, nz=16)
    gam = 5.0 / 3.0
    assert math.sqrt(gam * p["p"][0, 0, 0] / p["rho"][0, 0, 0]) == np.float64(1.0) or \
        abs(math.sqrt(gam * p["p"][0, 0, 0] / p["rho"][0, 0, 0]) - 1.0) < 1e-15
    U, B = oracle.initial_state(p)
    assert np.abs(oracle.divb(B, p["dx"])).max() * p["dx"] < 1e-15
    y = (np.arange(n) + 0.5) / n
    x = y
    assert np.allclose(p["vx"][0, :, 0], -np.sin(2 * np.pi * y), atol=1e-15)
    assert np.allclose(p["vy"][0, 0, :], np.sin(2 * np.pi * x), atol=1e-15)
    b0 = math.sqrt(p["p"][0, 0, 0] / gam)
    h = math.pi / n
    assert np.allclose(p["bx"][0, :, 0], -b0 * math.sin(h) / h * np.sin(2 * np.pi * y), atol=1e-15)
    h2 = 2 * math.pi / n
    assert np.allclose(p["by"][0, 0, :], b0 * math.sin(h2) / h2 * np.sin(4 * np.pi * x), atol=1e-15)
    assert np.all(p["bz"] == 0) and np.all(p["vz"] == 0)
    # uniform along z
    assert np.array_equal(p["bx"], np.broadcast_to(p["bx"][:1], p["bx"].shape))
