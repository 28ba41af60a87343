"""Seeded synthetic inputs for the MHD update.

This module defines problems only.  It holds none of the update's arithmetic
(no equation of state, no flux, no reconstruction, no constrained transport):
it returns primitive cell fields (density, velocity, gas pressure) and
face-area-averaged magnetic field components, which the GPU library and the
test oracle each convert to conserved variables with their own code.

Layout: every array is C-ordered ``[z][y][x]`` (x fastest), float64.
Face fields follow the staggered placement of the paper's Sec. 3.1 (Eq. 14):
``bx[k, j, i]`` is the area average of B_x over the x-face at x = i*dx (the
lower face of cell i), and likewise ``by`` on y-faces, ``bz`` on z-faces.

Problems:

* ``abc``: the Arnold-Beltrami-Childress force-free field of Sec. 4.1(v),
  Eq. 20, in a uniform plasma, with i.i.d. uniform velocity noise drawn from
  ``numpy.random.default_rng(seed).uniform(-amp, amp, (3, nz, ny, nx))``
  (component-major, then z, y, x).  Face values are exact area averages of
  Eq. 20 (each component is independent of its own coordinate, so the
  discrete divergence of Eq. 16 is exactly zero).
* ``smooth``: a generalised field of the same structure (B_x = f(y, z),
  B_y = g(z, x), B_z = h(x, y)) built from a few seeded Fourier modes, periodic
  on any nx x ny x nz box of cubic cells, with seeded smooth positive density
  and pressure and smooth velocity.  Used for ragged, non-cubic test shapes.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["abc_problem", "smooth_problem", "abc_face_field", "velocity_noise", "Problem"]


class Problem(dict):
    """dict with keys rho, vx, vy, vz, p (cell) and bx, by, bz (faces), plus dx."""

    @property
    def shape(self):
        return self["rho"].shape


def _centres(n: int, d: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * d


def _cell_avg_factor(k: float, d: float) -> float:
    """Ratio of the cell average of sin/cos(k s) to its centre value."""
    h = 0.5 * k * d
    return 1.0 if h == 0.0 else math.sin(h) / h


def abc_face_field(n: int, A: float = 1.0, B: float = 1.0, C: float = 1.0,
                   mode: int = 1, L: float = 1.0, face_average: bool = True):
    """Face-centred ABC field of Eq. 20 on an n^3 periodic box of side L.

    Returns (bx, by, bz), each (n, n, n).  With ``face_average`` the values are
    the exact area averages over each face (Eq. 14); otherwise the point value
    at the face centre.
    """
    d = L / n
    k = 2.0 * math.pi * mode / L
    s = _cell_avg_factor(k, d) if face_average else 1.0
    c = _centres(n, d)
    sx = np.sin(k * c)[None, None, :]
    cx = np.cos(k * c)[None, None, :]
    sy = np.sin(k * c)[None, :, None]
    cy = np.cos(k * c)[None, :, None]
    sz = np.sin(k * c)[:, None, None]
    cz = np.cos(k * c)[:, None, None]
    full = (n, n, n)
    bx = np.broadcast_to(s * (A * sz + C * cy), full).copy()
    by = np.broadcast_to(s * (B * sx + A * cz), full).copy()
    bz = np.broadcast_to(s * (C * sy + B * cx), full).copy()
    return bx, by, bz


def velocity_noise(shape, amp: float, seed: int) -> np.ndarray:
    """(3, nz, ny, nx) i.i.d. uniform noise in [-amp, amp] from ``seed``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(3,) + tuple(shape))


def abc_problem(n: int, amp: float = 0.01, seed: int = 0, rho0: float = 1.0,
                p0: float = 1.0, A: float = 1.0, B: float = 1.0, C: float = 1.0,
                mode: int = 1, drift=(0.0, 0.0, 0.0)) -> Problem:
    """The ABC box: uniform rho0, p0, Eq. 20 field, seeded velocity noise.

    ``drift`` adds a uniform velocity (the paper's optional diagonal drift).
    """
    bx, by, bz = abc_face_field(n, A, B, C, mode)
    shape = (n, n, n)
    if amp > 0.0:
        v = velocity_noise(shape, amp, seed)
    else:
        v = np.zeros((3,) + shape)
    return Problem(rho=np.full(shape, rho0), vx=v[0] + drift[0], vy=v[1] + drift[1],
                   vz=v[2] + drift[2], p=np.full(shape, p0), bx=bx, by=by, bz=bz,
                   dx=1.0 / n)


def smooth_problem(nx: int, ny: int, nz: int, seed: int = 0, dx: float | None = None,
                   vamp: float = 0.3, bamp: float = 1.0, modes: int = 2) -> Problem:
    """Smooth periodic state on a ragged nx x ny x nz box of cubic cells.

    Density and pressure are 1 + 0.3 * (normalised smooth field), so both stay
    within [0.7, 1.3].  B components are sums of ``modes`` seeded Fourier modes
    in the two coordinates they depend on (divergence-free by construction).
    """
    rng = np.random.default_rng(seed)
    if dx is None:
        dx = 1.0 / max(nx, ny, nz)
    Lx, Ly, Lz = nx * dx, ny * dx, nz * dx
    x = _centres(nx, dx)[None, None, :]
    y = _centres(ny, dx)[None, :, None]
    z = _centres(nz, dx)[:, None, None]
    shape = (nz, ny, nx)

    def scalar_field():
        f = np.zeros(shape)
        for _ in range(modes):
            mx, my, mz = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            f = f + np.cos(2 * math.pi * (mx * x / Lx + my * y / Ly + mz * z / Lz) + ph)
        return f / modes

    def face_component(u, Lu, nu_axis, w, Lw, nw_axis):
        # sum of modes in (u, w), exact average over the face's extent in u and w
        f = np.zeros(shape)
        for _ in range(modes):
            mu, mw = rng.integers(1, 3, size=2)
            amp = rng.uniform(0.5, 1.0)
            ph = rng.uniform(0, 2 * math.pi)
            ku, kw = 2 * math.pi * mu / Lu, 2 * math.pi * mw / Lw
            # average of cos(ku u + kw w + ph) over a dx x dx face = centre value * sinc * sinc
            fac = _cell_avg_factor(ku, dx) * _cell_avg_factor(kw, dx)
            f = f + amp * fac * np.cos(ku * u + kw * w + ph)
        return bamp * np.broadcast_to(f, shape).copy() / modes

    rho = 1.0 + 0.3 * scalar_field()
    p = 1.0 + 0.3 * scalar_field()
    vx = vamp * scalar_field()
    vy = vamp * scalar_field()
    vz = vamp * scalar_field()
    bx = face_component(y, Ly, 1, z, Lz, 0) + 0.4
    by = face_component(z, Lz, 0, x, Lx, 2) - 0.3
    bz = face_component(x, Lx, 2, y, Ly, 1) + 0.2
    return Problem(rho=rho, vx=vx, vy=vy, vz=vz, p=p, bx=bx, by=by, bz=bz, dx=dx)
