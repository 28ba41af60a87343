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

* ``abc``: the Arnold-Beltrami-Childress force-free field of Sec. 5.1(v),
  Eq. 20, in a uniform plasma, with i.i.d. uniform velocity noise drawn from
  ``numpy.random.default_rng(seed).uniform(-amp, amp, (3, nz, ny, nx))``
  (component-major, then z, y, x).  Face values are exact area averages of
  Eq. 20 (each component is independent of its own coordinate, so the
  discrete divergence of Eq. 16 is exactly zero).
* ``abc_relaxation``: the paper's relaxation run of Sec. 5.1(v): the n = 2
  ABC field with A = B = C = sqrt(P0), the printed unstable eigenmode of
  Eqs. 21-23 added (exact face averages), and a uniform drift along the box
  diagonal of magnitude C_s / (8 sqrt(gamma)).
* ``orszag_tang``: the vortex of Sec. 5.1(iii), Eq. 18 (2D, uniform along z
  on a periodic slab).
* ``shock_tube``: the 1D Riemann problems of Table 1 (RJ2a, Torrilhon) on a
  periodic pencil: the left state fills the middle half of the pencil, the
  right state the rest, so the tabulated left|right discontinuity sits at
  3/4 of the length (a mirrored right|left one at 1/4); all fields depend on
  the pencil coordinate only.
* ``smooth``: a generalised field of the same structure (B_x = f(y, z),
  B_y = g(z, x), B_z = h(x, y)) built from a few seeded Fourier modes, periodic
  on any nx x ny x nz box of cubic cells, with seeded smooth positive density
  and pressure and smooth velocity.  Used for ragged, non-cubic test shapes.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["abc_problem", "smooth_problem", "abc_face_field", "velocity_noise", "Problem", "shock_tube",
           "SHOCK_TUBES", "abc_relaxation_problem", "eigenmode_face_field", "orszag_tang"]


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


_S4PI = math.sqrt(4.0 * math.pi)

# Table 1: (rho, vx, vy, vz, p, by, bz) left and right, the normal field bx, and
# the end time of the paper's figures
SHOCK_TUBES = {
    "rj2a": {"left": (1.08, 1.2, 0.01, 0.5, 0.95, 3.6 / _S4PI, 2.0 / _S4PI),
             "right": (1.0, 0.0, 0.0, 0.0, 1.0, 4.0 / _S4PI, 2.0 / _S4PI),
             "bx": 2.0 / _S4PI, "t_end": 0.2},
    "torrilhon": {"left": (1.0, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0),
                  "right": (0.2, 0.0, 0.0, 0.0, 0.2, math.cos(3.0), math.sin(3.0)),
                  "bx": 1.0, "t_end": 0.08},
}


def shock_tube(name: str, cells_per_unit: int = 512, length: float = 3.0, axis: int = 0,
               width: int = 8) -> Problem:
    """A Table 1 Riemann problem on a periodic pencil along ``axis``.

    The pencil has n = round(cells_per_unit * length) cells of width
    1 / cells_per_unit along ``axis`` and ``width`` cells across.  Cells whose
    centre lies in [L/4, 3L/4) hold the left state, the others the right
    state.  The problem's normal direction is ``axis`` and its two transverse
    directions are the next two axes in cyclic order, so (vx, vy, vz) and
    (bx, by, bz) of the table land on components (axis, axis + 1, axis + 2)
    mod 3.  Also returns the discontinuity's cell index ``x0`` (first right
    cell), ``t_end`` and ``axis``.
    """
    tube = SHOCK_TUBES[name]
    dx = 1.0 / cells_per_unit
    n = int(round(cells_per_unit * length))
    L = n * dx
    xc = _centres(n, dx)
    left = (xc >= 0.25 * L) & (xc < 0.75 * L)
    prof = {}
    for q, key in enumerate(("rho", "v0", "v1", "v2", "p", "b1", "b2")):
        prof[key] = np.where(left, tube["left"][q], tube["right"][q])
    prof["b0"] = np.full(n, tube["bx"])
    # problem frame arrays [zeta][eta][xi] with xi along the pencil
    frame = {k: np.broadcast_to(v[None, None, :], (width, width, n)) for k, v in prof.items()}
    # box dim i holds box axis q = 2 - i, which carries problem axis (q - axis) mod 3
    perm = [2 - ((2 - i - axis) % 3) for i in range(3)]

    def box(a):
        return np.ascontiguousarray(np.transpose(a, perm), dtype=np.float64)

    comp = {}
    for q in range(3):           # box component q = problem component (q - axis) mod 3
        pq = (q - axis) % 3
        comp["v" + "xyz"[q]] = box(frame["v%d" % pq])
        comp["b" + "xyz"[q]] = box(frame["b%d" % pq])
    x0 = int(np.flatnonzero(xc >= 0.75 * L)[0])
    return Problem(rho=box(frame["rho"]), vx=comp["vx"], vy=comp["vy"], vz=comp["vz"], p=box(frame["p"]),
                   bx=comp["bx"], by=comp["by"], bz=comp["bz"], dx=dx, x0=x0, t_end=tube["t_end"], axis=axis)


# Eqs. 21-23: each component of the eigenmode, in units of 1e-2 sqrt(P0), as
# (cos amplitude, sin amplitude, wave vector in units of 2 pi / L)
EIGENMODE = {
    0: [(2.37, 2.10, (1, 1, 0)), (-3.48, -3.18, (1, 0, 1)), (-5.86, 5.60, (0, -1, 1)), (2.08, 1.94, (1, 0, -1))],
    1: [(-2.37, -2.10, (1, 1, 0)), (-4.90, 5.37, (1, 0, 1)), (3.60, 3.80, (0, -1, 1)), (-3.00, 3.22, (1, 0, -1))],
    2: [(-3.23, 3.66, (1, 1, 0)), (3.48, 3.18, (1, 0, 1)), (3.60, 3.80, (0, -1, 1)), (2.08, 1.94, (1, 0, -1))],
}


def eigenmode_face_field(n: int, scale: float = 1.0, L: float = 1.0):
    """Face-area averages of the perturbation of Eqs. 21-23 (times scale) on
    an n^3 periodic box: component a on the a-faces, exact (the average of
    cos(k.r + phi) over a face is its centre value times the sinc factors of
    the two in-face directions)."""
    d = L / n
    out = []
    for a in range(3):
        pos = [_centres(n, d)] * 3
        pos = [p.copy() for p in pos]
        pos[a] = np.arange(n, dtype=np.float64) * d         # the face plane
        X = pos[0][None, None, :]
        Y = pos[1][None, :, None]
        Z = pos[2][:, None, None]
        f = np.zeros((n, n, n))
        for ca, sa, kv in EIGENMODE[a]:
            k = [2.0 * math.pi * q / L for q in kv]
            fac = 1.0
            for q in range(3):
                if q != a:
                    fac *= _cell_avg_factor(k[q], d)
            ph = k[0] * X + k[1] * Y + k[2] * Z
            f = f + fac * (ca * np.cos(ph) + sa * np.sin(ph))
        out.append(1e-2 * scale * f)
    return tuple(out)


def abc_relaxation_problem(n: int, rho0: float = 1.0, p0: float = 1.0, gamma: float = 5.0 / 3.0,
                           perturb: bool = True, drift: bool = True, noise: float = 1e-3,
                           seed: int = 0) -> Problem:
    """Sec. 5.1(v): n = 2 ABC field, A = B = C = sqrt(P0) (plasma beta 1),
    the eigenmode of Eqs. 21-23 and a diagonal drift V0 (1, 1, 1) / sqrt(3) with
    |V0| = C_s / (8 sqrt(gamma)), C_s = sqrt(gamma P0 / rho0).

    The n = 2 field and the eigenmode hold only wave vectors with an even
    sum of components (units 2 pi / L), so the state is invariant under a
    shift by (L/2, L/2, L/2), which an even grid keeps exactly: the n = 1
    modes of the relaxed state could never appear.  ``noise`` adds seeded
    i.i.d. uniform velocity noise in [-noise, noise] C_s (velocity_noise) to
    break that symmetry, standing in for the numerical noise from which the
    paper's n = 1 perturbation grew."""
    a = math.sqrt(p0)
    bx, by, bz = abc_face_field(n, a, a, a, mode=2)
    if perturb:
        dbx, dby, dbz = eigenmode_face_field(n, scale=math.sqrt(p0))
        bx, by, bz = bx + dbx, by + dby, bz + dbz
    shape = (n, n, n)
    cs = math.sqrt(gamma * p0 / rho0)
    v0 = cs / (8.0 * math.sqrt(gamma)) / math.sqrt(3.0) if drift else 0.0
    v = velocity_noise(shape, noise * cs, seed) if noise > 0.0 else np.zeros((3,) + shape)
    return Problem(rho=np.full(shape, rho0), vx=v[0] + v0, vy=v[1] + v0, vz=v[2] + v0,
                   p=np.full(shape, p0), bx=bx, by=by, bz=bz, dx=1.0 / n)


def orszag_tang(n: int, nz: int = 16, gamma: float = 5.0 / 3.0, rho0: float = 25.0 / (36.0 * math.pi),
                p0: float = 5.0 / (12.0 * math.pi)) -> Problem:
    """Sec. 5.1(iii), Eq. 18 on an n x n x nz periodic slab of side 1 in x, y
    (cells 1/n), uniform along z: V = C_s (-sin 2 pi y, sin 2 pi x, 0),
    B = sqrt(P0/gamma) (-sin 2 pi y, sin 4 pi x, 0), rho0, P0 constant
    (defaults give C_s = 1).  Bx on x-faces and By on y-faces are exact
    face averages (each depends on one transverse coordinate only), so the
    discrete divergence is zero."""
    dx = 1.0 / n
    shape = (nz, n, n)
    cs = math.sqrt(gamma * p0 / rho0)
    b0 = math.sqrt(p0 / gamma)
    x = _centres(n, dx)[None, None, :]
    y = _centres(n, dx)[None, :, None]
    k1, k2 = 2.0 * math.pi, 4.0 * math.pi
    vx = np.broadcast_to(-cs * np.sin(k1 * y), shape).copy()
    vy = np.broadcast_to(cs * np.sin(k1 * x), shape).copy()
    bx = np.broadcast_to(-b0 * _cell_avg_factor(k1, dx) * np.sin(k1 * y), shape).copy()
    by = np.broadcast_to(b0 * _cell_avg_factor(k2, dx) * np.sin(k2 * x), shape).copy()
    return Problem(rho=np.full(shape, rho0), vx=vx, vy=vy, vz=np.zeros(shape), p=np.full(shape, p0),
                   bx=bx, by=by, bz=np.zeros(shape), dx=dx)
