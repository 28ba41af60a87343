"""Linear MHD waves along the box diagonal (paper Sec. 5.1(i)).

The background state and eigenvectors are not printed in the paper; this
module fixes them: rho = 1, p = 1/gamma (sound speed 1), field 1 along the
wave vector and 1.5 across it, wave vector k = 2 pi (1, 1, 1) on the unit box.
Eigenvectors come from the textbook primitive-variable Jacobian of 1D ideal
MHD (rho, u, v, w, p, By, Bz with Bx fixed), written out here and
diagonalised with numpy, so they share nothing with the oracle's Riemann
solvers.

Face field: the perturbation of B is perpendicular to k, and with all three
components of k equal the face-area averages cos(k.x) * sinc^2 give an exactly
zero discrete divergence (Eq. 16).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 5.0 / 3.0


def prim_jacobian(rho, u, v, w, p, bx, by, bz, gamma=GAMMA):
    A = np.zeros((7, 7))
    A[0] = [u, rho, 0, 0, 0, 0, 0]
    A[1] = [0, u, 0, 0, 1 / rho, by / rho, bz / rho]
    A[2] = [0, 0, u, 0, 0, -bx / rho, 0]
    A[3] = [0, 0, 0, u, 0, 0, -bx / rho]
    A[4] = [0, gamma * p, 0, 0, u, 0, 0]
    A[5] = [0, by, -bx, 0, 0, u, 0]
    A[6] = [0, bz, 0, -bx, 0, 0, u]
    return A


WAVES = {"fast": 6, "alfven": 5, "slow": 4, "entropy": 3}


def wave_setup(n: int, wave: str, amp: float = 1e-6, bpar: float = 1.0, bperp: float = 1.5):
    """Return (W5, B, period, dx): primitive cell fields and face field."""
    khat = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    e1 = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
    e2 = np.cross(khat, e1)
    rho0, p0 = 1.0, 1.0 / GAMMA
    A = prim_jacobian(rho0, 0.0, 0.0, 0.0, p0, bpar, bperp, 0.0)
    lam, R = np.linalg.eig(A)
    order = np.argsort(lam.real)
    lam, R = lam.real[order], R.real[:, order]
    idx = WAVES[wave]
    speed = lam[idx]
    r = R[:, idx] / np.max(np.abs(R[:, idx]))
    B0 = bpar * khat + bperp * e1
    dx = 1.0 / n
    kvec = 2.0 * math.pi * np.ones(3)
    kabs = np.linalg.norm(kvec)
    c = (np.arange(n) + 0.5) * dx
    X, Y, Z = c[None, None, :], c[None, :, None], c[:, None, None]
    phase_c = kvec[0] * X + kvec[1] * Y + kvec[2] * Z
    # cell averages of cos(k.x) = centre value * sinc(k_d dx / 2)^3
    h = 0.5 * kvec[0] * dx
    s1 = math.sin(h) / h
    cosc = np.cos(phase_c) * s1 ** 3
    dv = (r[1] * khat + r[2] * e1 + r[3] * e2)
    db = (r[5] * e1 + r[6] * e2)
    shape = (n, n, n)
    W5 = np.empty((5,) + shape)
    W5[0] = rho0 + amp * r[0] * cosc
    for a in range(3):
        W5[1 + a] = amp * dv[a] * cosc
    W5[4] = p0 + amp * r[4] * cosc
    B = np.empty((3,) + shape)
    # face averages: face of axis a sits at coordinate i*dx along a
    for a in range(3):
        shift = np.zeros(3)
        shift[a] = -0.5 * dx
        ph = kvec[0] * (X + shift[0]) + kvec[1] * (Y + shift[1]) + kvec[2] * (Z + shift[2])
        B[a] = np.broadcast_to(B0[a] + amp * db[a] * np.cos(ph) * s1 ** 2, shape)
    wavelength = 2.0 * math.pi / kabs
    period = wavelength / abs(speed)
    return W5, B, period, dx


def pencil_setup(nx: int, n_perp: int, wave: str, amp: float = 1e-6, t: float = 0.0,
                 bpar: float = 1.0, bperp: float = 1.5):
    """A linear wave along x on an nx x n_perp x n_perp pencil of unit length:
    the background of wave_setup with the field (bpar, bperp, 0), the
    perturbation cos(2 pi (x - c t)) along the wave's eigenvector (cell and
    face averages exact; the normal field is uniform, so the discrete
    divergence is zero).  Returns (W5, B, dx, c) with c the wave's speed."""
    rho0, p0 = 1.0, 1.0 / GAMMA
    A = prim_jacobian(rho0, 0.0, 0.0, 0.0, p0, bpar, bperp, 0.0)
    lam, R = np.linalg.eig(A)
    order = np.argsort(lam.real)
    lam, R = lam.real[order], R.real[:, order]
    idx = WAVES[wave]
    c = lam[idx]
    r = R[:, idx] / np.max(np.abs(R[:, idx]))
    k = 2.0 * math.pi
    dx = 1.0 / nx
    xc = (np.arange(nx) + 0.5) * dx
    h = 0.5 * k * dx
    cosc = np.cos(k * (xc - c * t)) * math.sin(h) / h
    shape = (n_perp, n_perp, nx)
    W5 = np.empty((5,) + shape)
    W5[0] = rho0 + amp * r[0] * cosc
    for a in range(3):
        W5[1 + a] = amp * r[1 + a] * cosc
    W5[4] = p0 + amp * r[4] * cosc
    B = np.empty((3,) + shape)
    B[0] = bpar
    B[1] = bperp + amp * r[5] * cosc
    B[2] = amp * r[6] * cosc
    return W5, B, dx, c
