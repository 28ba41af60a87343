"""FP64 reference of the AMR support operators (test infrastructure only).

Prolongation from a coarse level (nc) to a fine level (2 nc) and restriction
back, for the refinement and correction operations of the paper's Sec. 3.3.
Written with explicit loops over coarse cells (small grids only).

Prolongation of the face field (Balsara's divergence-free reconstruction, as
the paper describes it in 2D, in 3D): a coarse face carries a linear profile
B + S_t1 t1 + S_t2 t2 in its two transverse coordinates (in units of the
coarse cell, t in [-1/2, 1/2]), with monotonized-central limited slopes of
the same face component across the neighbouring coarse faces; the four fine
faces on it take the profile at their centres (t = -1/4, +1/4).  Inside a
coarse cell the field is the quadratic
    Bx = a0 + ax x + ay y + az z + axx x^2 + axy xy + axz xz   (and cyclic)
whose face profiles match the six coarse-face profiles and whose divergence
has no x, y, z terms: axx = -(bxy + cxz)/2 with bxy (cxz) the jump of the
x-slope of By (Bz) between the upper and lower y- (z-) faces.  The interior
fine faces (the cell's mid-planes) take its values at their centres:
Bx(0, y, z) = a0 + ay y + az z with a0 = (Bx- + Bx+)/2 - axx/4 and ay, az the
mean transverse slopes of the two x-faces.  Every fine cell then has the
divergence of its parent.
Cell data (conservative): density and momentum are injected; the fine
energy is e_parent + (|b_child|^2 - <|b|^2>)/2 with b the fine cell-centred
field and <.> the mean over the eight children, so the children's energies
average to the parent's and their pressure is the parent's minus
(gamma - 1)(<|b|^2> - |b_parent|^2)/2.  Where that pressure would not be
positive, the parent's pressure is kept instead (e = p_parent / (gamma - 1)
+ parent's kinetic energy + |b_child|^2 / 2, not conservative).
Restriction: a coarse cell takes the mean of its eight children.
"""
from __future__ import annotations

import numpy as np


def mc(a, b):
    """Monotonized-central limited slope from two one-sided differences."""
    if a * b <= 0.0:
        return 0.0
    m = min(2.0 * abs(a), 2.0 * abs(b), 0.5 * abs(a + b))
    return m if a > 0 else -m


def face_slopes(Bc):
    """Limited transverse slopes S[a][t] (t = 0, 1 for the axes (a+1)%3,
    (a+2)%3) of every coarse a-face, shape (3, 2, nz, ny, nx)."""
    S = np.zeros((3, 2) + Bc.shape[1:])
    nz, ny, nx = Bc.shape[1:]
    n = (nx, ny, nz)
    for a in range(3):
        for ti, t in enumerate(((a + 1) % 3, (a + 2) % 3)):
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        c = [i, j, k]
                        up, dn = list(c), list(c)
                        up[t] = (up[t] + 1) % n[t]
                        dn[t] = (dn[t] - 1) % n[t]
                        v = Bc[a, k, j, i]
                        S[a, ti, k, j, i] = mc(Bc[a, up[2], up[1], up[0]] - v, v - Bc[a, dn[2], dn[1], dn[0]])
    return S


def prolong(Uc, Bc, gamma=5.0 / 3.0):
    nzc, nyc, nxc = Uc.shape[1:]
    nc = (nxc, nyc, nzc)
    Bf = np.empty((3,) + tuple(2 * x for x in Uc.shape[1:]))
    Uf = np.empty((5,) + Bf.shape[1:])
    S = face_slopes(Bc)

    def face(a, c):                      # coarse a-face value and slopes at cell c (lower face), periodic
        i, j, k = c[0] % nc[0], c[1] % nc[1], c[2] % nc[2]
        return Bc[a, k, j, i], S[a, 0, k, j, i], S[a, 1, k, j, i]

    for k in range(nzc):
        for j in range(nyc):
            for i in range(nxc):
                c = (i, j, k)
                for a in range(3):
                    b, cc = (a + 1) % 3, (a + 2) % 3
                    lo = face(a, c)
                    up_c = list(c)
                    up_c[a] += 1
                    hi = face(a, up_c)
                    # fine faces on the lower coarse a-face: profile at (+-1/4, +-1/4)
                    for q in range(4):
                        ob, oc = (q & 1), (q >> 1)
                        f = [2 * i, 2 * j, 2 * k]
                        f[b] += ob
                        f[cc] += oc
                        Bf[a, f[2], f[1], f[0]] = lo[0] + lo[1] * (ob - 0.5) * 0.5 + lo[2] * (oc - 0.5) * 0.5
                    # interior fine faces on the mid-plane of the cell
                    # slope of the b-face component along a: it is the slope index of axis a
                    # among (b+1)%3, (b+2)%3 of the b-faces
                    def slope_along(comp, cell, axis):
                        v = face(comp, cell)
                        t1 = (comp + 1) % 3
                        return v[1] if axis == t1 else v[2]
                    bl, bh = list(c), list(c)
                    bh[b] += 1
                    cl, ch = list(c), list(c)
                    ch[cc] += 1
                    b_xy = slope_along(b, bh, a) - slope_along(b, bl, a)
                    c_xz = slope_along(cc, ch, a) - slope_along(cc, cl, a)
                    a_xx = -0.5 * (b_xy + c_xz)
                    a0 = 0.5 * (lo[0] + hi[0]) - 0.25 * a_xx
                    a_b = 0.5 * (lo[1] + hi[1])
                    a_c = 0.5 * (lo[2] + hi[2])
                    for q in range(4):
                        ob, oc = (q & 1), (q >> 1)
                        f = [2 * i, 2 * j, 2 * k]
                        f[a] += 1
                        f[b] += ob
                        f[cc] += oc
                        Bf[a, f[2], f[1], f[0]] = a0 + a_b * (ob - 0.5) * 0.5 + a_c * (oc - 0.5) * 0.5
    nz, ny, nx = Bf.shape[1:]
    for k in range(nzc):
        for j in range(nyc):
            for i in range(nxc):
                bc = [0.5 * (Bc[0, k, j, i] + Bc[0, k, j, (i + 1) % nxc]),
                      0.5 * (Bc[1, k, j, i] + Bc[1, k, (j + 1) % nyc, i]),
                      0.5 * (Bc[2, k, j, i] + Bc[2, (k + 1) % nzc, j, i])]
                d = Uc[0, k, j, i]
                m = Uc[1:4, k, j, i]
                ek = 0.5 * float(m @ m) / d
                b2c = sum(x * x for x in bc)
                p = (gamma - 1) * (Uc[4, k, j, i] - ek - 0.5 * b2c)
                kids = [(2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2)) for q in range(8)]
                b2 = []
                for (I, J, K) in kids:
                    bf = [0.5 * (Bf[0, K, J, I] + Bf[0, K, J, (I + 1) % nx]),
                          0.5 * (Bf[1, K, J, I] + Bf[1, K, (J + 1) % ny, I]),
                          0.5 * (Bf[2, K, J, I] + Bf[2, (K + 1) % nz, J, I])]
                    b2.append(sum(x * x for x in bf))
                mean_b2 = sum(b2) / 8.0
                conservative = p - (gamma - 1) * 0.5 * (mean_b2 - b2c) > 0.0
                for (I, J, K), bb in zip(kids, b2):
                    Uf[0, K, J, I] = d
                    Uf[1:4, K, J, I] = m
                    if conservative:
                        Uf[4, K, J, I] = Uc[4, k, j, i] + 0.5 * (bb - mean_b2)
                    else:
                        Uf[4, K, J, I] = p / (gamma - 1) + ek + 0.5 * bb
    return Uf, Bf


def restrict(Uf):
    nz, ny, nx = Uf.shape[1:]
    Uc = np.zeros((5, nz // 2, ny // 2, nx // 2))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                Uc += Uf[:, dz::2, dy::2, dx::2]
    return Uc / 8.0
