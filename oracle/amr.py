"""FP64 reference of the AMR support operators (test infrastructure only).

Prolongation from a coarse level (nc) to a fine level (2 nc) and restriction
back, for the refinement and correction operations of the paper's Sec. 3.3.
Written with explicit loops over fine cells (small grids only).

Prolongation: fine density and momentum equal the parent's; the fine energy
is the parent's pressure / (gamma - 1) + the parent's kinetic energy + half
the square of the fine cell-centred field; a fine face on a coarse face takes
that coarse value, a fine face inside a coarse cell the mean of the two coarse
faces of that cell in its direction.
Restriction: a coarse cell takes the mean of its eight children.
"""
from __future__ import annotations

import numpy as np


def prolong(Uc, Bc, gamma=5.0 / 3.0):
    nzc, nyc, nxc = Uc.shape[1:]
    nz, ny, nx = 2 * nzc, 2 * nyc, 2 * nxc
    Bf = np.empty((3, nz, ny, nx))
    Uf = np.empty((5, nz, ny, nx))
    ncs = (nxc, nyc, nzc)
    for K in range(nz):
        for J in range(ny):
            for I in range(nx):
                fc = (I, J, K)
                cc = (I // 2, J // 2, K // 2)
                for a in range(3):
                    lo = Bc[a][cc[2], cc[1], cc[0]]
                    if fc[a] % 2 == 0:
                        Bf[a, K, J, I] = lo
                    else:
                        up = list(cc)
                        up[a] = (up[a] + 1) % ncs[a]
                        Bf[a, K, J, I] = 0.5 * (lo + Bc[a][up[2], up[1], up[0]])
    for K in range(nz):
        for J in range(ny):
            for I in range(nx):
                i, j, k = I // 2, J // 2, K // 2
                bc = [0.5 * (Bc[0, k, j, i] + Bc[0, k, j, (i + 1) % nxc]),
                      0.5 * (Bc[1, k, j, i] + Bc[1, k, (j + 1) % nyc, i]),
                      0.5 * (Bc[2, k, j, i] + Bc[2, (k + 1) % nzc, j, i])]
                bf = [0.5 * (Bf[0, K, J, I] + Bf[0, K, J, (I + 1) % nx]),
                      0.5 * (Bf[1, K, J, I] + Bf[1, K, (J + 1) % ny, I]),
                      0.5 * (Bf[2, K, J, I] + Bf[2, (K + 1) % nz, J, I])]
                d = Uc[0, k, j, i]
                m = Uc[1:4, k, j, i]
                ek = 0.5 * float(m @ m) / d
                p = (gamma - 1) * (Uc[4, k, j, i] - ek - 0.5 * sum(x * x for x in bc))
                Uf[0, K, J, I] = d
                Uf[1:4, K, J, I] = m
                Uf[4, K, J, I] = p / (gamma - 1) + ek + 0.5 * sum(x * x for x in bf)
    return Uf, Bf


def restrict(Uf):
    nz, ny, nx = Uf.shape[1:]
    Uc = np.zeros((5, nz // 2, ny // 2, nx // 2))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                Uc += Uf[:, dz::2, dy::2, dx::2]
    return Uc / 8.0
