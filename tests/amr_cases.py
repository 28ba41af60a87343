"""Shared AMR test cases (oracle pins and GPU parity use the same inputs)."""
import numpy as np

from oracle import amr
from paper_1804_03479_amd import inputs


def _curl_perturbation(shape, box, seed, amp=0.05):
    """Face field of the discrete curl of a random edge potential that is
    nonzero on the edges of the fine box [lo, hi) (inclusive of its
    boundary planes): divergence-free to round-off, and non-linear across
    the box's boundary faces."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    A = np.zeros((3,) + shape)            # A[a] on the a-edges at the lower corner of each cell
    (i0, j0, k0), (i1, j1, k1) = box
    A[:, k0:k1 + 1, j0:j1 + 1, i0:i1 + 1] = amp * rng.standard_normal((3, k1 - k0 + 1, j1 - j0 + 1, i1 - i0 + 1))
    dB = np.zeros((3,) + shape)
    # Bx = dAz/dy - dAy/dz on x-faces, cyclic (unit spacing; divergence-free discretely)
    dB[0] = (np.roll(A[2], -1, axis=1) - A[2]) - (np.roll(A[1], -1, axis=0) - A[1])
    dB[1] = (np.roll(A[0], -1, axis=0) - A[0]) - (np.roll(A[2], -1, axis=2) - A[2])
    dB[2] = (np.roll(A[1], -1, axis=2) - A[1]) - (np.roll(A[0], -1, axis=1) - A[0])
    return dB


def regrid_case(seed=0):
    """Coarse 16^3 state, fine level prolonged from it with one old group
    at (0, 0, 0) whose field is perturbed by a discrete curl reaching its
    boundary faces, the coarse faces of the old group's region reset to the
    fine means (as the restriction does)."""
    p = inputs.smooth_problem(16, 16, 16, seed=seed)
    import oracle
    Uc, Bc = oracle.initial_state(p)
    Uf, Bf = amr.prolong(Uc, Bc)
    old = np.array([[0, 0, 0]], dtype=np.int32)
    Bf = Bf + _curl_perturbation(Bf.shape[1:], ((0, 0, 0), (16, 16, 16)), seed)
    # restriction of the old group's faces (its cells and its upper boundary faces)
    Bc = Bc.copy()
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for k in range(9 if a == 2 else 8):
            for j in range(9 if a == 1 else 8):
                for i in range(9 if a == 0 else 8):
                    I = [2 * i, 2 * j, 2 * k]
                    s = 0.0
                    for q in range(4):
                        F = list(I)
                        F[b] += q & 1
                        F[c] += q >> 1
                        s += Bf[a, F[2] % 32, F[1] % 32, F[0] % 32]
                    Bc[a, k % 16, j % 16, i % 16] = 0.25 * s
    return p, Uc, Bc, Uf, Bf, old
