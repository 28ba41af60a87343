"""Shared helpers of the shock-tube tests: profiles of a pencil in the
problem frame (normal component first, then the two transverse components in
cyclic order)."""
import numpy as np


def pencil(a, axis):
    """(..., nz, ny, nx) array -> (..., n) profile along axis, after checking
    that every transverse row is the same."""
    moved = np.moveaxis(a, a.ndim - 1 - axis, -1)
    rows = moved.reshape(moved.shape[:-3] + (-1, moved.shape[-1]))
    assert np.array_equal(rows, np.broadcast_to(rows[..., :1, :], rows.shape)), "not uniform across the pencil"
    return rows[..., 0, :]


def frame_profiles(U, B, axis):
    """Conserved U (5, ...) and face B (3, ...) of a pencil along axis ->
    (5, n), (3, n) in the problem frame."""
    order = [axis, (axis + 1) % 3, (axis + 2) % 3]
    Up = pencil(U, axis)
    Bp = pencil(B, axis)
    return np.stack([Up[0], Up[1 + order[0]], Up[1 + order[1]], Up[1 + order[2]], Up[4]]), Bp[order]
