"""FP64 reference of the learned interface-flux surrogate (test
infrastructure only; see the package docstring).

The surrogate replaces the HLLD Riemann solver at smooth interfaces.  It is
an addition of this project, not part of the paper; the paper's solver it
stands in for is HLLD (Sec. 3.2, CTU step 2).

Features (15), built from the left and right primitive states in the face
frame w = (rho, vn, vt1, vt2, p, Bt1, Bt2) and the shared normal field Bn,
each component divided by its interface scale (rho0, v0, v0, v0, p0, B0, B0)
with rho0 = (rhoL + rhoR)/2, p0 = (pL + pR)/2, v0 = sqrt(p0/rho0),
B0 = sqrt(p0):
  x0      the normalised mean density (1 by construction: a constant input)
  x1..x3  the normalised mean velocity (vn, vt1, vt2)
  x4      the jump size s = |d|, d = normalised (wR - wL) (the normalised mean
          pressure is 1 by construction, so its slot carries s)
  x5, x6  the normalised mean transverse field
  x7..x13 the unit jump d / s (zero when s = 0)
  x14     Bn / B0
Targets (7): the dissipative part of the HLLD flux, F_HLLD - (F(wL) +
F(wR))/2 with F the physical flux of Eq. 7, divided by s times the flux
scales (rho0 v0, p0, p0, p0, p0 v0, B0 v0, B0 v0); the surrogate flux adds
the exact central part back.  Dividing by s keeps every operand of order
one, so the BF16 rounding of the network's inputs and activations is
relative to the dissipation itself, not to the (much larger) states.  Ideal
MHD maps (rho, p, v, B) -> (a rho, b p, sqrt(b/a) v, sqrt(b) B) to a
solution, and HLLD and F commute with that map, so the normalised target
depends on the features only.

Network: 15 -> 64 -> 64 -> 7, GELU (tanh form) after both hidden layers,
linear output.  Parameters are packed W1[15][64], b1[64], W2[64][64], b2[64],
W3[64][7], b3[7] (row-major, [in][out]): 5639 values.

``bf16=True`` reproduces the GPU kernels' rounding: inputs, weights and the
activations and gradients fed to each matrix product are rounded to bfloat16
(round to nearest even); sums are exact (FP64 here, FP32 on the GPU).
"""
from __future__ import annotations

import math

import numpy as np

NIN, NH, NOUT = 15, 64, 7
SHAPES = [(NIN, NH), (NH,), (NH, NH), (NH,), (NH, NOUT), (NOUT,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)
GELU_C = math.sqrt(2.0 / math.pi)


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = math.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def scales(wl, wr):
    rho0 = 0.5 * (wl[:, 0] + wr[:, 0])
    p0 = 0.5 * (wl[:, 4] + wr[:, 4])
    v0 = np.sqrt(p0 / rho0)
    b0 = np.sqrt(p0)
    return rho0, p0, v0, b0


def state_scales(wl, wr):
    rho0, p0, v0, b0 = scales(wl, wr)
    return np.stack([rho0, v0, v0, v0, p0, b0, b0], axis=1)


def jump_size(wl, wr):
    """s = Euclidean norm of the normalised jump (wR - wL)."""
    wl, wr = np.atleast_2d(wl), np.atleast_2d(wr)
    d = (wr - wl) / state_scales(wl, wr)
    return np.sqrt((d * d).sum(axis=1))


def features(wl, wr, bn):
    """(n, 7), (n, 7), (n,) face-frame states -> (n, 15) normalised features."""
    wl, wr, bn = np.atleast_2d(wl), np.atleast_2d(wr), np.atleast_1d(bn)
    sc = state_scales(wl, wr)
    mean = 0.5 * (wl + wr) / sc
    d = (wr - wl) / sc
    s = np.sqrt((d * d).sum(axis=1))
    unit = np.where(s[:, None] > 0, d / np.where(s > 0, s, 1.0)[:, None], 0.0)
    x = np.empty((wl.shape[0], NIN))
    x[:, 0] = mean[:, 0]
    x[:, 1:4] = mean[:, 1:4]
    x[:, 4] = s
    x[:, 5:7] = mean[:, 5:7]
    x[:, 7:14] = unit
    x[:, 14] = bn / sc[:, 5]
    return x


def flux_scales(wl, wr):
    rho0, p0, v0, b0 = scales(np.atleast_2d(wl), np.atleast_2d(wr))
    return np.stack([rho0 * v0, p0, p0, p0, p0 * v0, b0 * v0, b0 * v0], axis=1)


def output_scales(wl, wr):
    """What the network output is multiplied by: s times the flux scales."""
    return flux_scales(wl, wr) * jump_size(wl, wr)[:, None]


def fallback(wl, wr, dp: float = 0.3, drho: float = 0.3):
    """True where a jump is strong enough to use HLLD instead of the network."""
    wl, wr = np.atleast_2d(wl), np.atleast_2d(wr)
    jp = np.abs(wr[:, 4] - wl[:, 4]) / np.minimum(wl[:, 4], wr[:, 4])
    jr = np.abs(wr[:, 0] - wl[:, 0]) / np.minimum(wl[:, 0], wr[:, 0])
    return (jp > dp) | (jr > drho)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + 0.044715 * x ** 3)))


def gelu_prime(x):
    t = np.tanh(GELU_C * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3 * 0.044715 * x * x)


def forward(theta, X, bf16_ops: bool = False):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    r = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    Z1 = Xb @ r(W1) + b1
    H1 = r(gelu(Z1))
    Z2 = H1 @ r(W2) + b2
    H2 = r(gelu(Z2))
    Y = H2 @ r(W3) + b3
    return Y, (Xb, Z1, H1, Z2, H2)


def backward(theta, cache, dY, bf16_ops: bool = False):
    """Gradients of sum(dY * Y) with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    r = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    Xb, Z1, H1, Z2, H2 = cache
    dYb = r(dY)
    gW3 = H2.T @ dYb
    gb3 = dY.sum(axis=0)
    dZ2 = (dYb @ r(W3).T) * gelu_prime(Z2)
    dZ2b = r(dZ2)
    gW2 = H1.T @ dZ2b
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2b @ r(W2).T) * gelu_prime(Z1)
    dZ1b = r(dZ1)
    gW1 = Xb.T @ dZ1b
    gb1 = dZ1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def mse(theta, X, T):
    Y, _ = forward(theta, X)
    return float(np.mean((Y - T) ** 2))


def mse_grad(theta, X, T, bf16_ops: bool = False):
    Y, cache = forward(theta, X, bf16_ops)
    dY = 2.0 * (Y - T) / Y.size
    return float(np.mean((Y - T) ** 2)), backward(theta, cache, dY, bf16_ops)


def adam(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba) at step t >= 1; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def physical_flux(w, bn, gamma: float = 5.0 / 3.0):
    """Eq. 7 along the face normal for face-frame primitive states (n, 7)."""
    w, bn = np.atleast_2d(w), np.atleast_1d(bn)
    d, vn, v1, v2, p, b1, b2 = (w[:, m] for m in range(7))
    b2sum = bn * bn + b1 * b1 + b2 * b2
    pt = p + 0.5 * b2sum
    e = p / (gamma - 1.0) + 0.5 * d * (vn * vn + v1 * v1 + v2 * v2) + 0.5 * b2sum
    vb = vn * bn + v1 * b1 + v2 * b2
    return np.stack([d * vn, d * vn * vn + pt - bn * bn, d * vn * v1 - bn * b1, d * vn * v2 - bn * b2,
                     (e + pt) * vn - bn * vb, b1 * vn - bn * v1, b2 * vn - bn * v2], axis=1)


def central_flux(wl, wr, bn, gamma: float = 5.0 / 3.0):
    return 0.5 * (physical_flux(wl, bn, gamma) + physical_flux(wr, bn, gamma))


def targets(wl, wr, bn, flux, gamma: float = 5.0 / 3.0):
    """Normalised training targets of faces whose Riemann flux is `flux`."""
    osc = output_scales(wl, wr)
    d = np.atleast_2d(flux) - central_flux(wl, wr, bn, gamma)
    return np.where(osc > 0, d / np.where(osc > 0, osc, 1.0), 0.0)


def surrogate_flux(theta, wl, wr, bn, bf16_ops: bool = False, gamma: float = 5.0 / 3.0):
    """Surrogate flux (n, 7) in the face frame: exact central part plus the
    de-normalised network output."""
    Y, _ = forward(theta, features(wl, wr, bn), bf16_ops)
    return central_flux(wl, wr, bn, gamma) + Y * output_scales(wl, wr)
