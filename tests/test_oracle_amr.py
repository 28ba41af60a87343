"""Pins of the AMR support reference (paper Sec. 3.3 refinement and
correction operations) against what their definitions fix:
each fine cell's discrete divergence (Eq. 16) equals its parent's; the area
average of the fine faces on a coarse face equals that face (Eq. 14);
restriction after prolongation returns the coarse state exactly (energy
included: conservative interpolation); the children's pressure is uniform; the face-field
reconstruction reproduces any divergence-free field of its quadratic form
exactly and converges at second order on the ABC field."""
import numpy as np

from oracle import amr
from paper_1804_03479_amd import inputs


def test_prolongation_properties(orc):
    p = inputs.smooth_problem(6, 5, 4, seed=2)
    Uc, Bc = orc.initial_state(p)
    rng = np.random.default_rng(0)
    Bc = Bc + 0.01 * rng.standard_normal(Bc.shape)     # non-solenoidal on purpose
    dxc = p["dx"]
    Uf, Bf = amr.prolong(Uc, Bc)
    dc = orc.divb(Bc, dxc)
    df = orc.divb(Bf, dxc / 2)
    parent = np.repeat(np.repeat(np.repeat(dc, 2, 0), 2, 1), 2, 2)
    assert np.allclose(df, parent, rtol=1e-12, atol=1e-12 * np.abs(dc).max())
    # fine faces on coarse faces average to the coarse value
    assert np.allclose(0.25 * (Bf[0][0::2, 0::2, 0::2] + Bf[0][1::2, 0::2, 0::2] + Bf[0][0::2, 1::2, 0::2] +
                               Bf[0][1::2, 1::2, 0::2]), Bc[0], rtol=1e-14, atol=1e-14)
    assert np.allclose(0.25 * (Bf[2][0::2, 0::2, 0::2] + Bf[2][0::2, 1::2, 0::2] + Bf[2][0::2, 0::2, 1::2] +
                               Bf[2][0::2, 1::2, 1::2]), Bc[2], rtol=1e-14, atol=1e-14)
    Ur = amr.restrict(Uf)
    assert np.allclose(Ur, Uc, rtol=1e-14, atol=1e-15)        # conservative, energy included
    # the children's pressure is uniform in each parent: the parent's shifted
    # by (gamma - 1)/2 (|b_parent|^2 - <|b_child|^2>)
    Wc, Wf = orc.cons_to_prim(Uc, Bc), orc.cons_to_prim(Uf, Bf)
    pf = Wf[4].reshape(Wc[4].shape[0], 2, Wc[4].shape[1], 2, Wc[4].shape[2], 2)
    assert np.allclose(pf, pf[:, :1, :, :1, :, :1], rtol=1e-12)


def test_solenoidal_stays_solenoidal(orc):
    p = inputs.abc_problem(8, 0.05, seed=1)
    Uc, Bc = orc.initial_state(p)
    _, Bf = amr.prolong(Uc, Bc)
    assert np.abs(orc.divb(Bf, p["dx"] / 2)).max() * p["dx"] < 1e-13


def _poly_field(rng, n, h):
    """Face-centre values (= exact face averages) of a divergence-free field of
    the reconstruction's quadratic form on an n^3 grid of spacing h."""
    ax, ay, az, axy, axz = rng.standard_normal(5)
    bx, by, bz, bxy, byz = rng.standard_normal(5)
    cx, cy, cxz, cyz = rng.standard_normal(4)
    a0, b0, c0 = rng.standard_normal(3)
    cz = -ax - by
    axx, byy, czz = -0.5 * (bxy + cxz), -0.5 * (axy + cyz), -0.5 * (axz + byz)

    def Bx(x, y, z):
        return a0 + ax * x + ay * y + az * z + axx * x * x + axy * x * y + axz * x * z

    def By(x, y, z):
        return b0 + bx * x + by * y + bz * z + byy * y * y + bxy * x * y + byz * y * z

    def Bz(x, y, z):
        return c0 + cx * x + cy * y + cz * z + czz * z * z + cxz * x * z + cyz * y * z

    c = (np.arange(n) + 0.5) * h
    f = np.arange(n) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(f, f, f, indexing="ij")
    return np.stack([Bx(Xf, Y, Z), By(X, Yf, Z), Bz(X, Y, Zf)])


def test_prolongation_exact_for_quadratic_divergence_free_fields():
    """Balsara's reconstruction reproduces any divergence-free field of its
    quadratic form: away from the (non-periodic) grid edges the fine faces
    equal the exact fine-face averages."""
    rng = np.random.default_rng(12)
    nc, h = 8, 1.0 / 8
    Bc = _poly_field(rng, nc, h)
    Bf_exact = _poly_field(np.random.default_rng(12), 2 * nc, h / 2)
    Uc = np.ones((5, nc, nc, nc))
    Uc[4] = 10.0
    _, Bf = amr.prolong(Uc, Bc)
    sl = slice(2, 10)          # fine cells of coarse cells 1..4 (stencils inside the grid)
    for a in range(3):
        assert np.allclose(Bf[a][sl, sl, sl], Bf_exact[a][sl, sl, sl], rtol=1e-12, atol=1e-12)


def test_prolongation_is_second_order():
    """On the smooth ABC field the error of the prolonged fine faces against
    the exact fine-face averages falls about fourfold per doubling."""
    errs = []
    for nc in (8, 16):
        Bc = np.stack(inputs.abc_face_field(nc))
        exact = np.stack(inputs.abc_face_field(2 * nc))
        Uc = np.ones((5, nc, nc, nc))
        Uc[4] = 10.0
        _, Bf = amr.prolong(Uc, Bc)
        errs.append(np.abs(Bf - exact).max())
    assert errs[0] / errs[1] > 3.5, errs
