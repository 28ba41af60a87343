"""Pins of the AMR support reference (paper Sec. 3.3 refinement and
correction operations) against what their definitions fix:
each fine cell's discrete divergence (Eq. 16) equals its parent's; the area
average of the fine faces on a coarse face equals that face (Eq. 14);
restriction after prolongation returns the coarse density and momentum
exactly; the fine pressure equals the parent's."""
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
    assert np.allclose(Ur[:4], Uc[:4], rtol=1e-15, atol=1e-16)
    Wc, Wf = orc.cons_to_prim(Uc, Bc), orc.cons_to_prim(Uf, Bf)
    parent_p = np.repeat(np.repeat(np.repeat(Wc[4], 2, 0), 2, 1), 2, 2)
    assert np.allclose(Wf[4], parent_p, rtol=1e-12)


def test_solenoidal_stays_solenoidal(orc):
    p = inputs.abc_problem(8, 0.05, seed=1)
    Uc, Bc = orc.initial_state(p)
    _, Bf = amr.prolong(Uc, Bc)
    assert np.abs(orc.divb(Bf, p["dx"] / 2)).max() * p["dx"] < 1e-13
