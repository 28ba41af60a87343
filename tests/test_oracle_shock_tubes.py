"""Pins of the oracle on the Table 1 Riemann problems (paper Sec. 5.1(ii)):
the same tube along x, y and z gives the same profiles (a transposed index or
a swapped component in one direction's sweep breaks this), the totals of the
periodic pencil are conserved, and the initial data hold the tabulated
states with a divergence-free field."""
import numpy as np
import pytest

import oracle
from paper_1804_03479_amd import inputs

from shock_tube_util import frame_profiles


@pytest.mark.parametrize("name", ["rj2a", "torrilhon"])
def test_initial_states_follow_table_1(name):
    t = inputs.SHOCK_TUBES[name]
    p = inputs.shock_tube(name, 16, 3.0, axis=1, width=4)
    x0 = p["x0"]
    for key, q in (("rho", 0), ("vy", 1), ("vz", 2), ("vx", 3), ("p", 4)):
        prof = p[key][0, :, 0]
        assert prof[x0 - 1] == t["left"][q] and prof[x0] == t["right"][q]
    assert np.all(p["by"] == t["bx"])
    assert p["bz"][0, x0 - 1, 0] == t["left"][5] and p["bx"][0, x0, 0] == t["right"][6]
    U, B = oracle.initial_state(p)
    assert np.abs(oracle.divb(B, p["dx"])).max() == 0.0


@pytest.mark.parametrize("scheme,recon", [(oracle.CTU, oracle.PPM), (oracle.VL, oracle.PLM)])
@pytest.mark.parametrize("name", ["rj2a", "torrilhon"])
def test_oracle_tube_is_direction_independent_and_conservative(name, scheme, recon):
    res = []
    for axis in range(3):
        p = inputs.shock_tube(name, 16, 3.0, axis=axis, width=4)
        U, B = oracle.initial_state(p)
        tot0 = U.reshape(5, -1).sum(1)
        for _ in range(4):
            dt = oracle.cfl_dt(U, B, p["dx"])
            U, B = oracle.step(U, B, dt, p["dx"], scheme=scheme, recon=recon, riemann=oracle.ROE)
        tot = U.reshape(5, -1).sum(1)
        scale = np.abs(U).reshape(5, -1).sum(1)
        assert np.all(np.abs(tot - tot0) <= 1e-13 * scale)
        res.append(frame_profiles(U, B, axis))
    for Ua, Ba in res[1:]:
        assert np.allclose(Ua, res[0][0], rtol=1e-14, atol=1e-14)
        assert np.allclose(Ba, res[0][1], rtol=1e-14, atol=1e-14)
    # the waves left the initial profile
    p = inputs.shock_tube(name, 16, 3.0, axis=0, width=4)
    assert np.abs(res[0][0][0] - p["rho"][0, 0]).max() > 1e-2
