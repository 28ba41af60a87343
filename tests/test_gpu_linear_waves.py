"""Linear-wave convergence at the paper's set-up (Sec. 5.1(i)): CTU + PLM +
Roe in double precision, slow, Alfven and fast waves of relative amplitude
1e-6 along the box diagonal for one period, L1 error of the primitive
variables against the initial state (the paper's E_L1) at 32^3, 64^3 and
128^3 on the GPU.  The paper finds the error inversely proportional to the
square of the cell count per dimension.  With the minmod limiter that order
is reached only as the resolution grows (the limiter clips the wave's
extrema to first order on coarse grids: measured ratios 2.0-2.2 from 32^3
to 64^3 for the slow and Alfven waves, 3.2-3.4 from 64^3 to 128^3), so the
finest doubling must cut the error by more than 3.2 and the observed order
must rise with resolution."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1804_03479_amd.mhd import Solver  # noqa: E402

from linear_wave import wave_setup  # noqa: E402


def l1_error(n, wave, recon="plm", solver="roe"):
    W5, B, T, dx = wave_setup(n, wave)
    s = Solver("ctu", recon, solver, "f64")
    lv = s.level_from_primitives(torch.from_numpy(W5), torch.from_numpy(B), dx)
    U0 = lv.U.cpu().numpy()
    W0 = oracle.cons_to_prim(U0, B)
    t = 0.0
    while t < T * (1.0 - 1e-12):
        dt = min(s.cfl_dt(lv), T - t)
        s.step(lv, dt)
        t += dt
    torch.cuda.synchronize()
    U, Bf = lv.U.cpu().numpy(), lv.B.cpu().numpy()
    s.close()
    return float(np.abs(oracle.cons_to_prim(U, Bf) - W0).mean(axis=(1, 2, 3)).sum())


@pytest.mark.parametrize("wave", ["slow", "alfven", "fast"])
def test_linear_waves_converge_at_second_order(wave):
    e = [l1_error(n, wave) for n in (32, 64, 128)]
    order = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    print(wave, e, order)
    # measured e64 / e128 = 3.54 - 3.58 (order 1.82 - 1.84, rising as the
    # minmod limiter stops clipping the extrema)
    assert e[1] / e[2] > 3.4 and order[1] > order[0], (wave, e)
    assert e[2] < 1e-7, (wave, e)     # well below the 1e-6 amplitude (summed over the five fields)


@pytest.mark.parametrize("wave", ["slow", "alfven", "fast"])
def test_benchmark_scheme_linear_waves_converge(wave):
    # the precision form's scheme, CTU + PPM + HLLD, on the same waves
    e = [l1_error(n, wave, "ppm", "hlld") for n in (32, 64, 128)]
    order = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    print("ppm+hlld", wave, e, order)
    assert e[1] / e[2] > 3.0, (wave, e)
    assert e[2] < 1e-7, (wave, e)
