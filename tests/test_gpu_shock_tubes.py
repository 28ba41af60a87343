"""The Table 1 Riemann problems (paper Sec. 5.1(ii)) through the C ABI:
parity with the oracle on a coarse pencil, the same solution along x, y and
z, and at the paper's resolution (512 cells per unit length, PPM + Roe, FP64)
positive density and pressure everywhere and fast shocks captured in at most
4 cells.  The paper's Dirichlet ends are replaced by a periodic pencil three
units long, with the tabulated left|right discontinuity at x = 2.25; its
waves stay clear of the mirrored right|left discontinuity at x = 0.75 up to
the end times used here."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1804_03479_amd import inputs  # noqa: E402
from paper_1804_03479_amd.mhd import Level, Solver  # noqa: E402

from shock_tube_util import frame_profiles  # noqa: E402

SOLVERS = {"roe": oracle.ROE, "hlle": oracle.HLLE, "hlld": oracle.HLLD}
SCHEMES = {"ctu_ppm": ("ctu", "ppm", oracle.CTU, oracle.PPM), "vl_plm": ("vl", "plm", oracle.VL, oracle.PLM)}


def level_of(p):
    U, B = oracle.initial_state(p)
    return Level(torch.from_numpy(U).cuda().contiguous(), torch.from_numpy(B).cuda().contiguous(), p["dx"])


def fetch(lv):
    torch.cuda.synchronize()
    return lv.U.cpu().numpy(), lv.B.cpu().numpy()


@pytest.mark.parametrize("solver", sorted(SOLVERS))
@pytest.mark.parametrize("scheme", sorted(SCHEMES))
@pytest.mark.parametrize("name", ["rj2a", "torrilhon"])
def test_tube_parity_with_oracle(name, scheme, solver):
    sch, rec, osch, orec = SCHEMES[scheme]
    p = inputs.shock_tube(name, 32, 3.0, axis=0, width=4)
    U, B = oracle.initial_state(p)
    s = Solver(sch, rec, solver)
    lv = level_of(p)
    for _ in range(10):
        dt = oracle.cfl_dt(U, B, p["dx"])
        assert abs(s.cfl_dt(lv) - dt) <= 1e-13 * dt
        s.step(lv, dt)
        U, B = oracle.step(U, B, dt, p["dx"], scheme=osch, recon=orec, riemann=SOLVERS[solver])
    Ug, Bg = fetch(lv)
    for m in range(5):
        assert np.abs(Ug[m] - U[m]).max() <= 1e-12 * np.abs(U[m]).max(), m
    for m in range(3):
        assert np.abs(Bg[m] - B[m]).max() <= 1e-12 * np.abs(B).max(), m


def run_to(s, lv, t_end):
    t = 0.0
    while t < t_end:
        dt = min(s.cfl_dt(lv), t_end - t)
        s.step(lv, dt)
        t += dt
    return fetch(lv)


def run_tubes(name, cells_per_unit=512):
    out = []
    for axis in range(3):
        p = inputs.shock_tube(name, cells_per_unit, 3.0, axis=axis, width=4)
        s = Solver("ctu", "ppm", "roe")
        U, B = run_to(s, level_of(p), p["t_end"])
        s.close()
        out.append((p, frame_profiles(U, B, axis)))
    return out


def fast_shock_width(rho, upstream, start, direction):
    """10-90 % width (cells) of the first jump met when walking from the
    untouched upstream region at index start in direction (+1 / -1)."""
    i = start
    while abs(rho[i] - upstream) <= 1e-8 * upstream:
        i += direction
    front = i
    down = rho[front + 12 * direction]       # the post-shock plateau
    jump = down - upstream
    lo, hi = upstream + 0.1 * jump, upstream + 0.9 * jump
    seg = rho[front:front + 20 * direction:direction]
    inside = (seg - lo) * (seg - hi) < 0
    return int(inside.sum()), front, jump


@pytest.mark.parametrize("name", ["rj2a", "torrilhon"])
def test_tube_at_paper_resolution(name):
    res = run_tubes(name)
    (p, (Uf, Bf)) = res[0]
    for axis, (_, (Ua, Ba)) in enumerate(res[1:], start=1):
        dU = np.abs(Ua - Uf).max(axis=1) / np.abs(Uf).max()
        dB = np.abs(Ba - Bf).max(axis=1) / np.abs(Bf).max()
        print(name, "axis", axis, "max relative difference U", dU, "B", dB)
        # the three directions share their arithmetic up to FMA contraction and
        # the order of the CFL sum; Torrilhon's compound wave (a structure
        # that depends on small perturbations) amplifies that round-off more
        # than RJ2a does, a direction-dependent error would move whole waves
        # (differences of the order of the jumps, 1e-2 and above)
        bar = 1e-10 if name == "rj2a" else 1e-8
        assert dU.max() <= bar and dB.max() <= bar, (axis, dU, dB)
    gam = 5.0 / 3.0
    rho = Uf[0]
    bc = np.stack([0.5 * (Bf[0] + np.roll(Bf[0], -1)), Bf[1], Bf[2]])
    pres = (gam - 1) * (Uf[4] - 0.5 * (Uf[1] ** 2 + Uf[2] ** 2 + Uf[3] ** 2) / rho - 0.5 * (bc ** 2).sum(0))
    assert rho.min() > 0 and pres.min() > 0
    # the normal field stays uniform (div B = 0 in 1D)
    assert np.abs(Bf[0] - inputs.SHOCK_TUBES[name]["bx"]).max() <= 1e-13
    if name == "rj2a":
        t = inputs.SHOCK_TUBES[name]
        x0 = p["x0"]
        w_r, f_r, j_r = fast_shock_width(rho, t["right"][0], x0 + 300, -1)
        w_l, f_l, j_l = fast_shock_width(rho, t["left"][0], x0 - 300, +1)
        assert f_r > x0 + 50 and f_l < x0 - 10, (f_r, f_l)
        assert abs(j_r) > 0.1 and abs(j_l) > 0.1, (j_r, j_l)
        assert w_r <= 4 and w_l <= 4, (w_r, w_l)
