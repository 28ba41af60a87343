"""Pins of the AMR support reference (paper Sec. 3.3 refinement and
correction operations) against what their definitions fix:
each fine cell's discrete divergence (Eq. 16) equals its parent's; the area
average of the fine faces on a coarse face equals that face (Eq. 14);
restriction after prolongation returns the coarse state exactly (energy
included: conservative interpolation); linear cell data are reproduced
exactly and every child stays physical; the face-field
reconstruction reproduces any divergence-free field of its quadratic form
exactly and converges at second order on the ABC field."""
import numpy as np

from oracle import amr
from paper_1804_03479_amd import inputs

from amr_cases import regrid_case


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


def test_cell_prolongation_is_exact_for_linear_data(orc):
    # a conserved field linear along x (and constant along y, z) is
    # reproduced exactly by the limited-linear profile away from the
    # periodic wrap: each child gets the fine cell average of the line
    nz, ny, nx = 4, 4, 8
    Uc = np.zeros((5, nz, ny, nx))
    x = np.arange(nx, dtype=float)
    Uc[0] = 1.0 + 0.05 * x
    Uc[1] = 0.02 * x - 0.05
    Uc[4] = 5.0 + 0.1 * x
    Bc = np.zeros((3, nz, ny, nx))
    Bc[0] = 0.3                                   # uniform field: b2 equal in all children
    Uf, _ = amr.prolong(Uc, Bc)
    for m, (a0, a1) in ((0, (1.0, 0.05)), (1, (-0.05, 0.02)), (4, (5.0, 0.1))):
        fine_x = (np.arange(2 * nx) + 0.5) / 2 - 0.5   # fine centres in coarse-index units
        want = a0 + a1 * fine_x
        got = Uf[m, 0, 0, :]
        assert np.allclose(got[2:-2], want[2:-2], rtol=1e-14, atol=1e-14), m


def test_cell_prolongation_keeps_every_child_positive(orc):
    # a hostile field (large momentum jumps at low pressure): where the
    # linear profile would give a child non-positive density or pressure the
    # parent falls back to injection, so every child stays physical
    rng = np.random.default_rng(5)
    n = 6
    W5 = np.stack([rng.uniform(0.1, 10.0, (n, n, n)), rng.uniform(-5, 5, (n, n, n)),
                   rng.uniform(-5, 5, (n, n, n)), rng.uniform(-5, 5, (n, n, n)), rng.uniform(1e-4, 1e-2, (n, n, n))])
    Bc = 0.3 * rng.standard_normal((3, n, n, n))
    Uc = orc.prim_to_cons(W5, Bc)
    Uf, Bf = amr.prolong(Uc, Bc)
    Wf = orc.cons_to_prim(Uf, Bf)
    assert Wf[0].min() > 0 and Wf[4].min() > 0
    assert np.allclose(amr.restrict(Uf)[:4], Uc[:4], rtol=1e-13, atol=1e-13)


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


# ---- regridding (refinement / derefinement operation of Sec. 3.3)

def test_indicator_closed_form_on_the_abc_field():
    # the central-difference curl of the cell-centred ABC field is
    # sin(k dx) times the field (the discrete field stays Beltrami), so the
    # indicator |curl B| dx / |B| equals sin(2 pi / n) in every cell
    n = 32
    Bc = np.stack(inputs.abc_face_field(n))
    s = np.sin(2 * np.pi / n)
    assert amr.refine_indicator_exceeds(Bc, s * (1 - 1e-9)).all()
    assert not amr.refine_indicator_exceeds(Bc, s * (1 + 1e-9)).any()
    assert len(amr.refine_groups(Bc, s * (1 - 1e-9))) == (2 * n // 16) ** 3
    assert len(amr.refine_groups(Bc, s * (1 + 1e-9))) == 0
    assert not amr.refine_indicator_exceeds(np.ones((3, 8, 8, 8)), 1e-12).any()   # uniform field


def test_refine_groups_buffer_order_and_nesting():
    n = 32
    Bc = np.ones((3, n, n, n))
    Bc[1, 5, 9, 20] += 1.0            # a local current around coarse cell (20, 9, 5)
    hot = amr.refine_indicator_exceeds(Bc, 0.1)
    cells = {(i, j, k) for (k, j, i) in zip(*np.nonzero(hot))}
    assert cells and all(abs(i - 20) <= 1 and abs(j - 9) <= 1 and abs(k - 5) <= 1 for (i, j, k) in cells)
    g0 = amr.refine_groups(Bc, 0.1, buffer=0)
    want0 = sorted({(i // 8, j // 8, k // 8) for (i, j, k) in cells}, key=lambda t: (t[2], t[1], t[0]))
    assert [tuple(x // 16) for x in g0] == want0
    g2 = amr.refine_groups(Bc, 0.1, buffer=4)
    want2 = set()
    for (i, j, k) in cells:
        for di in (-4, 0, 4):
            for dj in (-4, 0, 4):
                for dk in (-4, 0, 4):
                    want2.add((((i + di) % n) // 8, ((j + dj) % n) // 8, ((k + dk) % n) // 8))
    got2 = [tuple(x // 16) for x in g2]
    assert set(got2) == want2 and got2 == sorted(got2, key=lambda t: (t[2], t[1], t[0]))
    # nesting: only candidates inside listed coarse groups survive
    g_n = amr.refine_groups(Bc, 0.1, buffer=4, coarse_groups=[(16, 0, 0)], coarse_edge=16)
    assert len(g_n) and all(16 <= x[0] // 2 < 32 and x[1] // 2 < 16 and x[2] // 2 < 16 for x in g_n)


def test_prolong_new_groups_without_old_groups_is_the_prolongation():
    p = inputs.smooth_problem(16, 16, 16, seed=3)
    import oracle
    Uc, Bc = oracle.initial_state(p)
    Uf, Bf = amr.prolong(Uc, Bc)
    allg = np.array([(i, j, k) for k in (0, 16) for j in (0, 16) for i in (0, 16)], dtype=np.int32)
    U2, B2 = amr.prolong_new_groups(Uc, Bc, np.zeros_like(Uf), np.zeros_like(Bf), allg, np.zeros((0, 3), np.int32))
    assert np.allclose(U2, Uf, rtol=1e-15, atol=1e-15) and np.allclose(B2, Bf, rtol=1e-15, atol=1e-15)


def test_prolong_new_groups_next_to_an_old_group():
    import oracle
    p, Uc, Bc, Uf, Bf, old = regrid_case(seed=1)
    new = np.array([[0, 0, 0], [16, 0, 0], [0, 16, 0], [16, 16, 16]], dtype=np.int32)
    U2, B2 = amr.prolong_new_groups(Uc, Bc, Uf, Bf, new, old)
    dxc = p["dx"]
    old_map = amr._in_groups(old, 16, Uf.shape[1:])
    made = amr._in_groups(new, 16, Uf.shape[1:]) & ~old_map
    # the old group's cells and faces are kept
    assert np.array_equal(U2[:, old_map], Uf[:, old_map]) and np.array_equal(B2[:, old_map], Bf[:, old_map])
    # every created fine cell has its parent's divergence (Eq. 16), twists included
    dc = oracle.divb(Bc, dxc)
    df = oracle.divb(B2, dxc / 2)
    parent = np.repeat(np.repeat(np.repeat(dc, 2, 0), 2, 1), 2, 2)
    scale = np.abs(Bc).max() / dxc
    assert np.abs(df[made] - parent[made]).max() <= 1e-12 * scale
    # the twist is real here: without giving it back the divergence would differ
    assert np.abs(dc).max() > 0 and np.abs(df[old_map]).max() <= 1e-12 * scale
    # conservative: the children of each created parent average to it
    Ur = amr.restrict(np.where(made[None], U2, 0.0))
    pm = made[::2, ::2, ::2]
    assert np.allclose(Ur[:, pm] * 1.0, Uc[:, pm] / 1.0, rtol=1e-14, atol=1e-14)
    # nothing outside the created groups moved
    rest = ~made & ~old_map
    assert np.array_equal(U2[:, rest], Uf[:, rest])
