"""FP64 reference of the AMR support operators (test infrastructure only).

Prolongation from a coarse level (nc) to a fine level (2 nc) and restriction
back, for the refinement and correction operations of the paper's Sec. 3.3.
Written with explicit loops over coarse cells (small grids only).

Prolongation of the face field (Balsara's divergence-free reconstruction, as
the paper describes it in 2D, in 3D): a coarse face carries a linear profile
B + S_t1 t1 + S_t2 t2 in its two transverse coordinates (in units of the
coarse cell, t in [-1/2, 1/2]), with monotonized-central limited slopes of
the same face component across the neighbouring coarse faces; the four fine
faces on it take the profile at their centres (t = -1/4, +1/4).  Inside a
coarse cell the field is the quadratic
    Bx = a0 + ax x + ay y + az z + axx x^2 + axy xy + axz xz   (and cyclic)
whose face profiles match the six coarse-face profiles and whose divergence
has no x, y, z terms: axx = -(bxy + cxz)/2 with bxy (cxz) the jump of the
x-slope of By (Bz) between the upper and lower y- (z-) faces.  The interior
fine faces (the cell's mid-planes) take its values at their centres:
Bx(0, y, z) = a0 + ay y + az z with a0 = (Bx- + Bx+)/2 - axx/4 and ay, az the
mean transverse slopes of the two x-faces.  Every fine cell then has the
divergence of its parent.
Cell data (conservative interpolation): each conserved component takes a
minmod-limited linear profile in the coarse cell, u_child = u + (s_x sx +
s_y sy + s_z sz)/4 with s the minmod of the two one-sided differences along
an axis and sx, sy, sz = -1 / +1 for the lower / upper child, so the eight
children average to the parent; the energy also moves the magnetic energy
to where the fine field has it, + (|b_child|^2 - <|b|^2>)/2 (b the fine
cell-centred field, <.> the mean over the children), which keeps the mean.
Where a child would get a non-positive density or pressure, the parent's
children take the parent's density and momentum instead, with energies
e_parent + (|b_child|^2 - <|b|^2>)/2 (a common pressure) or, where that
pressure would not be positive either, the parent's pressure (e = p_parent
/ (gamma - 1) + parent's kinetic energy + |b_child|^2 / 2, not
conservative).
Restriction: a coarse cell takes the mean of its eight children.
"""
from __future__ import annotations

import numpy as np


def mc(a, b):
    """Monotonized-central limited slope from two one-sided differences."""
    if a * b <= 0.0:
        return 0.0
    m = min(2.0 * abs(a), 2.0 * abs(b), 0.5 * abs(a + b))
    return m if a > 0 else -m


def minmod(a, b):
    """Minmod of two one-sided differences."""
    if a * b <= 0.0:
        return 0.0
    return a if abs(a) < abs(b) else b


def children_cells(Uc, Bc, i, j, k, b2, gamma):
    """Conserved data of the eight children (q = x + 2 y + 4 z) of coarse
    cell (i, j, k) given the children's |b|^2 (list of 8), as described in the
    module docstring."""
    nz, ny, nx = Uc.shape[1:]
    u0 = Uc[:, k, j, i]
    sl = np.zeros((5, 3))
    for m in range(5):
        for d, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            up = Uc[m, (k + dk) % nz, (j + dj) % ny, (i + di) % nx]
            dn = Uc[m, (k - dk) % nz, (j - dj) % ny, (i - di) % nx]
            sl[m, d] = minmod(u0[m] - dn, up - u0[m])
    mean_b2 = sum(b2) / 8.0
    kids, ok = [], True
    for q in range(8):
        sx, sy, sz = [1.0 if (q >> d) & 1 else -1.0 for d in range(3)]
        u = np.array([u0[m] + 0.25 * (sl[m, 0] * sx + sl[m, 1] * sy + sl[m, 2] * sz) for m in range(5)])
        u[4] = u[4] + 0.5 * (b2[q] - mean_b2)
        if not u[0] > 0.0:
            ok = False
        else:
            p = (gamma - 1) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0] - 0.5 * b2[q])
            ok = ok and p > 0.0
        kids.append(u)
    if ok:
        return kids
    bc = [0.5 * (Bc[0, k, j, i] + Bc[0, k, j, (i + 1) % nx]),
          0.5 * (Bc[1, k, j, i] + Bc[1, k, (j + 1) % ny, i]),
          0.5 * (Bc[2, k, j, i] + Bc[2, (k + 1) % nz, j, i])]
    d = u0[0]
    m = u0[1:4]
    ek = 0.5 * float(m @ m) / d
    b2c = sum(x * x for x in bc)
    p = (gamma - 1) * (u0[4] - ek - 0.5 * b2c)
    conservative = p - (gamma - 1) * 0.5 * (mean_b2 - b2c) > 0.0
    kids = []
    for q in range(8):
        e = u0[4] + 0.5 * (b2[q] - mean_b2) if conservative else p / (gamma - 1) + ek + 0.5 * b2[q]
        kids.append(np.array([d, m[0], m[1], m[2], e]))
    return kids


def face_slope(Bc, a, ti, c):
    """Limited transverse slope of the coarse a-face of cell c = (i, j, k)
    along the axis (a+1)%3 (ti = 0) or (a+2)%3 (ti = 1), periodic."""
    nz, ny, nx = Bc.shape[1:]
    n = (nx, ny, nz)
    t = (a + 1 + ti) % 3
    i, j, k = c
    up, dn = [i, j, k], [i, j, k]
    up[t] = (up[t] + 1) % n[t]
    dn[t] = (dn[t] - 1) % n[t]
    v = Bc[a, k, j, i]
    return mc(Bc[a, up[2], up[1], up[0]] - v, v - Bc[a, dn[2], dn[1], dn[0]])


def face_slopes(Bc):
    """Limited transverse slopes S[a][t] (t = 0, 1 for the axes (a+1)%3,
    (a+2)%3) of every coarse a-face, shape (3, 2, nz, ny, nx)."""
    S = np.zeros((3, 2) + Bc.shape[1:])
    nz, ny, nx = Bc.shape[1:]
    for a in range(3):
        for ti in range(2):
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        S[a, ti, k, j, i] = face_slope(Bc, a, ti, (i, j, k))
    return S


def prolong(Uc, Bc, gamma=5.0 / 3.0, cells=None):
    """Fine level (2 nc) from the coarse level.  cells: None (every coarse
    cell) or an iterable of coarse cells (i, j, k); then only their children
    and the children's faces are filled (NaN elsewhere)."""
    nzc, nyc, nxc = Uc.shape[1:]
    nc = (nxc, nyc, nzc)
    Bf = np.empty((3,) + tuple(2 * x for x in Uc.shape[1:]))
    Uf = np.empty((5,) + Bf.shape[1:])
    if cells is None:
        todo = [(i, j, k) for k in range(nzc) for j in range(nyc) for i in range(nxc)]
    else:
        Bf.fill(np.nan)
        Uf.fill(np.nan)
        todo = sorted({(i % nxc, j % nyc, k % nzc) for (i, j, k) in cells}, key=lambda c: (c[2], c[1], c[0]))
    # slopes of every face (whole level) or of the faces the subset reads
    S = face_slopes(Bc) if cells is None else {}

    def face(a, c):                      # coarse a-face value and slopes at cell c (lower face), periodic
        i, j, k = c[0] % nc[0], c[1] % nc[1], c[2] % nc[2]
        if cells is None:
            return Bc[a, k, j, i], S[a, 0, k, j, i], S[a, 1, k, j, i]
        key = (a, i, j, k)
        if key not in S:
            S[key] = (face_slope(Bc, a, 0, (i, j, k)), face_slope(Bc, a, 1, (i, j, k)))
        return (Bc[a, k, j, i],) + S[key]

    def faces_of(c):                     # the fine faces on c's lower faces and on its mid-planes
        i, j, k = c
        for a in range(3):
            b, cc = (a + 1) % 3, (a + 2) % 3
            lo = face(a, c)
            up_c = list(c)
            up_c[a] += 1
            hi = face(a, up_c)
            # fine faces on the lower coarse a-face: profile at (+-1/4, +-1/4)
            for q in range(4):
                ob, oc = (q & 1), (q >> 1)
                f = [2 * i, 2 * j, 2 * k]
                f[b] += ob
                f[cc] += oc
                Bf[a, f[2], f[1], f[0]] = lo[0] + lo[1] * (ob - 0.5) * 0.5 + lo[2] * (oc - 0.5) * 0.5
            # interior fine faces on the mid-plane of the cell
            # slope of the b-face component along a: it is the slope index of axis a
            # among (b+1)%3, (b+2)%3 of the b-faces
            def slope_along(comp, cell, axis):
                v = face(comp, cell)
                t1 = (comp + 1) % 3
                return v[1] if axis == t1 else v[2]
            bl, bh = list(c), list(c)
            bh[b] += 1
            cl, ch = list(c), list(c)
            ch[cc] += 1
            b_xy = slope_along(b, bh, a) - slope_along(b, bl, a)
            c_xz = slope_along(cc, ch, a) - slope_along(cc, cl, a)
            a_xx = -0.5 * (b_xy + c_xz)
            a0 = 0.5 * (lo[0] + hi[0]) - 0.25 * a_xx
            a_b = 0.5 * (lo[1] + hi[1])
            a_c = 0.5 * (lo[2] + hi[2])
            for q in range(4):
                ob, oc = (q & 1), (q >> 1)
                f = [2 * i, 2 * j, 2 * k]
                f[a] += 1
                f[b] += ob
                f[cc] += oc
                Bf[a, f[2], f[1], f[0]] = a0 + a_b * (ob - 0.5) * 0.5 + a_c * (oc - 0.5) * 0.5

    # the children's upper faces are the next coarse cells' lower faces
    face_cells = set(todo)
    if cells is not None:
        for (i, j, k) in todo:
            for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                face_cells.add(((i + d[0]) % nxc, (j + d[1]) % nyc, (k + d[2]) % nzc))
    for c in sorted(face_cells, key=lambda c: (c[2], c[1], c[0])):
        faces_of(c)
    nz, ny, nx = Bf.shape[1:]
    for (i, j, k) in todo:
        kids = [(2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2)) for q in range(8)]
        b2 = []
        for (I, J, K) in kids:
            bf = [0.5 * (Bf[0, K, J, I] + Bf[0, K, J, (I + 1) % nx]),
                  0.5 * (Bf[1, K, J, I] + Bf[1, K, (J + 1) % ny, I]),
                  0.5 * (Bf[2, K, J, I] + Bf[2, (K + 1) % nz, J, I])]
            b2.append(sum(x * x for x in bf))
        for (I, J, K), u in zip(kids, children_cells(Uc, Bc, i, j, k, b2, gamma)):
            Uf[:, K, J, I] = u
    return Uf, Bf


def restrict(Uf):
    nz, ny, nx = Uf.shape[1:]
    Uc = np.zeros((5, nz // 2, ny // 2, nx // 2))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                Uc += Uf[:, dz::2, dy::2, dx::2]
    return Uc / 8.0


# ---------------------------------------------------------------- regridding
# Refinement / derefinement operation of Sec. 3.3: fine groups are created
# where a refinement criterion holds on the coarse level and removed where
# it no longer does; a created group takes its data from the coarse level by
# the prolongation above, except that where it touches a fine group that
# already exists, the existing fine faces on the shared coarse face are kept.
# Those four faces need not follow a linear profile: beyond the linear part
# (mean m and slopes S_b, S_c, which the interior reconstruction uses) they
# carry a twist d s_b s_c (s = -1 / +1 for the first / second child along an
# axis).  The twist changes the divergence of the four children behind the
# face by -+d; it is given back to them through the mid-plane faces of the
# next axis b = (a+1)%3 in that layer of children: the b-mid-plane face of
# the children at position g along c = (a+2)%3 gets -d s_g (lower a-face) or
# +d s_g (upper a-face).  Then every created fine cell has its parent's
# divergence, as in the plain prolongation.

def refine_indicator_exceeds(Bc, thr):
    """Cells where |curl B| dx / |B| > thr, decided as
    (jx^2 + jy^2 + jz^2) > thr^2 (bx^2 + by^2 + bz^2) with j = dx curl B from
    central differences of the cell-centred field b (periodic)."""
    bx = 0.5 * (Bc[0] + np.roll(Bc[0], -1, axis=2))
    by = 0.5 * (Bc[1] + np.roll(Bc[1], -1, axis=1))
    bz = 0.5 * (Bc[2] + np.roll(Bc[2], -1, axis=0))

    def d(f, axis):          # (f(+1) - f(-1)) / 2 along array axis
        return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))

    jx = d(bz, 1) - d(by, 0)
    jy = d(bx, 0) - d(bz, 2)
    jz = d(by, 2) - d(bx, 1)
    return (jx * jx + jy * jy + jz * jz) > thr * thr * (bx * bx + by * by + bz * bz)


def refine_groups(Bc, thr, fine_edge=16, buffer=1, coarse_groups=None, coarse_edge=16):
    """Origins (fine cells) of the fine groups to hold after regridding, in
    increasing (z, y, x) group order: a candidate group (a block of
    fine_edge/2 coarse cells per axis) is kept when the criterion holds in a
    coarse cell of the block widened by `buffer` cells (periodic), and, when
    the coarse level has a group list, when its block lies in a listed coarse
    group (proper nesting)."""
    hit = refine_indicator_exceeds(Bc, thr)
    nz, ny, nx = hit.shape
    e = fine_edge // 2
    listed = None
    if coarse_groups is not None:
        listed = {tuple(int(v) // coarse_edge for v in g) for g in coarse_groups}
    out = []
    for gk in range(nz // e):
        for gj in range(ny // e):
            for gi in range(nx // e):
                if listed is not None and ((gi * e) // coarse_edge, (gj * e) // coarse_edge,
                                           (gk * e) // coarse_edge) not in listed:
                    continue
                ks = [(gk * e + t) % nz for t in range(-buffer, e + buffer)]
                js = [(gj * e + t) % ny for t in range(-buffer, e + buffer)]
                is_ = [(gi * e + t) % nx for t in range(-buffer, e + buffer)]
                if hit[np.ix_(ks, js, is_)].any():
                    out.append((gi * fine_edge, gj * fine_edge, gk * fine_edge))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def _in_groups(groups, edge, shape):
    """Boolean map of the fine cells inside the listed groups."""
    m = np.zeros(shape, bool)
    for (i, j, k) in groups:
        m[k:k + edge, j:j + edge, i:i + edge] = True
    return m


def prolong_new_groups(Uc, Bc, Uf, Bf, new_groups, old_groups, edge=16, gamma=5.0 / 3.0):
    """Fine level after regridding: groups of new_groups not in old_groups
    are filled from the coarse level (cells, their lower faces, and their
    upper boundary faces), faces shared with an old group are kept; every
    other fine value is left as it is.  Returns new arrays."""
    Uf, Bf = Uf.copy(), Bf.copy()
    nzc, nyc, nxc = Uc.shape[1:]
    nc = (nxc, nyc, nzc)
    nf = (2 * nxc, 2 * nyc, 2 * nzc)
    S = face_slopes(Bc)
    old_map = _in_groups(old_groups, edge, Bf.shape[1:])
    old_set = {tuple(int(v) for v in g) for g in old_groups}

    def old_at(I, J, K):
        return old_map[K % nf[2], J % nf[1], I % nf[0]]

    def sgn(x):
        return 1.0 if x else -1.0

    for g in new_groups:
        if tuple(int(v) for v in g) in old_set:
            continue
        o = [int(v) // 2 for v in g]
        for ck in range(o[2], o[2] + edge // 2):
            for cj in range(o[1], o[1] + edge // 2):
                for ci in range(o[0], o[0] + edge // 2):
                    c = (ci, cj, ck)
                    # per face (a, s): mean, slopes along (a+1)%3 and (a+2)%3, twist, and fixed values
                    m = np.zeros((3, 2))
                    sl = np.zeros((3, 2, 2))
                    tw = np.zeros((3, 2))
                    fixed = [[None, None] for _ in range(3)]
                    for a in range(3):
                        b, cc = (a + 1) % 3, (a + 2) % 3
                        for s in range(2):
                            cell = list(c)
                            cell[a] += s
                            beyond = [2 * c[0], 2 * c[1], 2 * c[2]]   # fine cell across the face
                            beyond[a] = 2 * c[a] - 1 if s == 0 else 2 * c[a] + 2
                            if old_at(*beyond):
                                f = []
                                for q in range(4):
                                    F = [2 * c[0], 2 * c[1], 2 * c[2]]
                                    F[a] = 2 * c[a] + 2 * s
                                    F[b] += q & 1
                                    F[cc] += q >> 1
                                    f.append(Bf[a, F[2] % nf[2], F[1] % nf[1], F[0] % nf[0]])
                                fixed[a][s] = f
                                m[a, s] = 0.25 * ((f[0] + f[1]) + (f[2] + f[3]))
                                sl[a, s, 0] = (f[1] - f[0]) + (f[3] - f[2])
                                sl[a, s, 1] = (f[2] - f[0]) + (f[3] - f[1])
                                tw[a, s] = 0.25 * ((f[0] - f[1]) + (f[3] - f[2]))
                            else:
                                i, j, k = cell[0] % nc[0], cell[1] % nc[1], cell[2] % nc[2]
                                m[a, s] = Bc[a, k, j, i]
                                sl[a, s, 0] = S[a, 0, k, j, i]
                                sl[a, s, 1] = S[a, 1, k, j, i]
                    # fine faces fine[a][p][q]: plane p (0 lower, 1 mid, 2 upper) of component a
                    fine = np.zeros((3, 3, 4))
                    for a in range(3):
                        b, cc = (a + 1) % 3, (a + 2) % 3
                        for q in range(4):
                            u, v = q & 1, q >> 1
                            tb, tc = 0.25 * sgn(u), 0.25 * sgn(v)
                            for s in range(2):
                                if fixed[a][s] is not None:
                                    fine[a, 2 * s, q] = fixed[a][s][q]
                                else:
                                    fine[a, 2 * s, q] = m[a, s] + sl[a, s, 0] * tb + sl[a, s, 1] * tc
                            # interior: the quadratic of the coarse cell (mid-plane of a)
                            b_xy = sl[b, 1, 1] - sl[b, 0, 1]       # slope of B_b along a (a = (b+2)%3)
                            c_xz = sl[cc, 1, 0] - sl[cc, 0, 0]     # slope of B_c along a (a = (c+1)%3)
                            a_xx = -0.5 * (b_xy + c_xz)
                            a0 = 0.5 * (m[a, 0] + m[a, 1]) - 0.25 * a_xx
                            a_b = 0.5 * (sl[a, 0, 0] + sl[a, 1, 0])
                            a_c = 0.5 * (sl[a, 0, 1] + sl[a, 1, 1])
                            fine[a, 1, q] = a0 + a_b * tb + a_c * tc
                    # give each twist back through the b-mid-plane faces of its layer
                    for a in range(3):
                        b = (a + 1) % 3
                        for s in range(2):
                            if tw[a, s] == 0.0:
                                continue
                            for gpos in range(2):     # position along (a+2)%3 = the first in-face axis of b
                                q = gpos + 2 * s       # b's second in-face axis is a: layer s
                                fine[b, 1, q] += (1.0 if s else -1.0) * tw[a, s] * sgn(gpos)
                    # children
                    kids = []
                    for q in range(8):
                        x, y, z = q & 1, (q >> 1) & 1, q >> 2
                        pos = (x, y, z)
                        bcell = []
                        for a in range(3):
                            b, cc = (a + 1) % 3, (a + 2) % 3
                            t = pos[b] + 2 * pos[cc]
                            bcell.append(0.5 * (fine[a, pos[a], t] + fine[a, pos[a] + 1, t]))
                        kids.append((pos, sum(w * w for w in bcell)))
                    cells = children_cells(Uc, Bc, ci % nc[0], cj % nc[1], ck % nc[2], [k2 for _, k2 in kids], gamma)
                    for (pos, _), u in zip(kids, cells):
                        I, J, K = 2 * ci + pos[0], 2 * cj + pos[1], 2 * ck + pos[2]
                        Uf[:, K, J, I] = u
                        for a in range(3):
                            b, cc = (a + 1) % 3, (a + 2) % 3
                            t = pos[b] + 2 * pos[cc]
                            if pos[a] == 0 and fixed[a][0] is not None:
                                continue
                            Bf[a, K, J, I] = fine[a, pos[a], t]
                    # upper boundary faces of the parent unless they belong to an old group
                    for a in range(3):
                        b, cc = (a + 1) % 3, (a + 2) % 3
                        if fixed[a][1] is not None:
                            continue
                        for q in range(4):
                            F = [2 * ci, 2 * cj, 2 * ck]
                            F[a] += 2
                            F[b] += q & 1
                            F[cc] += q >> 1
                            Bf[a, F[2] % nf[2], F[1] % nf[1], F[0] % nf[0]] = fine[a, 2, q]
    return Uf, Bf


# ---------------------------------------------------------------- two levels, one shared step
# A root level and one refined level whose listed patch groups (cubes of
# `edge` fine cells, origins in fine cells) are updated, advanced together
# by one time step (Sec. 3.3: the refined level's ghost zones are filled from
# the coarse level by interpolation, both levels are updated, then the
# correction operation puts the fine fluxes and EMFs on the coarse-fine
# interface and the restriction replaces refined coarse data by fine means).
# Fine cells that are neither listed nor ghosts are never read; the driver
# keeps them at NaN so that a dependence on them would show.

def listed_mask(groups, edge, shape):
    """Fine cells inside the listed groups."""
    m = np.zeros(shape, bool)
    for (i, j, k) in np.asarray(groups).reshape(-1, 3):
        m[k:k + edge, j:j + edge, i:i + edge] = True
    return m


def ghost_box_mask(groups, edge, halo, shape):
    """Fine cells from `halo` below to `halo` + 1 above each listed group
    (periodic): every cell whose state or lower faces a group's update reads
    (the extra layer holds the last ghost's upper faces)."""
    nz, ny, nx = shape
    m = np.zeros(shape, bool)
    for (i, j, k) in np.asarray(groups).reshape(-1, 3):
        ks = np.arange(k - halo, k + edge + halo + 1) % nz
        js = np.arange(j - halo, j + edge + halo + 1) % ny
        is_ = np.arange(i - halo, i + edge + halo + 1) % nx
        m[np.ix_(ks, js, is_)] = True
    return m


def _face_of_listed(listed, a):
    """Lower a-faces of the fine level that touch a listed cell."""
    return listed | np.roll(listed, 1, axis=2 - a)


def initial_fine(Uc, Bc, groups, edge=16, gamma=5.0 / 3.0, halo=0):
    """The refined level at the start: listed cells and their faces (with
    halo > 0 also the cells and faces of the ghost boxes, `halo` cells
    around each group) from the prolongation of their parents, NaN
    elsewhere.  A level that has refined levels of its own needs the halo:
    the prolongation of its cells reads their neighbours."""
    shape = tuple(2 * n for n in Uc.shape[1:])
    listed = listed_mask(groups, edge, shape)
    fill = listed | ghost_box_mask(groups, edge, halo, shape) if halo else listed
    parents = {(I // 2, J // 2, K // 2) for K, J, I in zip(*np.nonzero(fill))}
    Up, Bp = prolong(Uc, Bc, gamma, cells=parents)
    Uf = np.full((5,) + shape, np.nan)
    Bf = np.full((3,) + shape, np.nan)
    Uf[:, fill] = Up[:, fill]
    for a in range(3):
        m = _face_of_listed(fill, a)
        Bf[a][m] = Bp[a][m]
    return Uf, Bf


def refill_ghosts(Uc, Bc, Uf, Bf, groups, edge=16, halo=4, gamma=5.0 / 3.0):
    """Ghost cells of the listed groups (not listed themselves) take the
    prolongation of the coarse level, cell data and the faces that touch no
    listed cell; listed cells and every face of a listed cell keep theirs."""
    listed = listed_mask(groups, edge, Uf.shape[1:])
    ghost = ghost_box_mask(groups, edge, halo, Uf.shape[1:]) & ~listed
    parents = {(I // 2, J // 2, K // 2) for K, J, I in zip(*np.nonzero(ghost))}
    Up, Bp = prolong(Uc, Bc, gamma, cells=parents)
    Uf, Bf = Uf.copy(), Bf.copy()
    Uf[:, ghost] = Up[:, ghost]
    for a in range(3):
        m = ghost & ~np.roll(listed, 1, axis=2 - a)
        Bf[a][m] = Bp[a][m]
    return Uf, Bf


def cfl_dt_listed(U, B, dx, mask, gamma=5.0 / 3.0, courant=0.5):
    """The oracle's CFL step over the masked cells only: the other cells are
    put at rest with density 1e30 and pressure 1e-6 (1 + |B|^2) (a signal
    speed of order 1e-15 |B|), the face field (and so each masked cell's
    centred field) unchanged."""
    from . import cfl_dt, cons_to_prim
    Bn = np.nan_to_num(B, nan=0.0)
    W = cons_to_prim(np.nan_to_num(U, nan=1.0), Bn, gamma)
    b2 = W[5] ** 2 + W[6] ** 2 + W[7] ** 2
    Us = np.array(U)
    out = ~mask
    Us[0][out] = 1e30
    Us[1:4][:, out] = 0.0
    Us[4][out] = 1e-6 * (1.0 + b2[out]) / (gamma - 1.0) + 0.5 * b2[out]
    return cfl_dt(Us, Bn, dx, gamma, courant)


def refined_coarse(groups, edge, shape_c):
    """Coarse cells under the listed fine groups."""
    m = np.zeros(shape_c, bool)
    h = edge // 2
    for (i, j, k) in np.asarray(groups).reshape(-1, 3):
        m[k // 2:k // 2 + h, j // 2:j // 2 + h, i // 2:i // 2 + h] = True
    return m


def face_mean(Ff, a):
    """Mean of the four fine lower a-faces on each coarse lower a-face (Ff
    [..., nzf, nyf, nxf], result [..., nzc, nyc, nxc])."""
    ax = Ff.ndim - 1 - a                       # array axis of direction a
    t = [Ff.ndim - 1 - b for b in range(3) if b != a]
    sl = [slice(None)] * Ff.ndim
    sl[ax] = slice(0, None, 2)
    F = Ff[tuple(sl)]
    acc = 0.0
    for p in (0, 1):
        for q in (0, 1):
            s2 = [slice(None)] * Ff.ndim
            s2[t[0]] = slice(p, None, 2)
            s2[t[1]] = slice(q, None, 2)
            acc = acc + F[tuple(s2)]
    return 0.25 * acc


def edge_mean(Ef, a):
    """Mean of the two fine a-edges on each coarse a-edge (the edge along a
    at the cell's lower corner in the two other directions)."""
    ax = Ef.ndim - 1 - a
    sl = [slice(None)] * Ef.ndim
    for b in range(3):
        if b != a:
            sl[Ef.ndim - 1 - b] = slice(0, None, 2)
    E = Ef[tuple(sl)]
    s0 = [slice(None)] * Ef.ndim
    s1 = [slice(None)] * Ef.ndim
    s0[ax] = slice(0, None, 2)
    s1[ax] = slice(1, None, 2)
    return 0.5 * (E[tuple(s0)] + E[tuple(s1)])


def correct_and_restrict(Uc, Bc, Fc, Ec, Uf, Bf, Ff, Ef, refined, dt, dxc, correct=True):
    """The correction operation and the restriction after a shared step dt.

    Uc, Bc: the coarse level after its own update with fluxes Fc [3, 5, ...]
    and edge EMFs Ec [3, ...]; Uf, Bf, Ff, Ef the same of the refined level;
    refined: the coarse cells under listed fine groups.
      - an unrefined coarse cell sharing a face with a refined one takes,
        through that face, the mean of the four fine fluxes instead of its own;
      - on coarse edges of the refined region's boundary (some, not all, of
        the four cells around the edge refined) the EMF difference (mean of
        the two fine EMFs minus the coarse one) updates, by the CT formula,
        the coarse faces whose two cells are both unrefined;
      - refined coarse cells take the mean of their eight children, and every
        coarse face with a refined cell on either side the mean of its four
        fine faces.
    correct=False: the restriction alone (no correction)."""
    r = dt / dxc
    Uc, Bc = Uc.copy(), Bc.copy()
    out = ~refined
    for a in range(3 if correct else 0):
        ax = 2 - a
        dF = face_mean(Ff[a], a) - Fc[a]                 # [5, ...] on each coarse lower a-face
        m_lo = out & np.roll(refined, 1, axis=ax)         # refined neighbour below: own lower face
        Uc[:, m_lo] += r * dF[:, m_lo]
        m_hi = out & np.roll(refined, -1, axis=ax)        # refined neighbour above: its lower face
        dF_hi = np.roll(dF, -1, axis=ax + 1)
        Uc[:, m_hi] -= r * dF_hi[:, m_hi]
    dE = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        r00 = refined
        r10 = np.roll(refined, 1, axis=2 - b)
        r01 = np.roll(refined, 1, axis=2 - c)
        r11 = np.roll(r10, 1, axis=2 - c)
        boundary = (r00 | r10 | r01 | r11) & ~(r00 & r10 & r01 & r11)
        dE.append(np.where(boundary & correct, edge_mean(Ef[a], a) - Ec[a], 0.0))
    dEx, dEy, dEz = dE

    def up(f, ax):                       # the value one cell up along an array axis
        return np.roll(f, -1, axis=ax)
    dB = [-r * (up(dEz, 1) - dEz) + r * (up(dEy, 0) - dEy),
          -r * (up(dEx, 0) - dEx) + r * (up(dEz, 2) - dEz),
          -r * (up(dEy, 2) - dEy) + r * (up(dEx, 1) - dEx)]
    for a in range(3):
        both_out = out & np.roll(out, 1, axis=2 - a)
        Bc[a][both_out] += dB[a][both_out]
    Ur = restrict(np.nan_to_num(Uf))
    Uc[:, refined] = Ur[:, refined]
    for a in range(3):
        touched = refined | np.roll(refined, 1, axis=2 - a)
        Bm = face_mean(np.nan_to_num(Bf[a]), a)
        Bc[a][touched] = Bm[touched]
    return Uc, Bc


def replace_stored(Fc, Ec, Ff, Ef, refined):
    """After a correction the coarse level's stored fluxes and EMFs on the
    faces and edges of refined cells become the fine means, so that the next
    coarser level is corrected with the finest values (in place)."""
    for a in range(3):
        m = refined | np.roll(refined, 1, axis=2 - a)
        Fm = face_mean(Ff[a], a)
        Fc[a][:, m] = Fm[:, m]
        b, c = (a + 1) % 3, (a + 2) % 3
        r10 = np.roll(refined, 1, axis=2 - b)
        e = refined | r10 | np.roll(refined, 1, axis=2 - c) | np.roll(r10, 1, axis=2 - c)
        Em = edge_mean(Ef[a], a)
        Ec[a][e] = Em[e]


def hierarchy_step(levels, groups, dx0, edge=16, halo=4, scheme=1, recon=1, riemann=2, gamma=5.0 / 3.0,
                   courant=0.5, dt_max=np.inf, correct=True, subcycle=False):
    """One root step of a hierarchy: levels = [(U0, B0), (U1, B1), ...], the
    dense arrays of level l (cell size dx0 / 2^l; the root is updated whole),
    groups = [None, g1, g2, ...] the listed groups of each refined level
    (origins in its cells, each inside a listed group of its parent).
    scheme / recon / riemann: the oracle's codes (default CTU, PPM, HLLD).

    Shared step (subcycle=False): dt is the smallest CFL step of the levels
    (a refined one over its listed cells), at most dt_max; the ghosts of
    every refined level are refilled from its parent, coarse to fine, all
    levels are updated by dt, then, fine to coarse, each level corrects its
    parent, is restricted onto it, and the parent's stored fluxes and EMFs
    on the faces and edges of refined cells become its means.
    Sub-cycled (subcycle=True; the paper's level update: a level first,
    then its finer level evolved to the same time, then the correction;
    refinement ratio 2 in time): dt = min over l of 2^l times level l's
    CFL step, at most dt_max, and level l's step is dt / 2^l.  A level
    keeps its state before its update; its child takes two steps, the ghosts
    of sub-step s refilled from the parent at time fraction s / 2 (linear
    between the parent's states before and after its update); the
    correction uses the mean of the two sub-steps' fluxes and EMFs (as they
    stand after the child's own correction by its children).
    Returns (levels after the step, dt)."""
    from . import cfl_dt, step
    nl = len(levels)
    U = [np.array(u) for u, _ in levels]
    B = [np.array(b) for _, b in levels]
    dxs = [dx0 / 2 ** l for l in range(nl)]
    listed = [None] + [listed_mask(groups[l], edge, U[l].shape[1:]) for l in range(1, nl)]
    refined = [refined_coarse(groups[l + 1], edge, U[l].shape[1:]) for l in range(nl - 1)]
    kw = dict(scheme=scheme, recon=recon, riemann=riemann, gamma=gamma, return_fluxes=True)
    cfl = [cfl_dt(U[0], B[0], dxs[0], gamma, courant)] + \
          [cfl_dt_listed(U[l], B[l], dxs[l], listed[l], gamma, courant) for l in range(1, nl)]
    dt = min(min((2.0 ** l if subcycle else 1.0) * cfl[l] for l in range(nl)), dt_max)

    def update(l, tau):
        Un, Bn, F, E = step(U[l], B[l], tau, dxs[l], **kw)
        if l == 0:
            U[0], B[0] = Un, Bn
        else:
            U[l][:, listed[l]] = Un[:, listed[l]]
            for a in range(3):
                m = _face_of_listed(listed[l], a)
                B[l][a][m] = Bn[a][m]
        return F, E

    def refill(l, Up, Bp):
        U[l], B[l] = refill_ghosts(Up, Bp, U[l], B[l], groups[l], edge, halo, gamma)

    def close(l, F, E, Ff, Ef, tau):
        # level l + 1 corrects level l (own fluxes F, E; the child's Ff, Ef)
        U[l], B[l] = correct_and_restrict(U[l], B[l], F, E, U[l + 1], B[l + 1], Ff, Ef, refined[l], tau, dxs[l],
                                          correct)
        replace_stored(F, E, Ff, Ef, refined[l])

    if not subcycle:
        for l in range(1, nl):
            refill(l, U[l - 1], B[l - 1])
        FE = [update(l, dt) for l in range(nl)]
        for l in range(nl - 2, -1, -1):
            close(l, FE[l][0], FE[l][1], FE[l + 1][0], FE[l + 1][1], dt)
        return list(zip(U, B)), dt

    def advance(l, tau):
        Uo, Bo = U[l].copy(), B[l].copy()
        F, E = update(l, tau)
        if l == nl - 1:
            return F, E
        Fm, Em = 0.0, 0.0
        for alpha in (0.0, 0.5):
            Ua = Uo + alpha * (U[l] - Uo) if alpha else Uo
            Ba = Bo + alpha * (B[l] - Bo) if alpha else Bo
            refill(l + 1, Ua, Ba)
            Fc, Ec = advance(l + 1, 0.5 * tau)
            Fm = Fm + 0.5 * Fc
            Em = Em + 0.5 * Ec
        close(l, F, E, Fm, Em, tau)
        return F, E

    advance(0, dt)
    return list(zip(U, B)), dt


def two_level_step(Uc, Bc, Uf, Bf, groups, dxc, edge=16, halo=4, scheme=1, recon=1, riemann=2,
                   gamma=5.0 / 3.0, courant=0.5, dt_max=np.inf, correct=True, subcycle=False):
    """hierarchy_step of a root (Uc, Bc, cell size dxc) and one refined
    level (Uf, Bf) with the listed groups `groups`; returns (Uc, Bc, Uf, Bf,
    dt)."""
    ((Uc, Bc), (Uf, Bf)), dt = hierarchy_step([(Uc, Bc), (Uf, Bf)], [None, groups], dxc, edge, halo, scheme, recon,
                                              riemann, gamma, courant, dt_max, correct, subcycle)
    return Uc, Bc, Uf, Bf, dt
