// AMR support of the level update (paper Sec. 3.3): prolongation (whole
// levels, ghost halos, optionally interpolated in time), restriction, the
// correction operation across coarse-fine interfaces, time-mean registers of
// sub-cycled levels, and regridding by the refinement criterion.  Included
// after mhd_kernels.hpp, whose addressing (Work, Site, lin, wrapc, nbr,
// FOR_ITEMS) and slope limiter it uses.
#pragma once

#include "mhd_kernels.hpp"

namespace mhd {
// ------------------------------------------------------------ AMR support
// offset d of a cell from its group's origin on a periodic level of n cells,
// taken in the group box's own range [lo, lo + n) (lo = minus the box's
// ghost width): unique for every box position since levels with group
// lists are at least edge + 8 cells wide
__device__ __forceinline__ int box_offset(int d, int lo, int n) {
  const int r = (d - lo) % n;
  return (r < 0 ? r + n : r) + lo;
}

// Prolongation from a coarse level (nc) to a fine level (2 nc), paper
// Sec. 3.3 (refinement operation).  Cell data: conservative limited-linear
// interpolation of the conserved variables (child_cells).
// Face field (Balsara's divergence-free reconstruction, in 3D): a coarse
// face carries a linear profile B + S_t1 t1 + S_t2 t2 in its transverse
// coordinates (coarse-cell units, t in [-1/2, 1/2]) with MC-limited slopes
// of the same face component across its neighbouring coarse faces; fine
// faces on it take the profile at their centres (t = -+1/4).  Inside the
// coarse cell the field is the quadratic whose face profiles match the six
// coarse faces and whose divergence has no linear terms; the fine faces on
// the mid-planes take Bx(0, y, z) = a0 + ay y + az z with
// a0 = (Bx- + Bx+)/2 - axx/4, axx = -(bxy + cxz)/2 (bxy, cxz: the jumps of
// the x-slopes of By, Bz across the cell) and ay, az the mean transverse
// slopes of the two x-faces (and cyclic).  Every fine cell's divergence
// equals its parent's; the fine faces on a coarse face average to it.

// Coarse data read by the prolongation: one state, or the linear
// interpolation in time old + w (new - old) between a parent's states at the
// start and at the end of its step (the ghosts of a sub-cycled fine level).
template <typename T>
struct Coarse {
  const T* a;      // the state, or the old state
  const T* b;      // the new state (nullptr: no interpolation)
  T w;
  __device__ __forceinline__ T operator[](long long i) const { return b ? a[i] + w * (b[i] - a[i]) : a[i]; }
  __device__ __forceinline__ Coarse shift(long long o) const { return Coarse{a + o, b ? b + o : nullptr, w}; }
};

// The parent's six faces and the MC-limited slopes of each along its two
// in-face directions: everything its 36 fine faces depend on (30 loads).
template <typename T>
struct ParentFaces {
  T v[3][2];        // component A on the lower (0) and upper (1) A-face
  T s[3][2][2];     // its slope along (A + 1) % 3 (0) and (A + 2) % 3 (1)
};

template <typename T, int A>
__device__ __forceinline__ void load_face_pair(const Work& wc, const Coarse<T>& Bc, int i, int j, int k,
                                               ParentFaces<T>& P) {
  constexpr int b = (A + 1) % 3, c = (A + 2) % 3;
  const Coarse<T> Ba = Bc.shift((long long)A * wc.N);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    int C[3] = {i, j, k};
    C[A] += s;
    auto at = [&](int d, int o) {
      int D[3] = {C[0], C[1], C[2]};
      D[d] += o;
      return Ba[lin(wc, wrapc(D[0], wc.nx), wrapc(D[1], wc.ny), wrapc(D[2], wc.nz))];
    };
    const T v = at(b, 0);
    P.v[A][s] = v;
    P.s[A][s][0] = mc_slope(at(b, -1), v, at(b, 1));
    P.s[A][s][1] = mc_slope(at(c, -1), v, at(c, 1));
  }
}

// Fine face of component A on plane p of the parent (0: its lower A-face,
// 1: the mid-plane, 2: its upper A-face) at transverse position q = u + 2 v
// (u along (A + 1) % 3, v along (A + 2) % 3).
template <typename T, int A>
__device__ __forceinline__ T fine_face(const ParentFaces<T>& P, int p, int q) {
  constexpr int b = (A + 1) % 3, c = (A + 2) % 3;
  const T tb = (q & 1) ? T(0.25) : T(-0.25);
  const T tc = (q >> 1) ? T(0.25) : T(-0.25);
  if (p != 1) {
    const int s = p >> 1;
    return P.v[A][s] + P.s[A][s][0] * tb + P.s[A][s][1] * tc;
  }
  const T ab = T(0.5) * (P.s[A][0][0] + P.s[A][1][0]);
  const T ac = T(0.5) * (P.s[A][0][1] + P.s[A][1][1]);
  // jumps across the parent of the A-slopes of the two transverse components
  const T bxy = P.s[b][1][1] - P.s[b][0][1];     // A = (b + 2) % 3
  const T cxz = P.s[c][1][0] - P.s[c][0][0];     // A = (c + 1) % 3
  const T axx = T(-0.5) * (bxy + cxz);
  const T a0 = T(0.5) * (P.v[A][0] + P.v[A][1]) - T(0.25) * axx;
  return a0 + ab * tb + ac * tc;
}

// Conserved data of the eight children q = x + 2 y + 4 z of coarse cell
// (i, j, k), given the children's |b|^2 (conservative interpolation): each
// component takes the minmod-limited linear profile of the cell, u + (s_x sx
// + s_y sy + s_z sz)/4 with sx, sy, sz = -1 / +1 for the lower / upper child,
// so the children average to the parent; the energy also moves magnetic
// energy to where the fine field has it, + (|b_q|^2 - <|b|^2>)/2.  If a child
// would get a non-positive density or pressure, the children take the
// parent's density and momentum and energies e + (|b_q|^2 - <|b|^2>)/2 (one
// common pressure) or, where that pressure would not be positive, the
// parent's pressure.  (cbx, cby, cbz): the parent's cell-centred field.
template <typename T>
__device__ __forceinline__ void child_cells(const Work& wc, const Coarse<T>& Uc, int i, int j, int k, T cbx, T cby,
                                            T cbz, const T b2[8], T mean_b2, T gam, T u[8][5]) {
  const long long pc = lin(wc, i, j, k);
  const long long pu[3] = {lin(wc, wrapc(i + 1, wc.nx), j, k), lin(wc, i, wrapc(j + 1, wc.ny), k),
                           lin(wc, i, j, wrapc(k + 1, wc.nz))};
  const long long pd[3] = {lin(wc, wrapc(i - 1, wc.nx), j, k), lin(wc, i, wrapc(j - 1, wc.ny), k),
                           lin(wc, i, j, wrapc(k - 1, wc.nz))};
  T u0[5], sl[5][3];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    u0[m] = Uc[m * wc.N + pc];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      sl[m][d] = minmod(u0[m] - Uc[m * wc.N + pd[d]], Uc[m * wc.N + pu[d]] - u0[m]);
  }
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const T sx = (q & 1) ? T(1) : T(-1), sy = ((q >> 1) & 1) ? T(1) : T(-1), sz = (q >> 2) ? T(1) : T(-1);
#pragma unroll
    for (int m = 0; m < 5; ++m) u[q][m] = u0[m] + T(0.25) * (sl[m][0] * sx + sl[m][1] * sy + sl[m][2] * sz);
    u[q][4] = u[q][4] + T(0.5) * (b2[q] - mean_b2);
    if (!(u[q][0] > T(0))) {
      ok = false;
    } else {
      const T p = (gam - T(1)) * (u[q][4] - T(0.5) * (u[q][1] * u[q][1] + u[q][2] * u[q][2] + u[q][3] * u[q][3]) /
                                                u[q][0] - T(0.5) * b2[q]);
      ok = ok && p > T(0);
    }
  }
  if (ok) return;
  const T b2c = cbx * cbx + cby * cby + cbz * cbz;
  const T d = u0[0], mx = u0[1], my = u0[2], mz = u0[3], e = u0[4];
  const T ek = T(0.5) * (mx * mx + my * my + mz * mz) / d;
  const T pr = (gam - T(1)) * (e - ek - T(0.5) * b2c);
  const bool conservative = pr - (gam - T(1)) * T(0.5) * (mean_b2 - b2c) > T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    u[q][0] = d;
    u[q][1] = mx;
    u[q][2] = my;
    u[q][3] = mz;
    u[q][4] = conservative ? e + T(0.5) * (b2[q] - mean_b2) : pr / (gam - T(1)) + ek + T(0.5) * b2[q];
  }
}

// The eight children of coarse cell (i, j, k): conservative cell data
// (child_cells) and their lower faces, where allowed.  cell_ok[q] /
// face_ok[q][A] say which child q = a + 2 b + 4 c (position (a, b, c) in the
// parent) and which of its lower faces may be written.
template <typename T>
__device__ __forceinline__ void prolong_parent(const Work& wc, const Work& wf, const Coarse<T>& Uc,
                                               const Coarse<T>& Bc, T* __restrict__ Uf, T* __restrict__ Bf,
                                               int i, int j, int k, const bool cell_ok[8], const bool face_ok[8][3],
                                               T gam) {
  ParentFaces<T> P;
  load_face_pair<T, 0>(wc, Bc, i, j, k, P);
  load_face_pair<T, 1>(wc, Bc, i, j, k, P);
  load_face_pair<T, 2>(wc, Bc, i, j, k, P);
  // fine faces: F[A][p][q] on plane p of component A, transverse child q
  T F[3][3][4];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      F[0][p][q] = fine_face<T, 0>(P, p, q);
      F[1][p][q] = fine_face<T, 1>(P, p, q);
      F[2][p][q] = fine_face<T, 2>(P, p, q);
    }
  T b2[8];
  T mean_b2 = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    // child (a, b, c): x-faces at transverse (y, z) = (b, c), y-faces at (z, x) = (c, a), z-faces at (x, y) = (a, b)
    const T bx = T(0.5) * (F[0][a][b + 2 * c] + F[0][a + 1][b + 2 * c]);
    const T by = T(0.5) * (F[1][b][c + 2 * a] + F[1][b + 1][c + 2 * a]);
    const T bz = T(0.5) * (F[2][c][a + 2 * b] + F[2][c + 1][a + 2 * b]);
    b2[q] = bx * bx + by * by + bz * bz;
    mean_b2 += b2[q];
  }
  mean_b2 *= T(0.125);
  T u[8][5];
  child_cells(wc, Uc, i, j, k, T(0.5) * (P.v[0][0] + P.v[0][1]), T(0.5) * (P.v[1][0] + P.v[1][1]),
              T(0.5) * (P.v[2][0] + P.v[2][1]), b2, mean_b2, gam, u);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const long long pf = lin(wf, 2 * i + a, 2 * j + b, 2 * k + c);
    if (cell_ok[q]) {
#pragma unroll
      for (int m = 0; m < 5; ++m) Uf[m * wf.N + pf] = u[q][m];
    }
    if (face_ok[q][0]) Bf[pf] = F[0][a][b + 2 * c];
    if (face_ok[q][1]) Bf[wf.N + pf] = F[1][b][c + 2 * a];
    if (face_ok[q][2]) Bf[2 * wf.N + pf] = F[2][c][a + 2 * b];
  }
}

// whole fine level from the coarse level: one coarse cell per item
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_all(Work wc, Work wf, Coarse<T> Uc,
                                                        Coarse<T> Bc, T* __restrict__ Uf,
                                                        T* __restrict__ Bf, T gam) {
  bool cell_ok[8], face_ok[8][3];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    cell_ok[q] = true;
    face_ok[q][0] = face_ok[q][1] = face_ok[q][2] = true;
  }
  FOR_ITEMS(wc, t) {
    int i, j, k;
    cell_of(wc, t, i, j, k);
    prolong_parent(wc, wf, Uc, Bc, Uf, Bf, i, j, k, cell_ok, face_ok, gam);
  }
}

// ghost halos of the listed fine groups: items are the coarse cells over the
// halo boxes; a child is written when it lies outside every listed group, a
// child's lower face when both cells of that face do.  The eight children
// of a parent share one fine group (groups have an even edge), so one
// occupancy lookup decides all of them, and three more their lower
// neighbours across the parent's lower faces.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_ghosts(Work wc, Work wf, Coarse<T> Uc,
                                                           Coarse<T> Bc, T* __restrict__ Uf,
                                                           T* __restrict__ Bf, T gam) {
  const long long per = (long long)wc.box * wc.box * wc.box;
  FOR_ITEMS(wc, t) {
    int i, j, k, a0, b0, c0;
    cell_of(wc, t, i, j, k, a0, b0, c0);
    // parents under the item's own (listed) group have listed children only
    const int lo = wc.halo, hi = wc.halo + wc.edge;
    if (a0 >= lo && a0 < hi && b0 >= lo && b0 < hi && c0 >= lo && c0 < hi) continue;
    auto listed = [&](int x, int y, int z) {
      x = wrapc(x, wf.nx); y = wrapc(y, wf.ny); z = wrapc(z, wf.nz);
      return wf.occ[((long long)(z / wf.edge) * wf.gny + y / wf.edge) * wf.gnx + x / wf.edge] != 0;
    };
    const int I0 = 2 * i, J0 = 2 * j, K0 = 2 * k;
    if (listed(I0, J0, K0)) continue;
    const bool lx = listed(I0 - 1, J0, K0), ly = listed(I0, J0 - 1, K0), lz = listed(I0, J0, K0 - 1);
    // children inside the requested fine halo box [o - halo, o + edge + halo + 1) of this item's group
    const int* o = wf.groups + 3 * (t / per);
    auto in_box = [&](int x, int y, int z) {
      const int blo = -wf.halo, bhi = wf.edge + wf.halo + 1;
      const int dx = box_offset(x - o[0], blo, wf.nx), dy = box_offset(y - o[1], blo, wf.ny),
                dz = box_offset(z - o[2], blo, wf.nz);
      return dx >= blo && dx < bhi && dy >= blo && dy < bhi && dz >= blo && dz < bhi;
    };
    bool cell_ok[8], face_ok[8][3];
    bool any = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
      const bool ghost = in_box(I0 + a, J0 + b, K0 + c);
      cell_ok[q] = ghost;
      face_ok[q][0] = ghost && (a || !lx);
      face_ok[q][1] = ghost && (b || !ly);
      face_ok[q][2] = ghost && (c || !lz);
      any = any || ghost;
    }
    if (any) prolong_parent(wc, wf, Uc, Bc, Uf, Bf, i, j, k, cell_ok, face_ok, gam);
  }
}

// Is coarse cell (ci, cj, ck) covered by the fine level?  Whole fine level:
// always; group list: when the fine group holding its first child is listed.
__device__ __forceinline__ bool refined(const Work& wf, int ci, int cj, int ck) {
  if (!wf.groups) return true;
  const int I = wrapc(2 * ci, wf.nx), J = wrapc(2 * cj, wf.ny), K = wrapc(2 * ck, wf.nz);
  return wf.occ[((long long)(K / wf.edge) * wf.gny + J / wf.edge) * wf.gnx + I / wf.edge] != 0;
}

// mean of the four fine faces of direction A on the lower A-face of coarse
// cell (i, j, k)
template <typename T, int A>
__device__ __forceinline__ T fine_face_mean(const Work& wf, const T* __restrict__ Bf, int i, int j, int k) {
  constexpr int b = (A + 1) % 3, c = (A + 2) % 3;
  T s = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int f[3] = {2 * i, 2 * j, 2 * k};
    f[b] += q & 1;
    f[c] += q >> 1;
    s += Bf[A * wf.N + lin(wf, wrapc(f[0], wf.nx), wrapc(f[1], wf.ny), wrapc(f[2], wf.nz))];
  }
  return T(0.25) * s;
}

// restriction (Sec. 3.3, correction operation): coarse cells under listed
// fine groups take the volume average of their 8 children, and the coarse
// faces of those cells (including the faces on the boundary of the refined
// region) the area average of the 4 fine faces on them
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(Work wc, Work wf, const T* __restrict__ Uf, T* __restrict__ Uc,
                                                     const T* __restrict__ Bf, T* __restrict__ Bc) {
  // work items are coarse cells of the fine groups' footprints (edge/2)^3
  FOR_ITEMS(wc, t) {
    int i, j, k;
    cell_of(wc, t, i, j, k);
    const long long pc = lin(wc, i, j, k);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      T s = T(0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int I = 2 * i + (c & 1), J = 2 * j + ((c >> 1) & 1), K = 2 * k + (c >> 2);
        s += Uf[m * wf.N + lin(wf, I, J, K)];
      }
      Uc[m * wc.N + pc] = T(0.125) * s;
    }
    Bc[pc] = fine_face_mean<T, 0>(wf, Bf, i, j, k);
    Bc[wc.N + pc] = fine_face_mean<T, 1>(wf, Bf, i, j, k);
    Bc[2 * wc.N + pc] = fine_face_mean<T, 2>(wf, Bf, i, j, k);
    // upper faces on the boundary of the refined region (owned by the
    // unrefined neighbour)
    if (!refined(wf, i + 1, j, k))
      Bc[nbr(wc, i, j, k, 1, 0, 0)] = fine_face_mean<T, 0>(wf, Bf, wrapc(i + 1, wc.nx), j, k);
    if (!refined(wf, i, j + 1, k))
      Bc[wc.N + nbr(wc, i, j, k, 0, 1, 0)] = fine_face_mean<T, 1>(wf, Bf, i, wrapc(j + 1, wc.ny), k);
    if (!refined(wf, i, j, k + 1))
      Bc[2 * wc.N + nbr(wc, i, j, k, 0, 0, 1)] = fine_face_mean<T, 2>(wf, Bf, i, j, wrapc(k + 1, wc.nz));
  }
}

// Where a level's last update left its final face fluxes and edge EMFs, and
// how to address them (the stage scratch of its context).
struct LevelScratch {
  const void* F;        // [3][7] components of the final fluxes (store_flux order)
  const void* E;        // [3] components of the final edge EMFs
  long long NS;         // component stride
  int sb, ghost;        // per-group boxes (sb = 0: addressed like the level)
  const int* occ;       // group index + 1 per group of the level (list mode)
  const int* groups;
  int edge, gnx, gny, gnz, nx, ny, nz;
};


// listed group holding cell (i, j, k) of the level, or -1
__device__ __forceinline__ int group_at(const LevelScratch& v, int i, int j, int k) {
  i = wrapc(i, v.nx); j = wrapc(j, v.ny); k = wrapc(k, v.nz);
  return v.occ[((long long)(k / v.edge) * v.gny + j / v.edge) * v.gnx + i / v.edge] - 1;
}

// scratch slot of cell (i, j, k) inside the box of group g (list mode), or
// its level index (whole grid)
__device__ __forceinline__ long long slot_at(const LevelScratch& v, int i, int j, int k, int g) {
  if (!v.sb) return ((long long)wrapc(k, v.nz) * v.ny + wrapc(j, v.ny)) * v.nx + wrapc(i, v.nx);
  const int* o = v.groups + 3 * g;
  const long long sb = v.sb;
  const int a = box_offset(i - o[0], -v.ghost, v.nx) + v.ghost, b = box_offset(j - o[1], -v.ghost, v.ny) + v.ghost,
            c = box_offset(k - o[2], -v.ghost, v.nz) + v.ghost;
  return (long long)(g + 1) * sb * sb * sb + ((long long)c * sb + b) * sb + a;
}

// Correction of conserved variables (Sec. 3.3): a coarse cell outside the
// refined region that shares a face with it replaces the coarse flux through
// that face by the mean of the four fine fluxes over the same step.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_correct_u(Work wc, Work wf, LevelScratch sc, LevelScratch sf,
                                                      T* __restrict__ Uc, const double* dt, T inv_dx) {
  const T r = T(*dt) * inv_dx;
  const T* Fc = (const T*)sc.F;
  const T* Ff = (const T*)sf.F;
  FOR_ITEMS(wc, t) {
    int i, j, k;
    cell_of(wc, t, i, j, k);
    if (refined(wf, i, j, k)) continue;
    T du[5] = {T(0), T(0), T(0), T(0), T(0)};
    const int C[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
#pragma unroll
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int D[3] = {i, j, k};
        D[a] += sgn;
        if (!refined(wf, D[0], D[1], D[2])) continue;
        // the face is the lower a-face of its owner O (D above, C below)
        const int* O = sgn > 0 ? D : C;
        const int gc = sc.sb ? group_at(sc, O[0], O[1], O[2]) : 0;
        if (gc < 0) continue;
        const long long qc = slot_at(sc, O[0], O[1], O[2], gc);
        T ff[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int Of[3] = {2 * O[0], 2 * O[1], 2 * O[2]};
          Of[b] += q & 1;
          Of[c] += q >> 1;
          int In[3] = {Of[0], Of[1], Of[2]};   // a fine cell on the refined side
          if (sgn < 0) In[a] -= 1;
          const int gf = sf.sb ? group_at(sf, In[0], In[1], In[2]) : 0;
          const long long qf = slot_at(sf, Of[0], Of[1], Of[2], gf < 0 ? 0 : gf);
#pragma unroll
          for (int m = 0; m < 5; ++m) ff[m] += Ff[((long long)a * 7 + m) * sf.NS + qf];
        }
#pragma unroll
        for (int m = 0; m < 5; ++m) du[m] += T(sgn) * r * (Fc[((long long)a * 7 + m) * sc.NS + qc] - T(0.25) * ff[m]);
      }
    }
    const long long pc = lin(wc, i, j, k);
#pragma unroll
    for (int m = 0; m < 5; ++m) Uc[m * wc.N + pc] += du[m];
  }
}

// EMF difference on the coarse edge along Q owned by coarse cell X (its
// lower corner edge): mean of the two fine EMFs along it minus the coarse
// EMF, when the edge touches the refined region, else 0.
template <typename T, int Q>
__device__ __forceinline__ T edge_emf_jump(const Work& wf, const LevelScratch& sc, const LevelScratch& sf,
                                           const T* __restrict__ Ec, const T* __restrict__ Ef, int x, int y, int z) {
  constexpr int q1 = (Q + 1) % 3, q2 = (Q + 2) % 3;
  const int X[3] = {x, y, z};
  int Y[3] = {0, 0, 0};
  bool touch = false;
#pragma unroll
  for (int s = 0; s < 4 && !touch; ++s) {
    int Z[3] = {X[0], X[1], X[2]};
    Z[q1] -= s & 1;
    Z[q2] -= s >> 1;
    if (refined(wf, Z[0], Z[1], Z[2])) {
      touch = true;
      Y[0] = Z[0]; Y[1] = Z[1]; Y[2] = Z[2];
    }
  }
  if (!touch) return T(0);
  const int gc = sc.sb ? group_at(sc, Y[0], Y[1], Y[2]) : 0;
  if (gc < 0) return T(0);
  const T ec = Ec[(long long)Q * sc.NS + slot_at(sc, X[0], X[1], X[2], gc)];
  T ef = T(0);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int Xf[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
    Xf[Q] += h;
    // a refined fine cell next to the fine edge gives the group whose box holds it
    int In[3] = {2 * Y[0], 2 * Y[1], 2 * Y[2]};
    In[Q] = Xf[Q];
    In[q1] = Y[q1] < X[q1] ? Xf[q1] - 1 : Xf[q1];
    In[q2] = Y[q2] < X[q2] ? Xf[q2] - 1 : Xf[q2];
    const int gf = sf.sb ? group_at(sf, In[0], In[1], In[2]) : 0;
    ef += Ef[(long long)Q * sf.NS + slot_at(sf, Xf[0], Xf[1], Xf[2], gf < 0 ? 0 : gf)];
  }
  return T(0.5) * ef - ec;
}

template <typename T, int A>
__device__ __forceinline__ T face_emf_correction(const Work& wf, const LevelScratch& sc, const LevelScratch& sf,
                                                 const T* __restrict__ Ec, const T* __restrict__ Ef, int x, int y,
                                                 int z, T r) {
  // CT update of the lower A-face of cell (x, y, z) by the edge EMF jumps
  // (same stencil as the update of Eq. 13)
  constexpr int b = (A + 1) % 3, c = (A + 2) % 3;
  int Pb[3] = {x, y, z}, Pc[3] = {x, y, z};
  Pb[b] += 1;
  Pc[c] += 1;
  const T dc0 = edge_emf_jump<T, c>(wf, sc, sf, Ec, Ef, x, y, z);
  const T dc1 = edge_emf_jump<T, c>(wf, sc, sf, Ec, Ef, Pb[0], Pb[1], Pb[2]);
  const T db0 = edge_emf_jump<T, b>(wf, sc, sf, Ec, Ef, x, y, z);
  const T db1 = edge_emf_jump<T, b>(wf, sc, sf, Ec, Ef, Pc[0], Pc[1], Pc[2]);
  return -r * (dc1 - dc0) + r * (db1 - db0);
}

// After the corrections: the coarse level's final fluxes on every face, and
// its final EMFs on every edge, of a refined coarse cell take the fine means,
// so that a correction of the next coarser level across the same interface
// uses the finest fluxes and EMFs (the hierarchy need not be properly
// nested).  Items: the coarse footprints of the fine groups.  Faces and edges
// shared by refined cells are written with the same value by each of them.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_correct_registers(Work wcf, Work wf, LevelScratch sc, LevelScratch sf) {
  T* Fc = (T*)sc.F;
  T* Ec = (T*)sc.E;
  const T* Ff = (const T*)sf.F;
  const T* Ef = (const T*)sf.E;
  FOR_ITEMS(wcf, t) {
    int i, j, k;
    cell_of(wcf, t, i, j, k);
    const int gc = sc.sb ? group_at(sc, i, j, k) : 0;
    if (gc < 0) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      // the lower and the upper a-face of cell (i, j, k)
#pragma unroll
      for (int up = 0; up < 2; ++up) {
        int O[3] = {i, j, k};
        O[a] += up;
        T ff[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int Of[3] = {2 * O[0], 2 * O[1], 2 * O[2]};
          Of[b] += q & 1;
          Of[c] += q >> 1;
          int In[3] = {Of[0], Of[1], Of[2]};
          if (up) In[a] -= 1;    // the refined fine cell below the face
          const int gf = sf.sb ? group_at(sf, In[0], In[1], In[2]) : 0;
          const long long qf = slot_at(sf, Of[0], Of[1], Of[2], gf < 0 ? 0 : gf);
#pragma unroll
          for (int m = 0; m < 7; ++m) ff[m] += Ff[((long long)a * 7 + m) * sf.NS + qf];
        }
        // every listed coarse group whose box holds the face keeps a copy
        int L[3] = {O[0], O[1], O[2]};
        L[a] -= 1;
        const int gs[2] = {sc.sb ? group_at(sc, O[0], O[1], O[2]) : 0, sc.sb ? group_at(sc, L[0], L[1], L[2]) : 0};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (gs[u] < 0 || (u == 1 && gs[1] == gs[0])) continue;
          const long long qc = slot_at(sc, O[0], O[1], O[2], gs[u]);
#pragma unroll
          for (int m = 0; m < 7; ++m) Fc[((long long)a * 7 + m) * sc.NS + qc] = T(0.25) * ff[m];
        }
      }
      // the four a-edges of cell (i, j, k): owners (i, j, k) + {0, e_b} + {0, e_c}
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int X[3] = {i, j, k};
        X[b] += e & 1;
        X[c] += e >> 1;
        T ef = T(0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          int Xf[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
          Xf[a] += h;
          int In[3] = {Xf[0], Xf[1], Xf[2]};   // a fine child of (i, j, k) next to the fine edge
          if (e & 1) In[b] -= 1;
          if (e >> 1) In[c] -= 1;
          const int gf = sf.sb ? group_at(sf, In[0], In[1], In[2]) : 0;
          ef += Ef[(long long)a * sf.NS + slot_at(sf, Xf[0], Xf[1], Xf[2], gf < 0 ? 0 : gf)];
        }
        // every listed coarse group whose box holds the edge keeps a copy
        int gs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int Z[3] = {X[0], X[1], X[2]};
          Z[b] -= u & 1;
          Z[c] -= u >> 1;
          gs[u] = sc.sb ? group_at(sc, Z[0], Z[1], Z[2]) : 0;
          bool dup = gs[u] < 0;
#pragma unroll
          for (int v = 0; v < u; ++v) dup = dup || gs[v] == gs[u];
          if (!dup) Ec[(long long)a * sc.NS + slot_at(sc, X[0], X[1], X[2], gs[u])] = T(0.5) * ef;
        }
      }
    }
  }
}

// Correction of the magnetic field (Sec. 3.3): coarse faces with both cells
// outside the refined region take the CT update of the EMF differences on
// their edges that lie on the coarse-fine interface.  Each listed coarse
// cell owns its lower faces, and its upper faces where the next group is not
// listed (as in the update itself).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_correct_b(Work wc, Work wf, LevelScratch sc, LevelScratch sf,
                                                      T* __restrict__ Bc, const double* dt, T inv_dx) {
  const T r = T(*dt) * inv_dx;
  const T* Ec = (const T*)sc.E;
  const T* Ef = (const T*)sf.E;
  FOR_ITEMS(wc, t) {
    int i, j, k, a0, b0, c0;
    cell_of(wc, t, i, j, k, a0, b0, c0);
    const int pos[3] = {a0, b0, c0};
#pragma unroll
    for (int A = 0; A < 3; ++A) {
#pragma unroll
      for (int up = 0; up < 2; ++up) {
        int H[3] = {i, j, k};   // cell above the face (its owner)
        if (up) {
          if (!wc.groups || pos[A] != wc.edge - 1) continue;
          int G[3] = {i / wc.edge, j / wc.edge, k / wc.edge};
          G[A] += 1;
          const bool listed = wc.occ[((long long)wrapc(G[2], wc.gnz) * wc.gny + wrapc(G[1], wc.gny)) * wc.gnx +
                                     wrapc(G[0], wc.gnx)] != 0;
          if (listed) continue;
          H[A] += 1;
        }
        int L[3] = {H[0], H[1], H[2]};
        L[A] -= 1;
        if (refined(wf, L[0], L[1], L[2]) || refined(wf, H[0], H[1], H[2])) continue;
        T db;
        if (A == 0) db = face_emf_correction<T, 0>(wf, sc, sf, Ec, Ef, H[0], H[1], H[2], r);
        else if (A == 1) db = face_emf_correction<T, 1>(wf, sc, sf, Ec, Ef, H[0], H[1], H[2], r);
        else db = face_emf_correction<T, 2>(wf, sc, sf, Ec, Ef, H[0], H[1], H[2], r);
        if (db != T(0))
          Bc[A * wc.N + lin(wc, wrapc(H[0], wc.nx), wrapc(H[1], wc.ny), wrapc(H[2], wc.nz))] += db;
      }
    }
  }
}

// ---- regridding (refinement / derefinement operation, Sec. 3.3)
// Criterion: |curl B| dx / |B| > thr on the coarse level, decided as
// (jx^2 + jy^2 + jz^2) > thr^2 (bx^2 + by^2 + bz^2) with b the cell-centred
// field and j = dx curl b by central differences.  Contraction is off so
// that the decision rounds like the plain definition.
template <typename T>
__device__ __forceinline__ T cell_b(const Work& w, const T* __restrict__ B, int A, int i, int j, int k) {
  const T* Ba = B + (long long)A * w.N;
  const long long p = lin(w, wrapc(i, w.nx), wrapc(j, w.ny), wrapc(k, w.nz));
  const long long q = lin(w, wrapc(i + (A == 0), w.nx), wrapc(j + (A == 1), w.ny), wrapc(k + (A == 2), w.nz));
  return T(0.5) * (Ba[p] + Ba[q]);
}

template <typename T>
__device__ bool refine_hit(const Work& w, const T* __restrict__ B, int i, int j, int k, T thr) {
#pragma clang fp contract(off)
  const T bx = cell_b(w, B, 0, i, j, k), by = cell_b(w, B, 1, i, j, k), bz = cell_b(w, B, 2, i, j, k);
  const T jx = T(0.5) * (cell_b(w, B, 2, i, j + 1, k) - cell_b(w, B, 2, i, j - 1, k)) -
               T(0.5) * (cell_b(w, B, 1, i, j, k + 1) - cell_b(w, B, 1, i, j, k - 1));
  const T jy = T(0.5) * (cell_b(w, B, 0, i, j, k + 1) - cell_b(w, B, 0, i, j, k - 1)) -
               T(0.5) * (cell_b(w, B, 2, i + 1, j, k) - cell_b(w, B, 2, i - 1, j, k));
  const T jz = T(0.5) * (cell_b(w, B, 1, i + 1, j, k) - cell_b(w, B, 1, i - 1, j, k)) -
               T(0.5) * (cell_b(w, B, 0, i, j + 1, k) - cell_b(w, B, 0, i, j - 1, k));
  return (jx * jx + jy * jy + jz * jz) > thr * thr * (bx * bx + by * by + bz * bz);
}

__global__ void __launch_bounds__(kBlock) k_fill_int(int* p, long long n, int v) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) p[t] = v;
}

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Marks every candidate fine group (a block of e coarse cells per axis,
// g = gnx x gny x gnz of them) whose block widened by `buffer` cells holds a
// coarse cell where the criterion holds.  Items: the coarse cells.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_refine_mark(Work w, const T* __restrict__ B, T thr, int e, int buffer,
                                                        int gnx, int gny, int gnz, int* __restrict__ flags) {
  FOR_ITEMS(w, t) {
    int i, j, k;
    cell_of(w, t, i, j, k);
    if (!refine_hit(w, B, i, j, k, thr)) continue;
    const int xs = floor_div(i - buffer, e), xe = floor_div(i + buffer, e);
    const int ys = floor_div(j - buffer, e), ye = floor_div(j + buffer, e);
    const int zs = floor_div(k - buffer, e), ze = floor_div(k + buffer, e);
    for (int z = zs; z <= ze; ++z)
      for (int y = ys; y <= ye; ++y)
        for (int x = xs; x <= xe; ++x) {
          const long long g = ((long long)wrapc(z, gnz) * gny + wrapc(y, gny)) * gnx + wrapc(x, gnx);
          atomicOr(flags + g, 1);
        }
  }
}

// One block: the marked candidates (inside a listed coarse group when a
// coarse occupancy map is given) become the group list in increasing
// (z, y, x) order; at most `capacity` origins (fine cells) are written,
// *count = min(wanted, capacity), *wanted = the number marked.
__global__ void __launch_bounds__(1024) k_compact_groups(const int* __restrict__ flags, int gnx, int gny, int gnz,
                                                         int e, int fine_edge, const int* __restrict__ cocc,
                                                         int cgnx, int cgny, int coarse_edge,
                                                         int* __restrict__ out, int capacity, int* count,
                                                         int* wanted) {
  __shared__ int wave_sum[16];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  const long long total = (long long)gnx * gny * gnz;
  for (long long c0 = 0; c0 < total; c0 += 1024) {
    const long long g = c0 + tid;
    bool ok = false;
    int gi = 0, gj = 0, gk = 0;
    if (g < total && flags[g]) {
      gi = (int)(g % gnx);
      gj = (int)((g / gnx) % gny);
      gk = (int)(g / ((long long)gnx * gny));
      ok = true;
      if (cocc) {
        const int ci = gi * e / coarse_edge, cj = gj * e / coarse_edge, ck = gk * e / coarse_edge;
        ok = cocc[((long long)ck * cgny + cj) * cgnx + ci] != 0;
      }
    }
    const unsigned long long ballot = __ballot(ok);
    const int before = __popcll(ballot & ((1ull << lane) - 1ull));
    if (lane == 0) wave_sum[wave] = __popcll(ballot);
    __syncthreads();
    int offset = base;
    for (int v = 0; v < wave; ++v) offset += wave_sum[v];
    const int pos = offset + before;
    if (ok && pos < capacity) {
      out[3 * pos + 0] = gi * fine_edge;
      out[3 * pos + 1] = gj * fine_edge;
      out[3 * pos + 2] = gk * fine_edge;
    }
    __syncthreads();
    if (tid == 0) {
      int add = 0;
      for (int v = 0; v < 16; ++v) add += wave_sum[v];
      base += add;
    }
    __syncthreads();
  }
  if (tid == 0) {
    *wanted = base;
    *count = base < capacity ? base : capacity;
  }
}

// Children of a parent under a created fine group.  Faces of the parent
// whose far side is a fine cell of an existing group (occ_old) keep their
// four fine values: their mean and slopes replace the coarse ones in the
// reconstruction and their twist d (the bilinear part) is given back through
// the b-mid-plane faces (b = (A+1)%3) of that layer of children, -d s_g or
// +d s_g for the lower or upper A-face, g the child's position along
// (A+2)%3.  Writes the cells, their lower faces, and the parent's upper
// boundary faces, except faces kept from existing groups.
template <typename T>
__device__ __forceinline__ void prolong_parent_kept(const Work& wc, const Work& wf, const Coarse<T>& Uc,
                                                    const Coarse<T>& Bc, T* __restrict__ Uf, T* __restrict__ Bf,
                                                    const int* __restrict__ occ_old, int i, int j, int k, T gam) {
  auto old_at = [&](int x, int y, int z) {
    if (!occ_old) return false;
    x = wrapc(x, wf.nx); y = wrapc(y, wf.ny); z = wrapc(z, wf.nz);
    return occ_old[((long long)(z / wf.edge) * wf.gny + y / wf.edge) * wf.gnx + x / wf.edge] != 0;
  };
  ParentFaces<T> P;
  load_face_pair<T, 0>(wc, Bc, i, j, k, P);
  load_face_pair<T, 1>(wc, Bc, i, j, k, P);
  load_face_pair<T, 2>(wc, Bc, i, j, k, P);
  const int C[3] = {i, j, k};
  bool kept[3][2];
  T fv[3][2][4];
  T tw[3][2];
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    const int b = (A + 1) % 3, c = (A + 2) % 3;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      int X[3] = {2 * C[0], 2 * C[1], 2 * C[2]};
      X[A] = s ? 2 * C[A] + 2 : 2 * C[A] - 1;
      kept[A][s] = old_at(X[0], X[1], X[2]);
      tw[A][s] = T(0);
      if (kept[A][s]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int F[3] = {2 * C[0], 2 * C[1], 2 * C[2]};
          F[A] = 2 * C[A] + 2 * s;
          F[b] += q & 1;
          F[c] += q >> 1;
          fv[A][s][q] = Bf[(long long)A * wf.N + lin(wf, wrapc(F[0], wf.nx), wrapc(F[1], wf.ny), wrapc(F[2], wf.nz))];
        }
        const T* f = fv[A][s];
        P.v[A][s] = T(0.25) * ((f[0] + f[1]) + (f[2] + f[3]));
        P.s[A][s][0] = (f[1] - f[0]) + (f[3] - f[2]);
        P.s[A][s][1] = (f[2] - f[0]) + (f[3] - f[1]);
        tw[A][s] = T(0.25) * ((f[0] - f[1]) + (f[3] - f[2]));
      }
    }
  }
  T F[3][3][4];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      F[0][p][q] = fine_face<T, 0>(P, p, q);
      F[1][p][q] = fine_face<T, 1>(P, p, q);
      F[2][p][q] = fine_face<T, 2>(P, p, q);
    }
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    const int b = (A + 1) % 3;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!kept[A][s]) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) F[A][2 * s][q] = fv[A][s][q];
#pragma unroll
      for (int g = 0; g < 2; ++g) F[b][1][g + 2 * s] += (s ? T(1) : T(-1)) * tw[A][s] * (g ? T(1) : T(-1));
    }
  }
  T b2[8];
  T mean_b2 = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const T bx = T(0.5) * (F[0][a][b + 2 * c] + F[0][a + 1][b + 2 * c]);
    const T by = T(0.5) * (F[1][b][c + 2 * a] + F[1][b + 1][c + 2 * a]);
    const T bz = T(0.5) * (F[2][c][a + 2 * b] + F[2][c + 1][a + 2 * b]);
    b2[q] = bx * bx + by * by + bz * bz;
    mean_b2 += b2[q];
  }
  mean_b2 *= T(0.125);
  const long long pc = lin(wc, i, j, k);
  // the parent's cell-centred field from its coarse faces
  const Coarse<T> B0 = Bc, B1 = Bc.shift(wc.N), B2 = Bc.shift(2 * wc.N);
  T u[8][5];
  child_cells(wc, Uc, i, j, k, T(0.5) * (B0[pc] + B0[nbr(wc, i, j, k, 1, 0, 0)]),
              T(0.5) * (B1[pc] + B1[nbr(wc, i, j, k, 0, 1, 0)]), T(0.5) * (B2[pc] + B2[nbr(wc, i, j, k, 0, 0, 1)]),
              b2, mean_b2, gam, u);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const long long pf = lin(wf, 2 * i + a, 2 * j + b, 2 * k + c);
#pragma unroll
    for (int m = 0; m < 5; ++m) Uf[m * wf.N + pf] = u[q][m];
    if (a || !kept[0][0]) Bf[pf] = F[0][a][b + 2 * c];
    if (b || !kept[1][0]) Bf[wf.N + pf] = F[1][b][c + 2 * a];
    if (c || !kept[2][0]) Bf[2 * wf.N + pf] = F[2][c][a + 2 * b];
  }
  // the parent's upper boundary faces
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    if (kept[A][1]) continue;
    const int b = (A + 1) % 3, c = (A + 2) % 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int G[3] = {2 * C[0], 2 * C[1], 2 * C[2]};
      G[A] += 2;
      G[b] += q & 1;
      G[c] += q >> 1;
      Bf[(long long)A * wf.N + lin(wf, wrapc(G[0], wf.nx), wrapc(G[1], wf.ny), wrapc(G[2], wf.nz))] = F[A][2][q];
    }
  }
}

// Created fine groups: items are the coarse cells under the groups of the
// new list; groups present in the old list (occ_old) keep their data.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_created(Work wc, Work wf, Coarse<T> Uc, Coarse<T> Bc,
                                                            T* __restrict__ Uf, T* __restrict__ Bf,
                                                            const int* __restrict__ occ_old, T gam) {
  FOR_ITEMS(wc, t) {
    int i, j, k;
    cell_of(wc, t, i, j, k);
    if (occ_old) {
      const int I = wrapc(2 * i, wf.nx), J = wrapc(2 * j, wf.ny), K = wrapc(2 * k, wf.nz);
      if (occ_old[((long long)(K / wf.edge) * wf.gny + J / wf.edge) * wf.gnx + I / wf.edge] != 0) continue;
    }
    prolong_parent_kept(wc, wf, Uc, Bc, Uf, Bf, occ_old, i, j, k, gam);
  }
}

// Time-averaged registers of a sub-cycled level: R = (reset ? 0 : R) + w S
// over the final fluxes and EMFs S of the level's last update.  Whole grid
// (sb = 0): every slot; group list: the slots on each group's boundary shell
// (box positions ghost .. ghost + edge with one coordinate at either end).
// A correction reads registers only on the boundary of the refined region,
// and a group of a finer level never straddles a group boundary of this one
// (groups nest in their parent's groups), so interior slots are never read.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_accumulate_registers(const T* __restrict__ F, const T* __restrict__ E,
                                                                 T* __restrict__ RF, T* __restrict__ RE, long long NS,
                                                                 int sb, int ghost, int edge, long long items, T w,
                                                                 int reset) {
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < items; t += stride) {
    long long q = t;
    if (sb) {
      const long long m = edge + 1, per = m * m * m;
      const long long g = t / per, r = t - g * per;
      const long long a = r % m, b = (r / m) % m, c = r / (m * m);
      if (a != 0 && a != edge && b != 0 && b != edge && c != 0 && c != edge) continue;
      q = (g + 1) * sb * sb * sb + ((c + ghost) * sb + (b + ghost)) * sb + (a + ghost);
    }
#pragma unroll
    for (int m = 0; m < 21; ++m) {
      const long long o = (long long)m * NS + q;
      RF[o] = reset ? w * F[o] : RF[o] + w * F[o];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const long long o = (long long)m * NS + q;
      RE[o] = reset ? w * E[o] : RE[o] + w * E[o];
    }
  }
}

// the step of a sub-cycled finer level: *fine = *coarse / parts
__global__ void k_subdivide_dt(const double* coarse, int parts, double* fine) { *fine = *coarse / parts; }

}  // namespace mhd
