// mhd_kernels.hpp -- stage kernels of the unsplit MHD update on a dense
// periodic level, and the diagnostics reductions.  Included once by
// mhd_api.hip, which instantiates and launches them.
//
// Storage (all SoA, x fastest, N = nx*ny*nz per component):
//   U [5][N]  rho, Mx, My, Mz, e at cell centres
//   B [3][N]  face-area-averaged field on the lower x/y/z face of each cell
//   W [8][N]  primitives rho, vx, vy, vz, p, Bcx, Bcy, Bcz (cell-centred field
//             = mean of the two opposite faces)
//   F [3][7][N] face fluxes of the lower face of each cell, per direction:
//             0 mass, 1..3 momentum x/y/z, 4 energy, 5 E_t1, 6 E_t2 -- the two
//             edge-parallel EMF components carried by the face (E = -V x B)
//   E [3][N]  edge EMFs: Ex on the x-edge at the lower (y, z) corner of the
//             cell, Ey at the lower (z, x) corner, Ez at the lower (x, y) corner.
//
// Work mapping: a launch covers a list of units.  With no group list the
// single unit is the whole grid; with a list each unit is the box of
// (edge + 2*halo)^3 cells around one patch group, with periodic wrap.  Each
// thread owns one cell of one unit.  Block ids are remapped so that each of
// the eight XCDs (which take blocks round-robin) works on a contiguous range
// of cells, which keeps stencil neighbours in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mhd_device.hpp"
#include "mhd_mlp.hpp"

namespace mhd {

constexpr int kBlock = 256;

struct Work {
  int nx, ny, nz;
  long long N;          // cells of the grid
  const int* groups;    // nullptr: whole grid
  int edge;             // group edge in cells
  int halo;             // extra cells around each group
  int box;              // edge + 2 * halo
  long long items;      // work items (cells), upper bound when n_dev is set
  const int* occ;       // group occupancy map (list mode), gnx*gny*gnz
  int gnx, gny, gnz;    // groups per dimension
  const int* n_dev;     // list mode: number of groups read from device memory, or nullptr
  int oshift;           // list mode: group origins are divided by 2^oshift (coarse footprint)
  // Stage scratch (W, F, E, Q, Bh, ...) addressing.  Whole grid: like the
  // level (slot = cell index, stride N).  Group list: each group owns a
  // contiguous box of sb^3 slots (its cells plus sb/2 - edge/2 ghost layers),
  // group g at slot (g + 1) sb^3, with one unused box before and after so
  // stencil reads past a box edge stay inside the allocation.
  long long NS;         // component stride of the scratch arrays
  int sb;               // scratch box edge (0: scratch addressed like the level)
  int soff;             // offset of this stage's item box inside the scratch box
};

// A work item's cell: global coordinates, level index p and scratch slot s;
// (a, b, c) is its position inside the stage's item box.
struct Site {
  int i, j, k;
  int a, b, c;
  long long p, s;
};

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ long long lin(const Work& w, int i, int j, int k) {
  return ((long long)k * w.ny + j) * w.nx + i;
}

// neighbour index with periodic wrap; |di|, |dj|, |dk| <= grid size
__device__ __forceinline__ long long nbr(const Work& w, int i, int j, int k, int di, int dj, int dk) {
  return lin(w, wrapc(i + di, w.nx), wrapc(j + dj, w.ny), wrapc(k + dk, w.nz));
}

// Blocks are dispatched to the 8 XCDs round-robin (block b to XCD b % 8);
// the rank remaps them so each XCD gets a contiguous range of ranks.
__device__ __forceinline__ unsigned block_rank() {
  const unsigned nb = gridDim.x;
  const unsigned b = blockIdx.x;
  const unsigned q = nb >> 3;
  return b < (q << 3) ? (b & 7u) * q + (b >> 3) : b;
}

__device__ __forceinline__ long long block_linear_id() { return (long long)block_rank() * kBlock + threadIdx.x; }

// Persistent launches: a grid of at most a tuned number of blocks walks the
// work items with a grid-wide stride; the item count of a group list may be
// read from device memory, so a captured graph replays over a changed list.
__device__ __forceinline__ long long work_items(const Work& w) {
  if (w.n_dev) {
    const long long n = *w.n_dev;
    const long long m = (long long)w.box * w.box * w.box * n;
    return m < w.items ? m : w.items;
  }
  return w.items;
}
__device__ __forceinline__ long long item_stride() { return (long long)gridDim.x * kBlock; }

// cell of work item t.  (a, b, c) is the position inside the unit's box (the
// cell itself for a whole grid).
__device__ __forceinline__ void cell_of(const Work& w, long long t, int& i, int& j, int& k, int& a, int& b, int& c) {
  if (w.groups == nullptr) {
    i = (int)(t % w.nx);
    const long long r = t / w.nx;
    j = (int)(r % w.ny);
    k = (int)(r / w.ny);
    a = i; b = j; c = k;
  } else {
    const long long per = (long long)w.box * w.box * w.box;
    const int g = (int)(t / per);
    const int l = (int)(t - (long long)g * per);
    a = l % w.box;
    b = (l / w.box) % w.box;
    c = l / (w.box * w.box);
    i = wrapc((w.groups[3 * g + 0] >> w.oshift) - w.halo + a, w.nx);
    j = wrapc((w.groups[3 * g + 1] >> w.oshift) - w.halo + b, w.ny);
    k = wrapc((w.groups[3 * g + 2] >> w.oshift) - w.halo + c, w.nz);
  }
}

__device__ __forceinline__ void cell_of(const Work& w, long long t, int& i, int& j, int& k) {
  int a, b, c;
  cell_of(w, t, i, j, k, a, b, c);
}

// L: list mode with per-group scratch boxes (compile time, so the
// whole-grid kernels carry no list arithmetic)
template <bool L>
__device__ __forceinline__ Site site_of(const Work& w, long long t) {
  Site st;
  cell_of(w, t, st.i, st.j, st.k, st.a, st.b, st.c);
  st.p = lin(w, st.i, st.j, st.k);
  if constexpr (L) {
    const long long per = (long long)w.box * w.box * w.box;
    const long long g = t / per;
    const long long sb = w.sb;
    st.s = (g + 1) * sb * sb * sb + ((long long)(st.c + w.soff) * sb + (st.b + w.soff)) * sb + (st.a + w.soff);
  } else {
    st.s = st.p;
  }
  return st;
}

// scratch slot of the cell (di, dj, dk) away
template <bool L>
__device__ __forceinline__ long long snb(const Work& w, const Site& st, int di, int dj, int dk) {
  if constexpr (L) return st.s + di + (long long)dj * w.sb + (long long)dk * w.sb * w.sb;
  else return nbr(w, st.i, st.j, st.k, di, dj, dk);
}

// the neighbouring cell as a site (level index and scratch slot)
template <bool L>
__device__ __forceinline__ Site site_nb(const Work& w, const Site& st, int di, int dj, int dk) {
  Site n;
  n.i = wrapc(st.i + di, w.nx);
  n.j = wrapc(st.j + dj, w.ny);
  n.k = wrapc(st.k + dk, w.nz);
  n.a = st.a + di; n.b = st.b + dj; n.c = st.c + dk;
  n.p = lin(w, n.i, n.j, n.k);
  if constexpr (L) n.s = st.s + di + (long long)dj * w.sb + (long long)dk * w.sb * w.sb;
  else n.s = n.p;
  return n;
}

// loop over this thread's work items
#define FOR_ITEMS(w, t) for (long long t = block_linear_id(), t##_n = work_items(w); t < t##_n; t += item_stride())


// time step source: explicit value, device scalar, or CFL maximum signal
// speed (stored as the bit pattern of a positive double)
struct DtSrc {
  double val;
  const double* ptr;
  const unsigned long long* smax;
  double courant_dx;
};

__device__ __forceinline__ double get_dt(const DtSrc& s) {
  if (s.smax) return s.courant_dx / __longlong_as_double((long long)*s.smax);
  if (s.ptr) return *s.ptr;
  return s.val;
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------ primitives
// Energy storage of the mixed form: total energy in double, and the plasma
// beta below which the pressure is recovered in double.
struct Mix {
  double* E64;      // nullptr unless the mixed form
  double beta;
};

// gas pressure from the total energy (Eq. 5).  In the mixed form the
// subtraction p = (gam-1)(e - rho v^2/2 - B^2/2) is redone in double when
// the plasma beta 2p/|B|^2 of the float estimate is below mix.beta: there
// the kinetic and magnetic terms nearly cancel e.
template <typename T, bool MIX>
__device__ __forceinline__ T recover_pressure(double e, T d, T vx, T vy, T vz, T bx, T by, T bz, T gam,
                                              double beta) {
  const T b2 = bx * bx + by * by + bz * bz;
  const T pf = (gam - T(1)) * (T(e) - T(0.5) * d * (vx * vx + vy * vy + vz * vz) - T(0.5) * b2);
  if (MIX && T(2) * pf < T(beta) * b2) {
    const double dd = d, ux = vx, uy = vy, uz = vz, b2d = (double)bx * bx + (double)by * by + (double)bz * bz;
    return T(((double)gam - 1.0) * (e - 0.5 * dd * (ux * ux + uy * uy + uz * uz) - 0.5 * b2d));
  }
  return pf;
}

template <typename T, bool MIX>
__device__ __forceinline__ void cell_prims(const Work& w, const T* __restrict__ U, const T* __restrict__ B,
                                           const Mix& mix, int i, int j, int k, T gam, T out[8]) {
  const long long N = w.N;
  const long long p = lin(w, i, j, k);
  const T bx = T(0.5) * (B[p] + B[nbr(w, i, j, k, 1, 0, 0)]);
  const T by = T(0.5) * (B[N + p] + B[N + nbr(w, i, j, k, 0, 1, 0)]);
  const T bz = T(0.5) * (B[2 * N + p] + B[2 * N + nbr(w, i, j, k, 0, 0, 1)]);
  const T d = U[p];
  const T id = T(1) / d;
  const T vx = U[N + p] * id, vy = U[2 * N + p] * id, vz = U[3 * N + p] * id;
  T pr;
  if (MIX) {
    pr = recover_pressure<T, true>(mix.E64[p], d, vx, vy, vz, bx, by, bz, gam, mix.beta);
  } else {
    pr = (gam - T(1)) * (U[4 * N + p] - T(0.5) * d * (vx * vx + vy * vy + vz * vz) -
                         T(0.5) * (bx * bx + by * by + bz * bz));
  }
  out[0] = d; out[1] = vx; out[2] = vy; out[3] = vz; out[4] = pr; out[5] = bx; out[6] = by; out[7] = bz;
}

// sum over directions of |v_d| + c_f,d, in double
template <typename T>
__device__ __forceinline__ double signal_speed(const T q[8], T gam) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const T cf = fast_speed(q[0], q[4], q[5 + a], q[5 + b], q[5 + c], gam);
    s += (double)(dabs(q[1 + a]) + cf);
  }
  return s;
}

__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* smax) {
  __shared__ double red[kBlock / 64];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int q = 1; q < kBlock / 64; ++q) m = fmax(m, red[q]);
    // most blocks see a maximum already reached: skip their atomic
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    if (m > 0.0 && bits > *(volatile unsigned long long*)smax) atomicMax(smax, bits);
  }
}

// Primitive state of every cell; optionally the CFL maximum signal speed and
// the sticky non-physical flag.
template <typename T, bool CFL, bool MIX, bool L>
__global__ void __launch_bounds__(kBlock) k_prim(Work w, const T* __restrict__ U, const T* __restrict__ B, Mix mix,
                                                 T* __restrict__ W, T gam, unsigned long long* smax,
                                                 int* flag) {
  double s = 0.0;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    T q[8];
    cell_prims<T, MIX>(w, U, B, mix, st.i, st.j, st.k, gam, q);
#pragma unroll
    for (int m = 0; m < 8; ++m) W[m * w.NS + st.s] = q[m];
    if (!(q[0] > T(0)) || !(q[4] > T(0))) atomicOr(flag, 1);
    else if (CFL) s = fmax(s, signal_speed(q, gam));
  }
  if (CFL) block_max_atomic(s, smax);
}

// CFL maximum signal speed only
template <typename T, bool MIX>
__global__ void __launch_bounds__(kBlock) k_cfl(Work w, const T* __restrict__ U, const T* __restrict__ B, Mix mix,
                                                T gam, unsigned long long* smax, int* flag) {
  double s = 0.0;
  FOR_ITEMS(w, t) {
    int i, j, k;
    cell_of(w, t, i, j, k);
    T q[8];
    cell_prims<T, MIX>(w, U, B, mix, i, j, k, gam, q);
    if (!(q[0] > T(0)) || !(q[4] > T(0))) atomicOr(flag, 1);
    else s = fmax(s, signal_speed(q, gam));
  }
  block_max_atomic(s, smax);
}

__global__ void k_reset_smax(unsigned long long* smax) { *smax = 0ull; }

// *dt = min(*dt, courant dx / smax)
__global__ void k_min_dt(const unsigned long long* smax, double courant_dx, double* dt) {
  const double v = courant_dx / __longlong_as_double((long long)*smax);
  if (v < *dt) *dt = v;
}

// dt = courant dx / smax into an output scalar, and t += dt
__global__ void k_publish_dt(const unsigned long long* smax, double courant_dx, double* dt_out, double* t_out) {
  const double dt = courant_dx / __longlong_as_double((long long)*smax);
  if (dt_out) *dt_out = dt;
  if (t_out) *t_out += dt;
}

// ------------------------------------------------------------ fluxes
template <typename T, int D>
__device__ __forceinline__ void load_w1d(const T* __restrict__ W, long long N, long long q, T w[7]) {
  constexpr int n = D, t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  w[0] = W[q];
  w[1] = W[(1 + n) * N + q];
  w[2] = W[(1 + t1) * N + q];
  w[3] = W[(1 + t2) * N + q];
  w[4] = W[4 * N + q];
  w[5] = W[(5 + t1) * N + q];
  w[6] = W[(5 + t2) * N + q];
}

// RECON: 0 = first order (cell states), 1 = PLM with minmod on primitives.
// The normal field Bn is the level's B (predictor: Bn[D N + p]) or the
// half-step scratch Bh (corrector: Bn[D NS + s]); RECON 1 is the corrector.
template <typename T, int D, int RECON, int SOLVER, bool L>
__device__ __forceinline__ int face_flux(const Work& w, const T* __restrict__ W, const T* __restrict__ Bn,
                                         T* __restrict__ F, const Site& st, T gam) {
  const long long NS = w.NS;
  const long long pR = st.s;
  const long long pL = snb<L>(w, st, D == 0 ? -1 : 0, D == 1 ? -1 : 0, D == 2 ? -1 : 0);
  T wl[7], wr[7];
  load_w1d<T, D>(W, NS, pL, wl);
  load_w1d<T, D>(W, NS, pR, wr);
  if (RECON == 1) {
    const long long pLL = snb<L>(w, st, D == 0 ? -2 : 0, D == 1 ? -2 : 0, D == 2 ? -2 : 0);
    const long long pRR = snb<L>(w, st, D == 0 ? 1 : 0, D == 1 ? 1 : 0, D == 2 ? 1 : 0);
    T wll[7], wrr[7];
    load_w1d<T, D>(W, NS, pLL, wll);
    load_w1d<T, D>(W, NS, pRR, wrr);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const T sL = minmod(wl[m] - wll[m], wr[m] - wl[m]);
      const T sR = minmod(wr[m] - wl[m], wrr[m] - wr[m]);
      wl[m] = wl[m] + T(0.5) * sL;
      wr[m] = wr[m] - T(0.5) * sR;
    }
  }
  const T bn = RECON == 1 ? Bn[D * NS + st.s] : Bn[D * w.N + st.p];
  T f[7];
  const int fb = riemann<SOLVER>(wl, wr, bn, gam, f);
  constexpr int n = D, t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  T* Fd = F + (long long)D * 7 * NS;
  Fd[pR] = f[0];
  Fd[(1 + n) * NS + pR] = f[1];
  Fd[(1 + t1) * NS + pR] = f[2];
  Fd[(1 + t2) * NS + pR] = f[3];
  Fd[4 * NS + pR] = f[4];
  Fd[5 * NS + pR] = f[6];    // E_t1 = F_n[B_t2]
  Fd[6 * NS + pR] = -f[5];   // E_t2 = -F_n[B_t1]
  return fb;
}

__device__ __forceinline__ void block_count_atomic(int v, unsigned long long* counter) {
  __shared__ int red[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kBlock / 64; ++q) s += red[q];
    if (s) atomicAdd(counter, (unsigned long long)s);
  }
}

// VL flux stage; B is the level's field for RECON 0 and the half-step
// scratch Bh for RECON 1 (see face_flux).
template <typename T, int RECON, int SOLVER, bool L>
__global__ void __launch_bounds__(kBlock) k_flux(Work w, const T* __restrict__ W, const T* __restrict__ B,
                                                 T* __restrict__ F, T gam, unsigned long long* nfb) {
  int fb = 0;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    fb += face_flux<T, 0, RECON, SOLVER, L>(w, W, B, F, st, gam);
    fb += face_flux<T, 1, RECON, SOLVER, L>(w, W, B, F, st, gam);
    fb += face_flux<T, 2, RECON, SOLVER, L>(w, W, B, F, st, gam);
  }
  if (SOLVER == 0) block_count_atomic(fb, nfb);
}

// ------------------------------------------------------------ edge EMFs
template <typename T>
__device__ __forceinline__ T ref_emf(const T* __restrict__ W, long long N, long long q, int a) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  return -(W[(1 + b) * N + q] * W[(5 + c) * N + q] - W[(1 + c) * N + q] * W[(5 + b) * N + q]);
}

template <typename T>
__device__ __forceinline__ T upwind(T m, T pos, T neg) {
  return m > T(0) ? pos : (m < T(0) ? neg : T(0.5) * (pos + neg));
}

// E_a on the edge at the lower (b, c) corner of cell (i, j, k), (a, b, c)
// cyclic, from the four faces around the edge (upwind CT average of
// Gardiner & Stone 2005): each face value is extrapolated to the edge with
// the derivative taken in the upwind cell (sign of the face mass flux), and
// the four extrapolations are averaged.
template <typename T, int A, bool L>
__device__ __forceinline__ T edge_emf(const Work& w, const T* __restrict__ F, const T* __restrict__ W,
                                      const Site& st) {
  constexpr int b = (A + 1) % 3, c = (A + 2) % 3;
  const long long N = w.NS;
  const T* Fb = F + (long long)b * 7 * N;
  const T* Fc = F + (long long)c * 7 * N;
  const int ob[3] = {b == 0 ? -1 : 0, b == 1 ? -1 : 0, b == 2 ? -1 : 0};
  const int oc[3] = {c == 0 ? -1 : 0, c == 1 ? -1 : 0, c == 2 ? -1 : 0};
  const long long p = st.s;
  const long long pb = snb<L>(w, st, ob[0], ob[1], ob[2]);
  const long long pc = snb<L>(w, st, oc[0], oc[1], oc[2]);
  const long long pbc = snb<L>(w, st, ob[0] + oc[0], ob[1] + oc[1], ob[2] + oc[2]);
  const T eb0 = Fb[6 * N + pc], eb1 = Fb[6 * N + p];
  const T ec0 = Fc[5 * N + pb], ec1 = Fc[5 * N + p];
  const T mb0 = Fb[pc], mb1 = Fb[p], mc0 = Fc[pb], mc1 = Fc[p];
  const T r00 = ref_emf(W, N, pbc, A), r10 = ref_emf(W, N, pc, A);
  const T r01 = ref_emf(W, N, pb, A), r11 = ref_emf(W, N, p, A);
  const T dc1 = upwind(mb1, r01 - ec0, r11 - ec1);
  const T dc0 = upwind(mb0, ec0 - r00, ec1 - r10);
  const T db1 = upwind(mc1, r10 - eb0, r11 - eb1);
  const T db0 = upwind(mc0, eb0 - r00, eb1 - r01);
  return T(0.25) * (eb0 + eb1 + ec0 + ec1) + T(0.25) * ((dc0 - dc1) + (db0 - db1));
}

template <typename T, bool L>
__global__ void __launch_bounds__(kBlock) k_emf(Work w, const T* __restrict__ F, const T* __restrict__ W,
                                                T* __restrict__ E) {
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    E[st.s] = edge_emf<T, 0, L>(w, F, W, st);
    E[w.NS + st.s] = edge_emf<T, 1, L>(w, F, W, st);
    E[2 * w.NS + st.s] = edge_emf<T, 2, L>(w, F, W, st);
  }
}

// ------------------------------------------------------------ updates
// U - r div F (Eq. 10), differences applied in the order x, y, z.  In the
// mixed form the energy is updated in double from E64 (returned in e64).
template <typename T, bool MIX, bool L>
__device__ __forceinline__ void cell_update(const Work& w, const T* __restrict__ U, const T* __restrict__ F,
                                            const Mix& mix, const Site& st, T r, T out[5], double& e64) {
  const long long N = w.N, NS = w.NS;
  const long long p = st.p, s = st.s;
  const long long px = snb<L>(w, st, 1, 0, 0), py = snb<L>(w, st, 0, 1, 0), pz = snb<L>(w, st, 0, 0, 1);
  const T* Fx = F;
  const T* Fy = F + 7 * NS;
  const T* Fz = F + 14 * NS;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (MIX && m == 4) {
      const double rd = (double)r;
      double v = mix.E64[p];
      v -= rd * ((double)Fx[4 * NS + px] - (double)Fx[4 * NS + s]);
      v -= rd * ((double)Fy[4 * NS + py] - (double)Fy[4 * NS + s]);
      v -= rd * ((double)Fz[4 * NS + pz] - (double)Fz[4 * NS + s]);
      e64 = v;
      out[4] = T(v);
      continue;
    }
    T v = U[m * N + p];
    v -= r * (Fx[m * NS + px] - Fx[m * NS + s]);
    v -= r * (Fy[m * NS + py] - Fy[m * NS + s]);
    v -= r * (Fz[m * NS + pz] - Fz[m * NS + s]);
    out[m] = v;
  }
  if (!MIX) e64 = (double)out[4];
}

// CT update of the three lower faces of cell (i, j, k) (Eq. 13)
template <typename T, bool L>
__device__ __forceinline__ void face_update(const Work& w, const T* __restrict__ B, const T* __restrict__ E,
                                            const Site& st, T r, T out[3]) {
  const long long N = w.N, NS = w.NS;
  const long long p = st.p, s = st.s;
  const long long px = snb<L>(w, st, 1, 0, 0), py = snb<L>(w, st, 0, 1, 0), pz = snb<L>(w, st, 0, 0, 1);
  const T* Ex = E;
  const T* Ey = E + NS;
  const T* Ez = E + 2 * NS;
  out[0] = B[p] - r * (Ez[py] - Ez[s]) + r * (Ey[pz] - Ey[s]);
  out[1] = B[N + p] - r * (Ex[pz] - Ex[s]) + r * (Ez[px] - Ez[s]);
  out[2] = B[2 * N + p] - r * (Ey[px] - Ey[s]) + r * (Ex[py] - Ex[s]);
}

// Half step over dt/2: U^{n+1/2} and face B^{n+1/2} from the predictor fluxes
// and EMFs, written as primitives Wh (cell-centred field from the updated
// faces, including the upper faces owned by the neighbours) and Bh.
template <typename T, bool MIX, bool L>
__global__ void __launch_bounds__(kBlock) k_half(Work w, const T* __restrict__ U, const T* __restrict__ B, Mix mix,
                                                 const T* __restrict__ F, const T* __restrict__ E, DtSrc dts,
                                                 T inv_dx, T gam, T* __restrict__ Wh, T* __restrict__ Bh) {
  const T r = T(0.5 * get_dt(dts)) * inv_dx;
  FOR_ITEMS(w, t) {
  const Site st = site_of<L>(w, t);
  T u[5], bl[3], bux[3], buy[3], buz[3];
  double eh;
  cell_update<T, MIX, L>(w, U, F, mix, st, r, u, eh);
  face_update<T, L>(w, B, E, st, r, bl);
  face_update<T, L>(w, B, E, site_nb<L>(w, st, 1, 0, 0), r, bux);
  face_update<T, L>(w, B, E, site_nb<L>(w, st, 0, 1, 0), r, buy);
  face_update<T, L>(w, B, E, site_nb<L>(w, st, 0, 0, 1), r, buz);
  const T bx = T(0.5) * (bl[0] + bux[0]);
  const T by = T(0.5) * (bl[1] + buy[1]);
  const T bz = T(0.5) * (bl[2] + buz[2]);
  const T d = u[0];
  const T id = T(1) / d;
  const T vx = u[1] * id, vy = u[2] * id, vz = u[3] * id;
  T pr;
  if (MIX) pr = recover_pressure<T, true>(eh, d, vx, vy, vz, bx, by, bz, gam, mix.beta);
  else pr = (gam - T(1)) * (u[4] - T(0.5) * d * (vx * vx + vy * vy + vz * vz) - T(0.5) * (bx * bx + by * by + bz * bz));
  const long long N = w.NS;
  const long long p = st.s;
  Wh[p] = d; Wh[N + p] = vx; Wh[2 * N + p] = vy; Wh[3 * N + p] = vz; Wh[4 * N + p] = pr;
  Wh[5 * N + p] = bx; Wh[6 * N + p] = by; Wh[7 * N + p] = bz;
  Bh[p] = bl[0]; Bh[N + p] = bl[1]; Bh[2 * N + p] = bl[2];
  }
}

// Full step over dt from time n (in place: each thread reads and writes only
// its own cell and its own lower faces).
//
// With a group list, a cell on the upper boundary of its group also updates
// the face it shares with the next cell when the next cell's group is not
// listed (occupancy map), so every face of a listed group advances exactly
// once and no face is read after another thread has written it.
template <typename T, bool MIX, bool L>
__global__ void __launch_bounds__(kBlock) k_final(Work w, T* __restrict__ U, T* __restrict__ B, Mix mix,
                                                  const T* __restrict__ F, const T* __restrict__ E, DtSrc dts,
                                                  T inv_dx) {
  const T r = T(get_dt(dts)) * inv_dx;
  const long long N = w.N;
  FOR_ITEMS(w, t) {
  const Site st = site_of<L>(w, t);
  const int i = st.i, j = st.j, k = st.k, a = st.a, b = st.b, c = st.c;
  T u[5], bf[3];
  double e64;
  cell_update<T, MIX, L>(w, U, F, mix, st, r, u, e64);
  face_update<T, L>(w, B, E, st, r, bf);
  T ux[3], uy[3], uz[3];
  bool ex = false, ey = false, ez = false;
  if constexpr (L) {
    const int gi = i / w.edge, gj = j / w.edge, gk = k / w.edge;
    auto listed = [&](int x, int y, int z) {
      return w.occ[((long long)wrapc(z, w.gnz) * w.gny + wrapc(y, w.gny)) * w.gnx + wrapc(x, w.gnx)] != 0;
    };
    ex = a == w.edge - 1 && !listed(gi + 1, gj, gk);
    ey = b == w.edge - 1 && !listed(gi, gj + 1, gk);
    ez = c == w.edge - 1 && !listed(gi, gj, gk + 1);
  }
  if (ex) face_update<T, L>(w, B, E, site_nb<L>(w, st, 1, 0, 0), r, ux);
  if (ey) face_update<T, L>(w, B, E, site_nb<L>(w, st, 0, 1, 0), r, uy);
  if (ez) face_update<T, L>(w, B, E, site_nb<L>(w, st, 0, 0, 1), r, uz);
  const long long p = st.p;
#pragma unroll
  for (int m = 0; m < 5; ++m) U[m * N + p] = u[m];
  if (MIX) mix.E64[p] = e64;
  B[p] = bf[0]; B[N + p] = bf[1]; B[2 * N + p] = bf[2];
  if (ex) B[nbr(w, i, j, k, 1, 0, 0)] = ux[0];
  if (ey) B[N + nbr(w, i, j, k, 0, 1, 0)] = uy[1];
  if (ez) B[2 * N + nbr(w, i, j, k, 0, 0, 1)] = uz[2];
  }
}

// ------------------------------------------------------------ CTU
// Step 1 of CTU: time-centred states at both edges of every cell in each
// direction.  Face-indexed outputs: QR[d][m][p] is the state above the lower
// d-face of cell p (from cell p), QL[d][m][p] the state below it (from the
// cell p - e_d; written by that cell as its upper-edge state).
template <typename T, int D, int RECON, bool L>
__device__ __forceinline__ void cell_states(const Work& w, const T* __restrict__ W, const T* __restrict__ B,
                                            T* __restrict__ QL, T* __restrict__ QR, const Site& st, T dtdx,
                                            T gam) {
  const long long N = w.N, NS = w.NS;
  T q[5][7];
#pragma unroll
  for (int s = -2; s <= 2; ++s) {
    const long long c = snb<L>(w, st, D == 0 ? s : 0, D == 1 ? s : 0, D == 2 ? s : 0);
    load_w1d<T, D>(W, NS, c, q[s + 2]);
  }
  const long long pu = nbr(w, st.i, st.j, st.k, D == 0 ? 1 : 0, D == 1 ? 1 : 0, D == 2 ? 1 : 0);
  const long long su = snb<L>(w, st, D == 0 ? 1 : 0, D == 1 ? 1 : 0, D == 2 ? 1 : 0);
  T sl[7], sr[7];
  trace_cell<T, RECON>(q, B[D * N + st.p], B[D * N + pu], dtdx, gam, sl, sr);
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    QR[((long long)D * 7 + m) * NS + st.s] = sl[m];
    QL[((long long)D * 7 + m) * NS + su] = sr[m];
  }
}

template <typename T, int RECON, bool L>
__global__ void __launch_bounds__(kBlock) k_ctu_states(Work w, const T* __restrict__ W, const T* __restrict__ B,
                                                       T* __restrict__ QL, T* __restrict__ QR, DtSrc dts,
                                                       T inv_dx, T gam) {
  const T dtdx = T(get_dt(dts)) * inv_dx;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    cell_states<T, 0, RECON, L>(w, W, B, QL, QR, st, dtdx, gam);
    cell_states<T, 1, RECON, L>(w, W, B, QL, QR, st, dtdx, gam);
    cell_states<T, 2, RECON, L>(w, W, B, QL, QR, st, dtdx, gam);
  }
}

template <typename T, int D>
__device__ __forceinline__ void store_flux(T* __restrict__ F, long long N, long long p, const T f[7]) {
  constexpr int n = D, t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  T* Fd = F + (long long)D * 7 * N;
  Fd[p] = f[0];
  Fd[(1 + n) * N + p] = f[1];
  Fd[(1 + t1) * N + p] = f[2];
  Fd[(1 + t2) * N + p] = f[3];
  Fd[4 * N + p] = f[4];
  Fd[5 * N + p] = f[6];
  Fd[6 * N + p] = -f[5];
}

// Step 2: Riemann fluxes from the stored states with the time-n normal field
template <typename T, int SOLVER, bool L>
__global__ void __launch_bounds__(kBlock) k_flux_q(Work w, const T* __restrict__ QL, const T* __restrict__ QR,
                                                   const T* __restrict__ B, T* __restrict__ F, T gam,
                                                   unsigned long long* nfb, Capture cp) {
  int fb = 0;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    const long long N = w.N, NS = w.NS;
    const long long p = st.p, s = st.s;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T wl[7], wr[7], f[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        wl[m] = QL[((long long)d * 7 + m) * NS + s];
        wr[m] = QR[((long long)d * 7 + m) * NS + s];
      }
      fb += riemann<SOLVER>(wl, wr, B[d * N + p], gam, f);
      if constexpr (sizeof(T) == 4) capture_face(cp, 3 * p + d, wl, wr, B[d * N + p], f);
      if (d == 0) store_flux<T, 0>(F, NS, s, f);
      else if (d == 1) store_flux<T, 1>(F, NS, s, f);
      else store_flux<T, 2>(F, NS, s, f);
    }
  }
  if (SOLVER == 0) block_count_atomic(fb, nfb);
}

// Step 5: transverse correction of a state of direction D that comes from
// cell (ci, cj, ck) and sits on a face with time-n normal field bn.  Hydro
// variables: minus dt/2 times the transverse flux differences of step 2 in
// that cell.  Transverse field: dt/2 times the transverse part of -curl E
// with the step-3 edge EMFs E_D averaged to the cell's faces.  The normal
// field of the conversion is kept.  Non-physical results keep the input.
template <typename T, int D, bool L>
__device__ __forceinline__ void correct_state(const Work& w, const T* __restrict__ F1, const T* __restrict__ E1,
                                              const Site& src, T bn, T hr, T gam, const T s[7], T out[7]) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const long long N = w.NS;
  T v[3], b[3];
  v[D] = s[1]; v[t1] = s[2]; v[t2] = s[3];
  b[D] = bn; b[t1] = s[5]; b[t2] = s[6];
  T u[5];
  u[0] = s[0];
  u[1] = s[0] * v[0];
  u[2] = s[0] * v[1];
  u[3] = s[0] * v[2];
  u[4] = s[4] / (gam - T(1)) + T(0.5) * s[0] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
         T(0.5) * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  const long long c = src.s;
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t = tt ? t2 : t1;
    const long long cp = snb<L>(w, src, t == 0, t == 1, t == 2);
    const T* Ft = F1 + (long long)t * 7 * N;
#pragma unroll
    for (int m = 0; m < 5; ++m) u[m] -= hr * (Ft[m * N + cp] - Ft[m * N + c]);
  }
  const T* Ed = E1 + (long long)D * N;
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int bax = tt ? t2 : t1;
    const int der = (bax == (D + 2) % 3) ? (D + 1) % 3 : (D + 2) % 3;
    const long long e_der = snb<L>(w, src, der == 0, der == 1, der == 2);
    const long long e_b = snb<L>(w, src, bax == 0, bax == 1, bax == 2);
    const long long e_db = snb<L>(w, src, (der == 0) + (bax == 0), (der == 1) + (bax == 1), (der == 2) + (bax == 2));
    const T up = T(0.5) * (Ed[e_der] + Ed[e_db]);
    const T lo = T(0.5) * (Ed[c] + Ed[e_b]);
    const T sign = (D == (bax + 1) % 3) ? T(1) : T(-1);
    b[bax] += hr * sign * (up - lo);
  }
  const T id = T(1) / u[0];
  const T vx = u[1] * id, vy = u[2] * id, vz = u[3] * id;
  const T pr = (gam - T(1)) * (u[4] - T(0.5) * u[0] * (vx * vx + vy * vy + vz * vz) -
                               T(0.5) * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
  if (u[0] > T(0) && pr > T(0)) {
    const T vv[3] = {vx, vy, vz};
    out[0] = u[0]; out[1] = vv[D]; out[2] = vv[t1]; out[3] = vv[t2]; out[4] = pr; out[5] = b[t1]; out[6] = b[t2];
  } else {
#pragma unroll
    for (int m = 0; m < 7; ++m) out[m] = s[m];
  }
}

template <typename T, int D, bool L>
__device__ __forceinline__ void corrected_states(const Work& w, const T* __restrict__ QL, const T* __restrict__ QR,
                                                 const T* __restrict__ F1, const T* __restrict__ E1,
                                                 const T* __restrict__ B, const Site& st, T hr, T gam, T wl[7],
                                                 T wr[7]) {
  const long long NS = w.NS;
  T sl[7], sr[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    sl[m] = QL[((long long)D * 7 + m) * NS + st.s];
    sr[m] = QR[((long long)D * 7 + m) * NS + st.s];
  }
  const T bn = B[D * w.N + st.p];
  correct_state<T, D, L>(w, F1, E1, site_nb<L>(w, st, -(D == 0), -(D == 1), -(D == 2)), bn, hr, gam, sl, wl);
  correct_state<T, D, L>(w, F1, E1, st, bn, hr, gam, sr, wr);
}

template <typename T, int D, int SOLVER, bool L>
__device__ __forceinline__ int corrected_face_flux(const Work& w, const T* __restrict__ QL, const T* __restrict__ QR,
                                                   const T* __restrict__ F1, const T* __restrict__ E1,
                                                   const T* __restrict__ B, const T* __restrict__ Bh,
                                                   T* __restrict__ F2, const Site& st, T hr, T gam,
                                                   const Capture& cp) {
  const long long NS = w.NS;
  T wl[7], wr[7], f[7];
  corrected_states<T, D, L>(w, QL, QR, F1, E1, B, st, hr, gam, wl, wr);
  const T bn = Bh[D * NS + st.s];
  const int fb = riemann<SOLVER>(wl, wr, bn, gam, f);
  if constexpr (sizeof(T) == 4) capture_face(cp, 3 * st.p + D, wl, wr, bn, f);
  store_flux<T, D>(F2, NS, st.s, f);
  return fb;
}

// Steps 5-6: corrected states and Riemann fluxes with the half-step normal field
template <typename T, int SOLVER, bool L>
__global__ void __launch_bounds__(kBlock) k_ctu_correct(Work w, const T* __restrict__ QL, const T* __restrict__ QR,
                                                        const T* __restrict__ F1, const T* __restrict__ E1,
                                                        const T* __restrict__ B, const T* __restrict__ Bh,
                                                        T* __restrict__ F2, DtSrc dts, T inv_dx, T gam,
                                                        unsigned long long* nfb, Capture cp) {
  int fb = 0;
  const T hr = T(0.5 * get_dt(dts)) * inv_dx;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    fb += corrected_face_flux<T, 0, SOLVER, L>(w, QL, QR, F1, E1, B, Bh, F2, st, hr, gam, cp);
    fb += corrected_face_flux<T, 1, SOLVER, L>(w, QL, QR, F1, E1, B, Bh, F2, st, hr, gam, cp);
    fb += corrected_face_flux<T, 2, SOLVER, L>(w, QL, QR, F1, E1, B, Bh, F2, st, hr, gam, cp);
  }
  if (SOLVER == 0) block_count_atomic(fb, nfb);
}

// Learned-flux form of steps 5-6, one direction D per launch pair: the
// corrected states of the D-faces go to Qc (14 words per cell: L then R),
// then the network (or HLLD at strong jumps) turns them into fluxes.  Split
// so that neither kernel holds the correction and the network at once.
template <int D, bool L>
__global__ void __launch_bounds__(kBlock) k_ctu_correct_dir(Work w, const float* __restrict__ QL,
                                                            const float* __restrict__ QR, const float* __restrict__ F1,
                                                            const float* __restrict__ E1, const float* __restrict__ B,
                                                            float* __restrict__ Qc, DtSrc dts, float inv_dx,
                                                            float gam) {
  const float hr = float(0.5 * get_dt(dts)) * inv_dx;
  const long long NS = w.NS;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    float wl[7], wr[7];
    corrected_states<float, D, L>(w, QL, QR, F1, E1, B, st, hr, gam, wl, wr);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      Qc[(long long)m * NS + st.s] = wl[m];
      Qc[(long long)(7 + m) * NS + st.s] = wr[m];
    }
  }
}

// Learned flux (HLLD at strong jumps) of the D-faces from scratch states
// QLd[m * NS + s], QRd[m * NS + s] (m = 0..6) and the normal field: the level's
// B[D * N + p] (predictor) or the half-step scratch Bh[D * NS + s] (BN_SCRATCH).
template <int D, bool BN_SCRATCH, bool L>
__global__ void __launch_bounds__(kBlock) k_flux_dir_mlp(Work w, const float* __restrict__ QLd,
                                                         const float* __restrict__ QRd, const float* __restrict__ Bn,
                                                         float* __restrict__ F, float gam, const MlpWeights* mw,
                                                         float dp, float drho, unsigned long long* nfb) {
  __shared__ MlpShared sh;
  mlp_load_weights(sh, mw);
  const long long N = w.N, NS = w.NS;
  const long long nitems = work_items(w);
  int fb = 0;
  // block-uniform trips: every lane of a wave takes part in the network
  for (long long base = block_linear_id() - threadIdx.x; base < nitems; base += item_stride()) {
    const long long t = base + threadIdx.x;
    const bool active = t < nitems;
    long long p = 0, s = 0;
    if (active) {
      const Site st = site_of<L>(w, t);
      p = st.p;
      s = st.s;
    }
    float wl[7], wr[7], f[7];
    float bn = 1.0f;
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      wl[m] = active ? QLd[(long long)m * NS + s] : 1.0f;
      wr[m] = active ? QRd[(long long)m * NS + s] : 1.0f;
    }
    if (active) bn = BN_SCRATCH ? Bn[D * NS + s] : Bn[D * N + p];
    fb += mlp_or_hlld(sh, active, wl, wr, bn, gam, dp, drho, f);
    if (active) store_flux<float, D>(F, NS, s, f);
  }
  block_count_atomic(fb, nfb);
}

// group occupancy map of a list: clear, then mark
__global__ void __launch_bounds__(kBlock) k_occ_clear(int* occ, long long n) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) occ[t] = 0;
}

__global__ void __launch_bounds__(kBlock) k_occ_set(int* occ, const int* groups, int n_groups, const int* n_dev,
                                                    int edge, int gnx, int gny) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int n = n_dev ? min(*n_dev, n_groups) : n_groups;
  if (g >= n) return;
  const int gi = groups[3 * g] / edge, gj = groups[3 * g + 1] / edge, gk = groups[3 * g + 2] / edge;
  occ[((long long)gk * gny + gj) * gnx + gi] = g + 1;   // 0: not listed, else group index + 1
}

// ------------------------------------------------------------ AMR support
__device__ __forceinline__ int wrap_delta(int d, int n) { return d > n / 2 ? d - n : (d < -(n / 2) ? d + n : d); }

// Prolongation from a coarse level (nc) to a fine level (2 nc), paper
// Sec. 3.3 (refinement operation).  Cell data: density and momentum are
// injected; the energy is shared out so that the children keep a common
// pressure and average to the parent (conservative, see prolong_parent).
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

// The eight children of coarse cell (i, j, k): conservative cell data and
// their lower faces, where allowed.  cell_ok[q] / face_ok[q][A] say which
// child q = a + 2 b + 4 c (position (a, b, c) in the parent) and which of its
// lower faces may be written.  The children's energies are
// e_parent + (|b_child|^2 - <|b|^2>)/2 (they average to the parent's); where
// the resulting common pressure would not be positive the parent's pressure
// is kept instead.
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
  const long long pc = lin(wc, i, j, k);
  const T cbx = T(0.5) * (P.v[0][0] + P.v[0][1]);
  const T cby = T(0.5) * (P.v[1][0] + P.v[1][1]);
  const T cbz = T(0.5) * (P.v[2][0] + P.v[2][1]);
  const T b2c = cbx * cbx + cby * cby + cbz * cbz;
  const T d = Uc[pc], mx = Uc[wc.N + pc], my = Uc[2 * wc.N + pc], mz = Uc[3 * wc.N + pc], e = Uc[4 * wc.N + pc];
  const T ek = T(0.5) * (mx * mx + my * my + mz * mz) / d;
  const T pr = (gam - T(1)) * (e - ek - T(0.5) * b2c);
  const bool conservative = pr - (gam - T(1)) * T(0.5) * (mean_b2 - b2c) > T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const long long pf = lin(wf, 2 * i + a, 2 * j + b, 2 * k + c);
    if (cell_ok[q]) {
      Uf[pf] = d;
      Uf[wf.N + pf] = mx;
      Uf[2 * wf.N + pf] = my;
      Uf[3 * wf.N + pf] = mz;
      Uf[4 * wf.N + pf] = conservative ? e + T(0.5) * (b2[q] - mean_b2) : pr / (gam - T(1)) + ek + T(0.5) * b2[q];
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
      const int dx = wrap_delta(x - o[0], wf.nx), dy = wrap_delta(y - o[1], wf.ny), dz = wrap_delta(z - o[2], wf.nz);
      const int blo = -wf.halo, bhi = wf.edge + wf.halo + 1;
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
  const int a = wrap_delta(i - o[0], v.nx) + v.ghost, b = wrap_delta(j - o[1], v.ny) + v.ghost,
            c = wrap_delta(k - o[2], v.nz) + v.ghost;
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
  const T cbx = T(0.5) * (B0[pc] + B0[nbr(wc, i, j, k, 1, 0, 0)]);
  const T cby = T(0.5) * (B1[pc] + B1[nbr(wc, i, j, k, 0, 1, 0)]);
  const T cbz = T(0.5) * (B2[pc] + B2[nbr(wc, i, j, k, 0, 0, 1)]);
  const T b2c = cbx * cbx + cby * cby + cbz * cbz;
  const T d = Uc[pc], mx = Uc[wc.N + pc], my = Uc[2 * wc.N + pc], mz = Uc[3 * wc.N + pc], e = Uc[4 * wc.N + pc];
  const T ek = T(0.5) * (mx * mx + my * my + mz * mz) / d;
  const T pr = (gam - T(1)) * (e - ek - T(0.5) * b2c);
  const bool conservative = pr - (gam - T(1)) * T(0.5) * (mean_b2 - b2c) > T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
    const long long pf = lin(wf, 2 * i + a, 2 * j + b, 2 * k + c);
    Uf[pf] = d;
    Uf[wf.N + pf] = mx;
    Uf[2 * wf.N + pf] = my;
    Uf[3 * wf.N + pf] = mz;
    Uf[4 * wf.N + pf] = conservative ? e + T(0.5) * (b2[q] - mean_b2) : pr / (gam - T(1)) + ek + T(0.5) * b2[q];
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
// (sb = 0): every slot; group list: the slots of each group's cells and of
// its upper boundary faces and edges (box positions ghost .. ghost + edge).
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

// ------------------------------------------------------------ set-up
template <typename T, bool MIX>
__global__ void __launch_bounds__(kBlock) k_prim_to_cons(Work w, const T* __restrict__ W5, const T* __restrict__ B,
                                                         T* __restrict__ U, Mix mix, T gam) {
  FOR_ITEMS(w, t) {
  int i, j, k;
  cell_of(w, t, i, j, k);
  const long long N = w.N;
  const long long p = lin(w, i, j, k);
  const T bx = T(0.5) * (B[p] + B[nbr(w, i, j, k, 1, 0, 0)]);
  const T by = T(0.5) * (B[N + p] + B[N + nbr(w, i, j, k, 0, 1, 0)]);
  const T bz = T(0.5) * (B[2 * N + p] + B[2 * N + nbr(w, i, j, k, 0, 0, 1)]);
  const T d = W5[p], vx = W5[N + p], vy = W5[2 * N + p], vz = W5[3 * N + p], pr = W5[4 * N + p];
  U[p] = d;
  U[N + p] = d * vx;
  U[2 * N + p] = d * vy;
  U[3 * N + p] = d * vz;
  if (MIX) {
    const double e = (double)pr / ((double)gam - 1.0) +
                     0.5 * (double)d * ((double)vx * vx + (double)vy * vy + (double)vz * vz) +
                     0.5 * ((double)bx * bx + (double)by * by + (double)bz * bz);
    mix.E64[p] = e;
    U[4 * N + p] = T(e);
  } else {
    U[4 * N + p] = pr / (gam - T(1)) + T(0.5) * d * (vx * vx + vy * vy + vz * vz) + T(0.5) * (bx * bx + by * by + bz * bz);
  }
  }
}

// ------------------------------------------------------------ diagnostics
// Two-pass deterministic reductions: fixed per-block trees write partials,
// one block combines them in index order.
template <int NQ>
__device__ __forceinline__ void block_partials(double v[NQ], double* part, int stride) {
  __shared__ double red[NQ][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = wave_sum(v[q]);
    if (lane == 0) red[q][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = red[q][0];
      for (int m = 1; m < kBlock / 64; ++m) s += red[q][m];
      part[(long long)q * stride + blockIdx.x] = s;
    }
  }
}

// discrete divergence (Eq. 16): partial sums of |div B| and partial maxima
template <typename T>
__global__ void __launch_bounds__(kBlock) k_divb(Work w, const T* __restrict__ B, double inv_dx, double* part) {
  double a = 0.0, amax = 0.0;
  FOR_ITEMS(w, t) {
    int i, j, k;
    cell_of(w, t, i, j, k);
    const long long N = w.N;
    const long long p = lin(w, i, j, k);
    const double dv = ((double)B[nbr(w, i, j, k, 1, 0, 0)] - (double)B[p]) * inv_dx +
                      ((double)B[N + nbr(w, i, j, k, 0, 1, 0)] - (double)B[N + p]) * inv_dx +
                      ((double)B[2 * N + nbr(w, i, j, k, 0, 0, 1)] - (double)B[2 * N + p]) * inv_dx;
    a += fabs(dv);
    amax = fmax(amax, fabs(dv));
  }
  __shared__ double mx[kBlock / 64];
  const double wm = wave_max(amax);
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = wm;
  double v[1] = {a};
  block_partials<1>(v, part, gridDim.x);
  if (threadIdx.x == 0) {
    double m = mx[0];
    for (int q = 1; q < kBlock / 64; ++q) m = fmax(m, mx[q]);
    part[(long long)gridDim.x + blockIdx.x] = m;
  }
}

// volume totals: mass, Mx, My, Mz, e, magnetic energy, kinetic energy
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sums(Work w, const T* __restrict__ U, const T* __restrict__ B,
                                                 const double* __restrict__ E64, double* part) {
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  FOR_ITEMS(w, t) {
    int i, j, k;
    cell_of(w, t, i, j, k);
    const long long N = w.N;
    const long long p = lin(w, i, j, k);
    double u[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) u[m] = (double)U[m * N + p];
    if (E64) u[4] = E64[p];
#pragma unroll
    for (int m = 0; m < 5; ++m) v[m] += u[m];
    const double bx = 0.5 * ((double)B[p] + (double)B[nbr(w, i, j, k, 1, 0, 0)]);
    const double by = 0.5 * ((double)B[N + p] + (double)B[N + nbr(w, i, j, k, 0, 1, 0)]);
    const double bz = 0.5 * ((double)B[2 * N + p] + (double)B[2 * N + nbr(w, i, j, k, 0, 0, 1)]);
    v[5] += 0.5 * (bx * bx + by * by + bz * bz);
    v[6] += 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
  }
  block_partials<7>(v, part, gridDim.x);
}

// combine nq rows of nb partials (sum for rows < nsum, max otherwise)
__global__ void __launch_bounds__(kBlock) k_finish(const double* part, int nb, int nq, int nsum, double* out) {
  __shared__ double red[kBlock];
  for (int q = 0; q < nq; ++q) {
    const bool is_max = q >= nsum;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
      const double x = part[(long long)q * nb + b];
      acc = is_max ? fmax(acc, x) : acc + x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] = is_max ? fmax(red[threadIdx.x], red[threadIdx.x + s])
                                                     : red[threadIdx.x] + red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
    __syncthreads();
  }
}

}  // namespace mhd
