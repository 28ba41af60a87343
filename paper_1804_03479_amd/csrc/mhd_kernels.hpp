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

constexpr int kBlock = 256;      // threads per block of the fixed-shape kernels
constexpr int kMaxBlock = 512;   // largest block of the step's stage kernels (tuned per context)

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
  int gbase;            // list mode: first group of this launch (a batch of the list)
  int gcount;           // list mode: groups of this launch at most
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

__device__ __forceinline__ long long block_linear_id() { return (long long)block_rank() * blockDim.x + threadIdx.x; }

// Persistent launches: a grid of at most a tuned number of blocks walks the
// work items with a grid-wide stride; the item count of a group list may be
// read from device memory, so a captured graph replays over a changed list.
__device__ __forceinline__ long long work_items(const Work& w) {
  if (w.n_dev) {
    long long n = (long long)*w.n_dev - w.gbase;
    n = n < 0 ? 0 : (n > w.gcount ? w.gcount : n);
    const long long m = (long long)w.box * w.box * w.box * n;
    return m < w.items ? m : w.items;
  }
  return w.items;
}
__device__ __forceinline__ long long item_stride() { return (long long)gridDim.x * blockDim.x; }

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
    const int* o = w.groups + 3LL * (w.gbase + g);
    i = wrapc((o[0] >> w.oshift) - w.halo + a, w.nx);
    j = wrapc((o[1] >> w.oshift) - w.halo + b, w.ny);
    k = wrapc((o[2] >> w.oshift) - w.halo + c, w.nz);
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
    const long long g = t / per + w.gbase;
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
  __shared__ double red[kMaxBlock / 64];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
    // most blocks see a maximum already reached: skip their atomic
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    if (m > 0.0 && bits > *(volatile unsigned long long*)smax) atomicMax(smax, bits);
  }
}

// Primitive state of every cell; optionally the CFL maximum signal speed and
// the sticky non-physical flag.
template <typename T, bool CFL, bool MIX, bool L>
__global__ void __launch_bounds__(kMaxBlock) k_prim(Work w, const T* __restrict__ U, const T* __restrict__ B, Mix mix,
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

// RECON: 0 = first order (cell states), 1 = PLM with minmod on primitives,
// 2 = PPM (the limited parabolas' upper edge of the left cell and lower edge
// of the right cell, no tracing: the VL predictor centres the data in time).
// The normal field Bn is the level's B (predictor, RECON 0: Bn[D N + p]) or
// the half-step scratch Bh (corrector, RECON 1 and 2: Bn[D NS + s]).
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
  } else if (RECON == 2) {
    // cells -3, -2 and 1, 2 around the face (-1 and 0 are wl, wr)
    T q3[7], q2[7], p1[7], p2[7];
    load_w1d<T, D>(W, NS, snb<L>(w, st, D == 0 ? -3 : 0, D == 1 ? -3 : 0, D == 2 ? -3 : 0), q3);
    load_w1d<T, D>(W, NS, snb<L>(w, st, D == 0 ? -2 : 0, D == 1 ? -2 : 0, D == 2 ? -2 : 0), q2);
    load_w1d<T, D>(W, NS, snb<L>(w, st, D == 0 ? 1 : 0, D == 1 ? 1 : 0, D == 2 ? 1 : 0), p1);
    load_w1d<T, D>(W, NS, snb<L>(w, st, D == 0 ? 2 : 0, D == 1 ? 2 : 0, D == 2 ? 2 : 0), p2);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      T lo, hi, lo2, hi2;
      ppm_edges(q3[m], q2[m], wl[m], wr[m], p1[m], lo, hi);     // cell -1
      ppm_edges(q2[m], wl[m], wr[m], p1[m], p2[m], lo2, hi2);   // cell 0
      wl[m] = hi;
      wr[m] = lo2;
    }
  }
  const T bn = RECON != 0 ? Bn[D * NS + st.s] : Bn[D * w.N + st.p];
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
  __shared__ int red[kMaxBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
    if (s) atomicAdd(counter, (unsigned long long)s);
  }
}

// VL flux stage; B is the level's field for RECON 0 and the half-step
// scratch Bh for RECON 1 and 2 (see face_flux).
template <typename T, int RECON, int SOLVER, bool L>
__global__ void __launch_bounds__(kMaxBlock) k_flux(Work w, const T* __restrict__ W, const T* __restrict__ B,
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

// The upwind CT average of one edge from its four face EMFs (eb0, eb1 on the
// b-faces below and at the cell, ec0, ec1 on the c-faces), the faces' mass
// fluxes (mb*, mc*) and the reference EMFs of the four cells around the edge
// (r00 at the cell below in b and c, r10 below in c, r01 below in b, r11 the
// cell itself)
template <typename T>
__device__ __forceinline__ T edge_emf_core(T eb0, T eb1, T ec0, T ec1, T mb0, T mb1, T mc0, T mc1, T r00, T r10,
                                           T r01, T r11) {
  const T dc1 = upwind(mb1, r01 - ec0, r11 - ec1);
  const T dc0 = upwind(mb0, ec0 - r00, ec1 - r10);
  const T db1 = upwind(mc1, r10 - eb0, r11 - eb1);
  const T db0 = upwind(mc0, eb0 - r00, eb1 - r01);
  return T(0.25) * (eb0 + eb1 + ec0 + ec1) + T(0.25) * ((dc0 - dc1) + (db0 - db1));
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
  return edge_emf_core(eb0, eb1, ec0, ec1, mb0, mb1, mc0, mc1, r00, r10, r01, r11);
}

template <typename T, bool L>
__global__ void __launch_bounds__(kMaxBlock) k_emf(Work w, const T* __restrict__ F, const T* __restrict__ W,
                                                T* __restrict__ E) {
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    E[st.s] = edge_emf<T, 0, L>(w, F, W, st);
    E[w.NS + st.s] = edge_emf<T, 1, L>(w, F, W, st);
    E[2 * w.NS + st.s] = edge_emf<T, 2, L>(w, F, W, st);
  }
}

// Edge EMFs of a whole grid on LDS tiles: each block stages, for its
// TX x TY x TZ cells and the layer below them along every direction, the
// cells' reference EMFs -v x B (three components) and, per face direction,
// the face's mass flux and its two EMF components (twelve values per cell,
// each loaded once per tile instead of once per edge that uses it), then
// computes the three lower-corner edges of each of its cells from LDS with
// the arithmetic of k_emf.  Grids need not be multiples of the tile (cells
// past the grid idle; the staged layer wraps periodically).
template <typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ) k_emf_tiled(Work w, const T* __restrict__ F, const T* __restrict__ W,
                                                         T* __restrict__ E) {
  constexpr int HX = TX + 1, HY = TY + 1, HZ = TZ + 1, NH = HX * HY * HZ, NT = TX * TY * TZ;
  __shared__ T sR[3][NH];
  __shared__ T sF[3][3][NH];
  const int ntx = (w.nx + TX - 1) / TX, nty = (w.ny + TY - 1) / TY;
  const int tile = (int)block_rank();
  const int tx0 = (tile % ntx) * TX, ty0 = ((tile / ntx) % nty) * TY, tz0 = (tile / (ntx * nty)) * TZ;
  const long long N = w.NS;
  for (int h = threadIdx.x; h < NH; h += NT) {
    const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
    const long long q = lin(w, wrapc(tx0 - 1 + hx, w.nx), wrapc(ty0 - 1 + hy, w.ny), wrapc(tz0 - 1 + hz, w.nz));
#pragma unroll
    for (int a = 0; a < 3; ++a) sR[a][h] = ref_emf(W, N, q, a);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sF[d][0][h] = F[(long long)(7 * d) * N + q];
      sF[d][1][h] = F[(long long)(7 * d + 5) * N + q];
      sF[d][2][h] = F[(long long)(7 * d + 6) * N + q];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int ax = t % TX, ay = (t / TX) % TY, az = t / (TX * TY);
  const int i = tx0 + ax, j = ty0 + ay, k = tz0 + az;
  if (i >= w.nx || j >= w.ny || k >= w.nz) return;
  const int h = ((az + 1) * HY + (ay + 1)) * HX + (ax + 1);
  const long long p = lin(w, i, j, k);
  constexpr int st[3] = {1, HX, HX * HY};
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    const int b = (A + 1) % 3, c = (A + 2) % 3;
    const int hb = h - st[b], hc = h - st[c], hbc = h - st[b] - st[c];
    E[(long long)A * N + p] = edge_emf_core(sF[b][2][hc], sF[b][2][h], sF[c][1][hb], sF[c][1][h], sF[b][0][hc],
                                            sF[b][0][h], sF[c][0][hb], sF[c][0][h], sR[A][hbc], sR[A][hc],
                                            sR[A][hb], sR[A][h]);
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
__global__ void __launch_bounds__(kMaxBlock) k_half(Work w, const T* __restrict__ U, const T* __restrict__ B, Mix mix,
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
__global__ void __launch_bounds__(kMaxBlock) k_final(Work w, T* __restrict__ U, T* __restrict__ B, Mix mix,
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
template <typename T, int D, int RECON, bool ALLW, bool L>
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
  trace_cell<T, RECON, ALLW>(q, B[D * N + st.p], B[D * N + pu], dtdx, gam, sl, sr);
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    QR[((long long)D * 7 + m) * NS + st.s] = sl[m];
    QL[((long long)D * 7 + m) * NS + su] = sr[m];
  }
}

// ALLW: trace waves moving away from an edge too (HLL-family solvers)
template <typename T, int RECON, bool ALLW, bool L>
__global__ void __launch_bounds__(kMaxBlock) k_ctu_states(Work w, const T* __restrict__ W, const T* __restrict__ B,
                                                       T* __restrict__ QL, T* __restrict__ QR, DtSrc dts,
                                                       T inv_dx, T gam) {
  const T dtdx = T(get_dt(dts)) * inv_dx;
  FOR_ITEMS(w, t) {
    const Site st = site_of<L>(w, t);
    cell_states<T, 0, RECON, ALLW, L>(w, W, B, QL, QR, st, dtdx, gam);
    cell_states<T, 1, RECON, ALLW, L>(w, W, B, QL, QR, st, dtdx, gam);
    cell_states<T, 2, RECON, ALLW, L>(w, W, B, QL, QR, st, dtdx, gam);
  }
}

// ---- step 1 with PPM, tiled in LDS
//
// A block owns a TX x TY x TZ tile of a unit (the whole grid, or the item
// box of one listed group).  Per direction D it stages the tile's 1D
// primitives with two more cells on each side along D in LDS, computes each
// MC slope of the padded tile and each PPM interface value of the tile's
// faces once (the per-cell form computes every slope three times and every
// interface twice), and then each thread limits and traces its own cell from
// the shared values.  Every value is computed with the per-cell form's
// arithmetic, so the states are the same.

// scratch slot of position (a, b, c) of unit gg (a group's item box in list
// mode, the grid otherwise); positions up to two cells outside the unit
template <bool L>
__device__ __forceinline__ long long unit_slot(const Work& w, long long gg, int a, int b, int c) {
  if constexpr (L) {
    const long long sb = w.sb;
    return (gg + 1) * sb * sb * sb + ((long long)(c + w.soff) * sb + (b + w.soff)) * sb + (a + w.soff);
  } else {
    return lin(w, wrapc(a, w.nx), wrapc(b, w.ny), wrapc(c, w.nz));
  }
}

// the site of position (a, b, c) inside unit gg
template <bool L>
__device__ __forceinline__ Site unit_site(const Work& w, long long gg, int a, int b, int c) {
  Site st;
  st.a = a; st.b = b; st.c = c;
  if constexpr (L) {
    const int* o = w.groups + 3 * gg;
    st.i = wrapc((o[0] >> w.oshift) - w.halo + a, w.nx);
    st.j = wrapc((o[1] >> w.oshift) - w.halo + b, w.ny);
    st.k = wrapc((o[2] >> w.oshift) - w.halo + c, w.nz);
  } else {
    st.i = a; st.j = b; st.k = c;
  }
  st.p = lin(w, st.i, st.j, st.k);
  st.s = L ? unit_slot<L>(w, gg, a, b, c) : st.p;
  return st;
}

// extents of the tile padded by P cells on each side along D
template <int TX, int TY, int TZ, int D, int P>
struct Padded {
  static constexpr int x = TX + (D == 0 ? 2 * P : 0);
  static constexpr int y = TY + (D == 1 ? 2 * P : 0);
  static constexpr int z = TZ + (D == 2 ? 2 * P : 0);
  static constexpr int n = x * y * z;
  static constexpr int stride = D == 0 ? 1 : (D == 1 ? x : x * y);   // index step along D
};

template <int TX, int TY, int TZ, int P>
constexpr int padded_max() {
  return Padded<TX, TY, TZ, 0, P>::n > Padded<TX, TY, TZ, 1, P>::n
             ? (Padded<TX, TY, TZ, 0, P>::n > Padded<TX, TY, TZ, 2, P>::n ? Padded<TX, TY, TZ, 0, P>::n
                                                                          : Padded<TX, TY, TZ, 2, P>::n)
             : (Padded<TX, TY, TZ, 1, P>::n > Padded<TX, TY, TZ, 2, P>::n ? Padded<TX, TY, TZ, 1, P>::n
                                                                          : Padded<TX, TY, TZ, 2, P>::n);
}

// faces of the tile along its largest direction count
template <int TX, int TY, int TZ>
constexpr int faces_max() {
  return (TX + 1) * TY * TZ > TX * (TY + 1) * TZ
             ? ((TX + 1) * TY * TZ > TX * TY * (TZ + 1) ? (TX + 1) * TY * TZ : TX * TY * (TZ + 1))
             : (TX * (TY + 1) * TZ > TX * TY * (TZ + 1) ? TX * (TY + 1) * TZ : TX * TY * (TZ + 1));
}

// A tile: its unit, its origin in the unit and the unit's extents.
struct Tile {
  long long gg;
  int a0, b0, c0;
  int ux, uy, uz;
};

// LDS arrays of one direction D (component-major, [7][n] each): sW the
// primitives at positions -2 .. T+1 along D (padding 2), sS the MC slopes at
// -1 .. T (padding 1), sE the interface values at faces 0 .. T (face f
// between cells f - 1 and f).
template <int TX, int TY, int TZ, int D>
struct TileLayout {
  using PW = Padded<TX, TY, TZ, D, 2>;
  using PS = Padded<TX, TY, TZ, D, 1>;
  static constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2), NF = FX * FY * FZ;
  static constexpr int SF = D == 0 ? 1 : (D == 1 ? FX : FX * FY);
  static constexpr int NT = TX * TY * TZ;
  static constexpr int dx = D == 0, dy = D == 1, dz = D == 2;
};

// padded cell e of direction D: inside the loaded range (within two cells of
// the unit along D, inside it across)?  Also returns its unit position.
template <int TX, int TY, int TZ, int D>
__device__ __forceinline__ bool padded_cell(const Tile& t, int e, int& a, int& b, int& c) {
  using Ly = TileLayout<TX, TY, TZ, D>;
  using PW = typename Ly::PW;
  const int x = e % PW::x, y = (e / PW::x) % PW::y, z = e / (PW::x * PW::y);
  a = t.a0 + x - 2 * Ly::dx;
  b = t.b0 + y - 2 * Ly::dy;
  c = t.c0 + z - 2 * Ly::dz;
  return a < t.ux + 2 * Ly::dx && b < t.uy + 2 * Ly::dy && c < t.uz + 2 * Ly::dz;
}

// the padded primitives of direction D into sW
template <typename T, bool L, int TX, int TY, int TZ, int D>
__device__ __forceinline__ void stage_prims(const Work& w, const T* __restrict__ W, const Tile& t, int tid, T* sW) {
  using Ly = TileLayout<TX, TY, TZ, D>;
  for (int e = tid; e < Ly::PW::n; e += Ly::NT) {
    int a, b, c;
    if (padded_cell<TX, TY, TZ, D>(t, e, a, b, c)) {
      T q[7];
      load_w1d<T, D>(W, w.NS, unit_slot<L>(w, t.gg, a, b, c), q);
#pragma unroll
      for (int m = 0; m < 7; ++m) sW[m * Ly::PW::n + e] = q[m];
    }
  }
}

// slopes and interface values of direction D from the staged primitives
// (two block barriers)
template <typename T, int TX, int TY, int TZ, int D>
__device__ __forceinline__ void tile_interfaces(int tid, const T* sW, T* sS, T* sE) {
  using Ly = TileLayout<TX, TY, TZ, D>;
  using PW = typename Ly::PW;
  using PS = typename Ly::PS;
  constexpr int dx = Ly::dx, dy = Ly::dy, dz = Ly::dz;
  // slopes: position -1 + s along D at padded index s; its cell sits one
  // further in the primitives' padding
  for (int e = tid; e < PS::n; e += Ly::NT) {
    const int x = e % PS::x, y = (e / PS::x) % PS::y, z = e / (PS::x * PS::y);
    const int iw = (x + dx) + PW::x * ((y + dy) + PW::y * (z + dz));
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const T* q = sW + m * PW::n + iw;
      sS[m * PS::n + e] = mc_slope(q[-PW::stride], q[0], q[PW::stride]);
    }
  }
  __syncthreads();
  // interface values: face f between cell f - 1 (primitive index f + 1,
  // slope index f along D) and cell f
  for (int e = tid; e < Ly::NF; e += Ly::NT) {
    const int x = e % Ly::FX, y = (e / Ly::FX) % Ly::FY, z = e / (Ly::FX * Ly::FY);
    const int iw = (x + dx) + PW::x * ((y + dy) + PW::y * (z + dz));
    const int is = x + PS::x * (y + PS::y * z);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const T* q = sW + m * PW::n + iw;
      const T* sl = sS + m * PS::n + is;
      sE[m * Ly::NF + e] = ppm_interface(q[0], q[PW::stride], sl[0], sl[PS::stride]);
    }
  }
  __syncthreads();
}

// each thread's own cell: limit its parabola, trace, store the two states
template <typename T, bool ALLW, bool L, int TX, int TY, int TZ, int D>
__device__ __forceinline__ void tile_trace(const Work& w, const T* __restrict__ B, T* __restrict__ QL,
                                           T* __restrict__ QR, const Tile& t, int tid, T dtdx, T gam,
                                           const T* sW, const T* sE) {
  using Ly = TileLayout<TX, TY, TZ, D>;
  using PW = typename Ly::PW;
  constexpr int dx = Ly::dx, dy = Ly::dy, dz = Ly::dz;
  const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
  const int a = t.a0 + lx, b = t.b0 + ly, c = t.c0 + lz;
  if (a < t.ux && b < t.uy && c < t.uz) {
    const int iw = (lx + 2 * dx) + PW::x * ((ly + 2 * dy) + PW::y * (lz + 2 * dz));
    const int ie = lx + Ly::FX * (ly + Ly::FY * lz);
    T q[7], sl[7], sr[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      q[m] = sW[m * PW::n + iw];
      sl[m] = sE[m * Ly::NF + ie];
      sr[m] = sE[m * Ly::NF + ie + Ly::SF];
      ppm_limit(q[m], sl[m], sr[m]);
    }
    const Site st = unit_site<L>(w, t.gg, a, b, c);
    const long long N = w.N, NS = w.NS;
    const long long pu = nbr(w, st.i, st.j, st.k, dx, dy, dz);
    const long long su = snb<L>(w, st, dx, dy, dz);
    trace_edges<T, ALLW>(q, B[D * N + st.p], B[D * N + pu], dtdx, gam, sl, sr);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      QR[((long long)D * 7 + m) * NS + st.s] = sl[m];
      QL[((long long)D * 7 + m) * NS + su] = sr[m];
    }
  }
}

// tiles of one unit
template <int TX, int TY, int TZ>
__host__ __device__ __forceinline__ long long unit_tiles(int ux, int uy, int uz) {
  return (long long)((ux + TX - 1) / TX) * ((uy + TY - 1) / TY) * ((uz + TZ - 1) / TZ);
}

// one direction of a tile: stage, slopes and interfaces, trace (four block
// barriers; the last one frees the arrays for the next direction)
template <typename T, bool ALLW, bool L, int TX, int TY, int TZ, int D>
__device__ __forceinline__ void tile_direction(const Work& w, const T* __restrict__ W, const T* __restrict__ B,
                                               T* __restrict__ QL, T* __restrict__ QR, const Tile& t, int tid, T dtdx,
                                               T gam, T* sW, T* sS, T* sE) {
  stage_prims<T, L, TX, TY, TZ, D>(w, W, t, tid, sW);
  __syncthreads();
  tile_interfaces<T, TX, TY, TZ, D>(tid, sW, sS, sE);
  tile_trace<T, ALLW, L, TX, TY, TZ, D>(w, B, QL, QR, t, tid, dtdx, gam, sW, sE);
  __syncthreads();
}

// One block per tile of TX * TY * TZ cells (one thread per cell), walking
// the tiles with a grid-wide stride.
template <typename T, bool ALLW, bool L, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ) k_ctu_states_tiled(Work w, const T* __restrict__ W,
                                                                     const T* __restrict__ B, T* __restrict__ QL,
                                                                     T* __restrict__ QR, DtSrc dts, T inv_dx,
                                                                     T gam) {
  constexpr int kW = padded_max<TX, TY, TZ, 2>(), kS = padded_max<TX, TY, TZ, 1>();
  constexpr int kE = faces_max<TX, TY, TZ>();
  __shared__ T smem[7 * (kW + kS + kE)];
  T* sW = smem;
  T* sS = smem + 7 * kW;
  T* sE = smem + 7 * (kW + kS);
  const int tid = (int)threadIdx.x;
  const T dtdx = T(get_dt(dts)) * inv_dx;
  const int ux = L ? w.box : w.nx, uy = L ? w.box : w.ny, uz = L ? w.box : w.nz;
  const int tx = (ux + TX - 1) / TX, ty = (uy + TY - 1) / TY;
  const long long per = unit_tiles<TX, TY, TZ>(ux, uy, uz);
  const long long units = L ? work_items(w) / ((long long)w.box * w.box * w.box) : 1;
  const long long ntiles = units * per;
  for (long long id = block_rank(); id < ntiles; id += gridDim.x) {   // uniform over the block
    Tile t;
    const long long g = id / per;
    const int r = (int)(id - g * per);
    t.a0 = (r % tx) * TX;
    t.b0 = ((r / tx) % ty) * TY;
    t.c0 = (r / (tx * ty)) * TZ;
    t.gg = L ? w.gbase + g : 0;
    t.ux = ux; t.uy = uy; t.uz = uz;
    tile_direction<T, ALLW, L, TX, TY, TZ, 0>(w, W, B, QL, QR, t, tid, dtdx, gam, sW, sS, sE);
    tile_direction<T, ALLW, L, TX, TY, TZ, 1>(w, W, B, QL, QR, t, tid, dtdx, gam, sW, sS, sE);
    tile_direction<T, ALLW, L, TX, TY, TZ, 2>(w, W, B, QL, QR, t, tid, dtdx, gam, sW, sS, sE);
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
__global__ void __launch_bounds__(kMaxBlock) k_flux_q(Work w, const T* __restrict__ QL, const T* __restrict__ QR,
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
// cell (ci, cj, ck) and sits on a face with normal field bn at time n and bnh
// after the half step.  Hydro variables: minus dt/2 times the transverse flux
// differences of step 2 in that cell.  Transverse field: dt/2 times the
// transverse part of -curl E with the step-3 edge EMFs E_D averaged to the
// cell's faces.  The state enters conserved form with bn and leaves it with
// bnh (the transverse energy fluxes carry the normal field's change of
// magnetic energy).  The conserved transverse flux differences hold the
// div B terms of their directions, dBn/dn (0, B, v.B, v): momentum and
// energy get (dt/2)(B, v.B) dBn/dn with dbn the source cell's normal-field
// difference (the field's share is in the traced state).  Non-physical
// results keep the input.
template <typename T, int D, bool L>
__device__ __forceinline__ void correct_state(const Work& w, const T* __restrict__ F1, const T* __restrict__ E1,
                                              const Site& src, T bn, T bnh, T dbn, T hr, T gam, const T s[7],
                                              T out[7]) {
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
  const T vb = v[0] * b[0] + v[1] * b[1] + v[2] * b[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) u[1 + a] += hr * dbn * b[a];
  u[4] += hr * dbn * vb;
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
  b[D] = bnh;
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
                                                 const T* __restrict__ B, T bnh, const Site& st, T hr, T gam,
                                                 T wl[7], T wr[7]) {
  const long long NS = w.NS;
  T sl[7], sr[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    sl[m] = QL[((long long)D * 7 + m) * NS + st.s];
    sr[m] = QR[((long long)D * 7 + m) * NS + st.s];
  }
  const T bn = B[D * w.N + st.p];
  const T bn_lo = B[D * w.N + nbr(w, st.i, st.j, st.k, -(D == 0), -(D == 1), -(D == 2))];
  const T bn_hi = B[D * w.N + nbr(w, st.i, st.j, st.k, D == 0, D == 1, D == 2)];
  correct_state<T, D, L>(w, F1, E1, site_nb<L>(w, st, -(D == 0), -(D == 1), -(D == 2)), bn, bnh, bn - bn_lo, hr,
                         gam, sl, wl);
  correct_state<T, D, L>(w, F1, E1, st, bn, bnh, bn_hi - bn, hr, gam, sr, wr);
}

template <typename T, int D, int SOLVER, bool L>
__device__ __forceinline__ int corrected_face_flux(const Work& w, const T* __restrict__ QL, const T* __restrict__ QR,
                                                   const T* __restrict__ F1, const T* __restrict__ E1,
                                                   const T* __restrict__ B, const T* __restrict__ Bh,
                                                   T* __restrict__ F2, const Site& st, T hr, T gam,
                                                   const Capture& cp) {
  const long long NS = w.NS;
  T wl[7], wr[7], f[7];
  const T bn = Bh[D * NS + st.s];
  corrected_states<T, D, L>(w, QL, QR, F1, E1, B, bn, st, hr, gam, wl, wr);
  const int fb = riemann<SOLVER>(wl, wr, bn, gam, f);
  if constexpr (sizeof(T) == 4) capture_face(cp, 3 * st.p + D, wl, wr, bn, f);
  store_flux<T, D>(F2, NS, st.s, f);
  return fb;
}

// Steps 5-6: corrected states and Riemann fluxes with the half-step normal field
template <typename T, int SOLVER, bool L>
__global__ void __launch_bounds__(kMaxBlock) k_ctu_correct(Work w, const T* __restrict__ QL, const T* __restrict__ QR,
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

// Learned flux (HLLD at strong jumps) of the D-faces in step 2 from the
// traced states QLd[m * NS + s], QRd[m * NS + s] (m = 0..6) and the level's
// time-n normal field B[D * N + p].  With capture on, the face's states and
// the flux it used are recorded.  Held to 128 VGPRs (four waves per SIMD,
// a few spilled words): the network's dependent MFMA and transcendental
// chains need the extra waves to hide their latency (12 % faster than
// three waves at 135 VGPRs without spills).
template <int D, bool L>
__global__ void __launch_bounds__(kBlock, 4) k_flux_dir_mlp(Work w, const float* __restrict__ QLd,
                                                         const float* __restrict__ QRd, const float* __restrict__ Bn,
                                                         float* __restrict__ F, float gam, const MlpWeights* mw,
                                                         float dp, float drho, unsigned long long* nfb,
                                                         Capture cp) {
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
    if (active) bn = Bn[D * N + p];
    fb += mlp_or_hlld(sh, active, wl, wr, bn, gam, dp, drho, f, cp, 3 * p + D);
    if (active) store_flux<float, D>(F, NS, s, f);
  }
  block_count_atomic(fb, nfb);
}

// Learned-flux form of steps 5-6 for the D-faces in one kernel: each lane
// corrects its face's two states (as k_ctu_correct does), then the network
// (or HLLD at strong jumps) gives the flux with the half-step normal field.
template <int D, bool L>
__global__ void __launch_bounds__(kBlock) k_ctu_correct_mlp(Work w, const float* __restrict__ QL,
                                                            const float* __restrict__ QR, const float* __restrict__ F1,
                                                            const float* __restrict__ E1, const float* __restrict__ B,
                                                            const float* __restrict__ Bh, float* __restrict__ F2,
                                                            DtSrc dts, float inv_dx, float gam, const MlpWeights* mw,
                                                            float dp, float drho, unsigned long long* nfb, Capture cp) {
  __shared__ MlpShared sh;
  mlp_load_weights(sh, mw);
  const float hr = float(0.5 * get_dt(dts)) * inv_dx;
  const long long NS = w.NS;
  const long long nitems = work_items(w);
  int fb = 0;
  // block-uniform trips: every lane of a wave takes part in the network
  for (long long base = block_linear_id() - threadIdx.x; base < nitems; base += item_stride()) {
    const long long t = base + threadIdx.x;
    const bool active = t < nitems;
    long long p = 0, s = 0;
    float wl[7], wr[7], f[7];
    float bn = 1.0f;
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      wl[m] = 1.0f;
      wr[m] = 1.0f;
    }
    if (active) {
      const Site st = site_of<L>(w, t);
      p = st.p;
      s = st.s;
      bn = Bh[D * NS + s];
      corrected_states<float, D, L>(w, QL, QR, F1, E1, B, bn, st, hr, gam, wl, wr);
    }
    fb += mlp_or_hlld(sh, active, wl, wr, bn, gam, dp, drho, f, cp, 3 * p + D);
    if (active) store_flux<float, D>(F2, NS, s, f);
  }
  block_count_atomic(fb, nfb);
}

// group occupancy map of a list: clear, then mark
__global__ void __launch_bounds__(kBlock) k_occ_clear(int* occ, long long n) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) occ[t] = 0;
}

__global__ void __launch_bounds__(kBlock) k_occ_set(int* occ, const int* groups, int n_groups, const int* n_dev,
                                                    int edge, int gnx, int gny, int gnz) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int n = n_dev ? min(*n_dev, n_groups) : n_groups;
  if (g >= n) return;
  const int gi = groups[3 * g] / edge, gj = groups[3 * g + 1] / edge, gk = groups[3 * g + 2] / edge;
  // origins outside the level are never written (the host binding rejects them)
  if (groups[3 * g] < 0 || groups[3 * g + 1] < 0 || groups[3 * g + 2] < 0 || gi >= gnx || gj >= gny || gk >= gnz) return;
  occ[((long long)gk * gny + gj) * gnx + gi] = g + 1;   // 0: not listed, else group index + 1
}

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
