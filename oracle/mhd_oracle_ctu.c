/*
 * mhd_oracle_ctu.c -- CTU (corner transport upwind) integrator of the FP64
 * oracle, paper Sec. 3.2, CTU steps 1-8.  TEST INFRASTRUCTURE ONLY (see
 * mhd_oracle.c).
 *
 * Readings of points the paper leaves to its references (Stone et al. 2008,
 * Gardiner & Stone 2005/2008):
 *  - Step 1: PPM (Colella & Woodward 1984) in primitive variables: MC-limited
 *    slopes, interface values (q_i + q_{i+1})/2 - (dq_{i+1} - dq_i)/6, the
 *    CW84 monotonicity constraints; then characteristic tracing (Colella
 *    1990) with the 1D primitive MHD eigenvectors of the cell: a state at a
 *    cell edge is the edge value minus, for every wave moving toward that
 *    edge, its share of the parabola's average over the wave's domain of
 *    dependence during dt.  With PLM the parabola is the minmod line.
 *    With the HLL-family solvers (HLLE, HLLD), which do not resolve every
 *    wave, waves moving away from an edge are traced too (the parabola
 *    continued past the edge), so that both states of a face are
 *    time-centred in every characteristic field; otherwise the jump left in
 *    a field between a traced and an untraced state is dissipated at first
 *    order.  Roe's solver upwinds each wave and takes waves moving toward
 *    the edge only.
 *    The transverse field of each state then receives the multidimensional
 *    source term (dt/2) v_t dBn/dn, dBn/dn from the cell's own faces.
 *    A traced state with rho <= 0 or p <= 0 is replaced by the cell state.
 *  - Step 5: the hydrodynamic variables of each state are corrected by the
 *    transverse flux differences of step 2 over dt/2 in the cell the state
 *    comes from; its transverse field by the transverse part of the curl of
 *    the step-3 edge EMFs (averaged to the cell's faces).  Conversion to
 *    conserved variables uses the face's time-n normal field, conversion
 *    back its half-step normal field (step 4), the field of the step-6
 *    Riemann problem: the transverse energy fluxes carry the change of the
 *    normal field's magnetic energy.  The transverse flux differences in
 *    conserved form hold the div B terms of their own directions, -(dBt1/dt1
 *    + dBt2/dt2) = dBn/dn times (0, B, v.B, v); the state's 1D tracing holds
 *    none, so momentum and energy receive (dt/2)(B, v.B) dBn/dn from the
 *    source cell's faces (the field's share is the step-1 source term).
 *    A corrected state with rho <= 0 or p <= 0 falls back to its step-1
 *    value.
 *  - Step 6 uses the half-step normal field of the face.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mhd_oracle.h"

typedef struct {
  int n[3];
  double dx, gam;
} ctu_grid;

static size_t ncells(const ctu_grid* g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }
static int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static size_t idx3(const ctu_grid* g, int i, int j, int k) {
  return ((size_t)wrapi(k, g->n[2]) * g->n[1] + wrapi(j, g->n[1])) * g->n[0] + wrapi(i, g->n[0]);
}
static size_t idx_off(const ctu_grid* g, const int c[3], int ax, int s) {
  int q[3] = {c[0], c[1], c[2]};
  q[ax] += s;
  return idx3(g, q[0], q[1], q[2]);
}

/* 1D primitive state of cell c in the cyclic frame of direction d */
static void w1d(const double* W, size_t N, size_t c, int d, double w[7]) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  w[0] = W[c]; w[1] = W[(1 + d) * N + c]; w[2] = W[(1 + t1) * N + c]; w[3] = W[(1 + t2) * N + c];
  w[4] = W[4 * N + c]; w[5] = W[(5 + t1) * N + c]; w[6] = W[(5 + t2) * N + c];
}

/* Right eigenvectors of the 1D primitive MHD system
 * (rho, vn, vt1, vt2, p, Bt1, Bt2 with Bn fixed), Roe & Balsara
 * normalisation; waves ordered u-cf, u-ca, u-cs, u, u+cs, u+ca, u+cf. */
static void prim_eigen(const double w[7], double bn, double gam, double lam[7], double R[7][7]) {
  double d = w[0], u = w[1], p = w[4], by = w[5], bz = w[6];
  double asq = gam * p / d, a = sqrt(asq);
  double casq = bn * bn / d, ctsq = (by * by + bz * bz) / d;
  double sum = asq + casq + ctsq, dif = casq + ctsq - asq;
  double cfsq = 0.5 * (sum + sqrt(dif * dif + 4.0 * asq * ctsq));
  double cssq = asq * casq / cfsq;
  double cf = sqrt(cfsq), cs = sqrt(cssq), ca = sqrt(casq);
  double bt = sqrt(by * by + bz * bz);
  double b2, b3;
  if (bt > 0.0) { b2 = by / bt; b3 = bz / bt; }
  else { b2 = 1.0 / sqrt(2.0); b3 = 1.0 / sqrt(2.0); }
  double af, as;
  if (cfsq - cssq <= 0.0) { af = 1.0; as = 0.0; }
  else if (asq - cssq <= 0.0) { af = 0.0; as = 1.0; }
  else if (cfsq - asq <= 0.0) { af = 1.0; as = 0.0; }
  else { af = sqrt((asq - cssq) / (cfsq - cssq)); as = sqrt((cfsq - asq) / (cfsq - cssq)); }
  double s = (bn >= 0.0) ? 1.0 : -1.0, sd = sqrt(d);
  double Cff = cf * af, Css = cs * as, Qf = cf * af * s, Qs = cs * as * s, Af = a * af * sd, As = a * as * sd;
  double col[7][7] = {
      {d * af, -Cff, Qs * b2, Qs * b3, d * asq * af, As * b2, As * b3},
      {0.0, 0.0, -b3, b2, 0.0, -s * sd * b3, s * sd * b2},
      {d * as, -Css, -Qf * b2, -Qf * b3, d * asq * as, -Af * b2, -Af * b3},
      {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
      {d * as, Css, Qf * b2, Qf * b3, d * asq * as, -Af * b2, -Af * b3},
      {0.0, 0.0, b3, -b2, 0.0, -s * sd * b3, s * sd * b2},
      {d * af, Cff, -Qs * b2, -Qs * b3, d * asq * af, As * b2, As * b3}};
  for (int k = 0; k < 7; ++k)
    for (int m = 0; m < 7; ++m) R[m][k] = col[k][m];
  lam[0] = u - cf; lam[1] = u - ca; lam[2] = u - cs; lam[3] = u;
  lam[4] = u + cs; lam[5] = u + ca; lam[6] = u + cf;
}

/* wave amplitudes: solve R x = v by Gaussian elimination with pivoting */
static void amplitudes(const double R[7][7], const double v[7], double x[7]) {
  double A[7][7], b[7];
  memcpy(A, R, sizeof A);
  memcpy(b, v, sizeof b);
  for (int c = 0; c < 7; ++c) {
    int piv = c;
    for (int r = c + 1; r < 7; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < 7; ++k) { double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
      double t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    for (int r = c + 1; r < 7; ++r) {
      double m = A[r][c] / A[c][c];
      for (int k = c; k < 7; ++k) A[r][k] -= m * A[c][k];
      b[r] -= m * b[c];
    }
  }
  for (int r = 6; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < 7; ++k) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
  }
}

static double minmod2(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (a > 0.0) ? fmin(a, b) : fmax(a, b);
}

/* monotonised-central slope of q0 between neighbours qm and qp */
static double mc_slope(double qm, double q0, double qp) {
  double dl = q0 - qm, dr = qp - q0;
  if (dl * dr <= 0.0) return 0.0;
  double dc = 0.5 * (qp - qm);
  double lim = 2.0 * fmin(fabs(dl), fabs(dr));
  double m = fmin(fabs(dc), lim);
  return dc > 0.0 ? m : -m;
}

/* PPM edge values of the centre cell of q[0..4] (CW84) */
static void ppm_edges(const double q[5], double* qL, double* qR) {
  double dm = mc_slope(q[0], q[1], q[2]);
  double d0 = mc_slope(q[1], q[2], q[3]);
  double dp = mc_slope(q[2], q[3], q[4]);
  double l = 0.5 * (q[1] + q[2]) - (d0 - dm) / 6.0;
  double r = 0.5 * (q[2] + q[3]) - (dp - d0) / 6.0;
  double c = q[2];
  if ((r - c) * (c - l) <= 0.0) {
    l = c; r = c;
  } else {
    double dq = r - l, m6 = dq * (c - 0.5 * (l + r)), dq2 = dq * dq / 6.0;
    if (m6 > dq2) l = 3.0 * c - 2.0 * r;
    else if (-dq2 > m6) r = 3.0 * c - 2.0 * l;
  }
  *qL = l; *qR = r;
}

/* PPM edge values of q[2] from the five cells q[0..4], exported for the
 * unit pins of the reconstruction (no other caller) */
void or_ppm_edges(const double* q, double* qL, double* qR) { ppm_edges(q, qL, qR); }

/* Time-centred states at the two edges of cell c in direction d.
 * sl: state at the cell's lower edge (right state of its lower face);
 * sr: state at its upper edge (left state of its upper face). */
static void traced_states(const ctu_grid* g, int recon, int all_waves, const double* W, const double* B,
                          const int c[3], int d, double dt, double sl[7], double sr[7]) {
  size_t N = ncells(g);
  double q[5][7];
  for (int s = -2; s <= 2; ++s) w1d(W, N, idx_off(g, c, d, s), d, q[s + 2]);
  double w[7], ql[7], qr[7], dq[7], q6[7];
  memcpy(w, q[2], sizeof w);
  for (int m = 0; m < 7; ++m) {
    if (recon == OR_PPM) {
      double col[5] = {q[0][m], q[1][m], q[2][m], q[3][m], q[4][m]};
      ppm_edges(col, &ql[m], &qr[m]);
    } else if (recon == OR_PPM_UNLIMITED) {
      /* fourth-order interface values, no limiting: an order-of-accuracy probe */
      ql[m] = (7.0 * (q[1][m] + q[2][m]) - (q[0][m] + q[3][m])) / 12.0;
      qr[m] = (7.0 * (q[2][m] + q[3][m]) - (q[1][m] + q[4][m])) / 12.0;
    } else {
      double sl_ = minmod2(q[2][m] - q[1][m], q[3][m] - q[2][m]);
      ql[m] = q[2][m] - 0.5 * sl_;
      qr[m] = q[2][m] + 0.5 * sl_;
    }
    dq[m] = qr[m] - ql[m];
    q6[m] = 6.0 * (q[2][m] - 0.5 * (ql[m] + qr[m]));
  }
  size_t cc = idx3(g, c[0], c[1], c[2]);
  double bn_lo = B[d * N + cc], bn_hi = B[d * N + idx_off(g, c, d, 1)];
  double bn = 0.5 * (bn_lo + bn_hi);
  double lam[7], R[7][7], adq[7], aq6[7];
  prim_eigen(w, bn, g->gam, lam, R);
  amplitudes(R, dq, adq);
  amplitudes(R, q6, aq6);
  memcpy(sl, ql, 7 * sizeof(double));
  memcpy(sr, qr, 7 * sizeof(double));
  double r = dt / g->dx;
  for (int k = 0; k < 7; ++k) {
    double xi = lam[k] * r;
    /* upper edge: the profile's average over [1 - xi, 1] (cell units); for a
     * wave moving away (xi < 0) the parabola is continued past the edge */
    if (xi > 0.0 || (all_waves && xi < 0.0)) {
      double amp = 0.5 * xi * (adq[k] - (1.0 - 2.0 * xi / 3.0) * aq6[k]);
      for (int m = 0; m < 7; ++m) sr[m] -= amp * R[m][k];
    }
    /* lower edge: the average over [0, -xi] */
    if (xi < 0.0 || (all_waves && xi > 0.0)) {
      double ax = -xi;
      double amp = 0.5 * ax * (adq[k] + (1.0 - 2.0 * ax / 3.0) * aq6[k]);
      for (int m = 0; m < 7; ++m) sl[m] += amp * R[m][k];
    }
  }
  /* multidimensional source term for the transverse field */
  double dbn = (bn_hi - bn_lo) / g->dx;
  for (int pass = 0; pass < 2; ++pass) {
    double* s = pass ? sr : sl;
    s[5] += 0.5 * dt * w[2] * dbn;
    s[6] += 0.5 * dt * w[3] * dbn;
    if (!(s[0] > 0.0) || !(s[4] > 0.0)) memcpy(s, w, 7 * sizeof(double));
  }
}

/* Transverse correction (step 5) of state s of direction d coming from cell c
 * and sitting on the face whose normal field is bn at time n and bnh after
 * the half step (step 4).  The state enters conserved form with bn; the
 * transverse energy fluxes then carry the change of the normal field's
 * magnetic energy over dt/2, so the corrected state leaves conserved form
 * with bnh, the field the step-6 Riemann problem uses. */
static void correct_state(const ctu_grid* g, const double* const F[3], const double* E, const int c[3], int d,
                          double bn, double bnh, double dbn, double dt, const double s[7], double out[7]) {
  size_t N = ncells(g);
  double gam = g->gam;
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  /* global conserved vector: rho, Mx, My, Mz, e; transverse field by axis */
  double v[3], b[3];
  v[d] = s[1]; v[t1] = s[2]; v[t2] = s[3];
  b[d] = bn; b[t1] = s[5]; b[t2] = s[6];
  double u[5];
  u[0] = s[0];
  for (int a = 0; a < 3; ++a) u[1 + a] = s[0] * v[a];
  u[4] = s[4] / (gam - 1.0) + 0.5 * s[0] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
         0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  size_t cc = idx3(g, c[0], c[1], c[2]);
  double hr = 0.5 * dt / g->dx;
  /* the state's share of the multidimensional source: momentum B dBn/dn,
   * energy (v.B) dBn/dn over dt/2, dbn = the source cell's normal-field
   * difference (its transverse-field share is in the traced state) */
  double vb = v[0] * b[0] + v[1] * b[1] + v[2] * b[2];
  for (int a = 0; a < 3; ++a) u[1 + a] += hr * dbn * b[a];
  u[4] += hr * dbn * vb;
  for (int tt = 0; tt < 2; ++tt) {
    int t = tt ? t2 : t1;
    size_t cp = idx_off(g, c, t, 1);
    for (int m = 0; m < 5; ++m) u[m] -= hr * (F[t][m * N + cp] - F[t][m * N + cc]);
  }
  /* transverse field: only the derivatives across d of the edge EMF E_d */
  for (int tt = 0; tt < 2; ++tt) {
    int bax = tt ? t2 : t1;              /* field component being corrected */
    int der = (bax == (d + 2) % 3) ? (d + 1) % 3 : (d + 2) % 3; /* derivative direction (not d, not bax) */
    /* E_d on the four d-edges of cell c, averaged to the two faces normal to der */
    size_t e00 = idx3(g, c[0], c[1], c[2]);
    size_t e_der = idx_off(g, c, der, 1);
    size_t e_b = idx_off(g, c, bax, 1);
    int qq[3] = {c[0], c[1], c[2]};
    qq[der] += 1; qq[bax] += 1;
    size_t e_derb = idx3(g, qq[0], qq[1], qq[2]);
    const double* Ed = E + (size_t)d * N;
    double up = 0.5 * (Ed[e_der] + Ed[e_derb]);
    double lo = 0.5 * (Ed[e00] + Ed[e_b]);
    double dEd = (up - lo) / g->dx;
    /* dB_bax/dt restricted to derivatives across d:
     *   +dE_d/d(der) if d = bax + 1 (mod 3), -dE_d/d(der) if d = bax + 2 */
    double sign = (d == (bax + 1) % 3) ? 1.0 : -1.0;
    b[bax] += 0.5 * dt * sign * dEd;
  }
  /* back to primitives with the half-step normal field */
  b[d] = bnh;
  double w[7];
  w[0] = u[0];
  double vx = u[1] / u[0], vy = u[2] / u[0], vz = u[3] / u[0];
  double vv[3] = {vx, vy, vz};
  w[1] = vv[d]; w[2] = vv[t1]; w[3] = vv[t2];
  w[5] = b[t1]; w[6] = b[t2];
  w[4] = (gam - 1.0) * (u[4] - 0.5 * u[0] * (vx * vx + vy * vy + vz * vz) -
                        0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
  if (w[0] > 0.0 && w[4] > 0.0) memcpy(out, w, sizeof w);
  else memcpy(out, s, 7 * sizeof(double));
}

/* store a 1D flux of direction d at face p of F[d] */
static void store_flux(double* Fd, size_t N, size_t p, int d, const double f[7]) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  Fd[p] = f[0];
  Fd[(1 + d) * N + p] = f[1];
  Fd[(1 + t1) * N + p] = f[2];
  Fd[(1 + t2) * N + p] = f[3];
  Fd[4 * N + p] = f[4];
  Fd[5 * N + p] = f[6];
  Fd[6 * N + p] = -f[5];
}

int or_ctu_step_impl(int nx, int ny, int nz, double dx, double gam, int recon, int solver,
                     const double* U, const double* B, double dt, double* Uo, double* Bo,
                     int* nfallback, double* Fout, double* Eout) {
  if (recon != OR_PLM && recon != OR_PPM && recon != OR_PPM_UNLIMITED) return -1;
  ctu_grid g;
  g.n[0] = nx; g.n[1] = ny; g.n[2] = nz; g.dx = dx; g.gam = gam;
  size_t N = ncells(&g);
  double* W = malloc(8 * N * sizeof(double));
  double* Wh = malloc(8 * N * sizeof(double));
  double* QL = malloc(21 * N * sizeof(double));   /* [d][m][face]: state below face */
  double* QR = malloc(21 * N * sizeof(double));   /* state above face */
  double* Fs[3];
  double* Fc[3];
  for (int d = 0; d < 3; ++d) {
    Fs[d] = malloc(7 * N * sizeof(double));
    Fc[d] = malloc(7 * N * sizeof(double));
  }
  double* Es = malloc(3 * N * sizeof(double));
  double* Ec = malloc(3 * N * sizeof(double));
  double* Uh = malloc(5 * N * sizeof(double));
  double* Bh = malloc(3 * N * sizeof(double));
  if (!W || !Wh || !QL || !QR || !Es || !Ec || !Uh || !Bh) return -2;
  const double* Fsc[3] = {Fs[0], Fs[1], Fs[2]};
  const double* Fcc[3] = {Fc[0], Fc[1], Fc[2]};
  int fb = 0;

  or__primitives(nx, ny, nz, dx, gam, U, B, W);
  /* 1. time-centred interface states */
  for (int d = 0; d < 3; ++d) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          int c[3] = {i, j, k};
          double sl[7], sr[7];
          traced_states(&g, recon, solver != OR_ROE, W, B, c, d, dt, sl, sr);
          size_t lo = idx3(&g, i, j, k), hi = idx_off(&g, c, d, 1);
          for (int m = 0; m < 7; ++m) {
            QR[((size_t)d * 7 + m) * N + lo] = sl[m];
            QL[((size_t)d * 7 + m) * N + hi] = sr[m];
          }
        }
  }
  /* 2. Riemann fluxes with the time-n normal field */
  for (int d = 0; d < 3; ++d) {
    int fbd = 0;
#pragma omp parallel for schedule(static) reduction(+ : fbd)
    for (size_t p = 0; p < N; ++p) {
      double wl[7], wr[7], f[7];
      for (int m = 0; m < 7; ++m) {
        wl[m] = QL[((size_t)d * 7 + m) * N + p];
        wr[m] = QR[((size_t)d * 7 + m) * N + p];
      }
      fbd += or__riemann(solver, wl, wr, B[d * N + p], gam, f);
      store_flux(Fs[d], N, p, d, f);
    }
    fb += fbd;
  }
  /* 3. edge EMFs, 4. half-step update */
  or__edge_emfs(nx, ny, nz, dx, Fsc, W, Es);
  or__apply_update(nx, ny, nz, dx, U, B, Fsc, Es, 0.5 * dt, Uh, Bh);
  or__primitives(nx, ny, nz, dx, gam, Uh, Bh, Wh);
  /* 5. transverse correction, 6. Riemann fluxes with the half-step normal field */
  for (int d = 0; d < 3; ++d) {
    int fbd = 0;
#pragma omp parallel for schedule(static) reduction(+ : fbd)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          int c[3] = {i, j, k};
          size_t p = idx3(&g, i, j, k);
          int cl[3] = {i, j, k};
          cl[d] -= 1;
          double sl[7], sr[7], wl[7], wr[7], f[7];
          for (int m = 0; m < 7; ++m) {
            sl[m] = QL[((size_t)d * 7 + m) * N + p];
            sr[m] = QR[((size_t)d * 7 + m) * N + p];
          }
          double bn = B[d * N + p];
          double bn_lo = B[d * N + idx_off(&g, c, d, -1)], bn_hi = B[d * N + idx_off(&g, c, d, 1)];
          correct_state(&g, Fsc, Es, cl, d, bn, Bh[d * N + p], bn - bn_lo, dt, sl, wl);
          correct_state(&g, Fsc, Es, c, d, bn, Bh[d * N + p], bn_hi - bn, dt, sr, wr);
          fbd += or__riemann(solver, wl, wr, Bh[d * N + p], gam, f);
          store_flux(Fc[d], N, p, d, f);
        }
    fb += fbd;
  }
  /* 7. edge EMFs with the half-step reference, 8. full update */
  or__edge_emfs(nx, ny, nz, dx, Fcc, Wh, Ec);
  or__apply_update(nx, ny, nz, dx, U, B, Fcc, Ec, dt, Uo, Bo);
  or__copy_final(N, Fcc, Ec, Fout, Eout);

  free(W); free(Wh); free(QL); free(QR); free(Es); free(Ec); free(Uh); free(Bh);
  for (int d = 0; d < 3; ++d) { free(Fs[d]); free(Fc[d]); }
  if (nfallback) *nfallback += fb;
  return 0;
}
