/*
 * mhd_oracle.c -- plain, slow, FP64 CPU reference of the unsplit ideal-MHD
 * update of "Magnetohydrodynamics with GAMER" (Zhang, Schive & Chiueh).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library, and the GPU library never calls it.
 *
 * Everything is written for clarity: whole-grid arrays, periodic wrap by
 * modular index arithmetic, one output per loop iteration, no tiling, no
 * fusion.  OpenMP splits only loops whose iterations are independent, so the
 * result is bit-identical for any thread count.  Build with
 * -ffp-contract=off so that no multiply-add is fused.
 *
 * Notation (paper Sec. 2, Eqs. 1-9): U = (rho, Mx, My, Mz, e) at cell centres
 * (Eq. 11 volume averages), face-area-averaged B on cell faces (Eq. 14), edge
 * EMFs E = -V x B (Eq. 15).  Units mu = 1.  Cells are cubic (Sec. 3.1).
 *
 * Array layout: [component][z][y][x], x fastest.  bx[k][j][i] sits on the
 * x-face at x = i*dx (the lower x-face of cell i), by on the lower y-face,
 * bz on the lower z-face.  Edge EMF ex[k][j][i] sits on the x-edge at
 * (y, z) = (j*dx, k*dx) through cell column i, ey on the y-edge at
 * (x, z) = (i*dx, k*dx), ez on the z-edge at (x, y) = (i*dx, j*dx).
 *
 * One-dimensional Riemann problems are solved in the frame of the face
 * normal n with tangential axes (t1, t2) chosen cyclically: x-faces use
 * (x, y, z), y-faces (y, z, x), z-faces (z, x, y).  A 1D primitive state is
 * w = (rho, vn, vt1, vt2, p, bt1, bt2) with the normal field bn passed apart;
 * the 1D flux is f = (rho, Mn, Mt1, Mt2, e, Bt1, Bt2) components of Eq. 7.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "mhd_oracle.h"

/* ------------------------------------------------------------------ */
/* grid helpers                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  int n[3];      /* nx, ny, nz */
  double dx;     /* cubic cell width */
  double gam;    /* adiabatic index */
} grid_t;

static size_t ncell(const grid_t* g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }

static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* linear index of cell (i, j, k) with periodic wrap */
static size_t at(const grid_t* g, int i, int j, int k) {
  return ((size_t)wrap(k, g->n[2]) * g->n[1] + wrap(j, g->n[1])) * g->n[0] + wrap(i, g->n[0]);
}

/* index of the neighbour of cell (i, j, k) displaced by s along axis ax */
static size_t at_shift(const grid_t* g, int i, int j, int k, int ax, int s) {
  int c[3] = {i, j, k};
  c[ax] += s;
  return at(g, c[0], c[1], c[2]);
}

/* cyclic frame of a face normal: n, t1, t2 */
static void frame(int d, int* n, int* t1, int* t2) { *n = d; *t1 = (d + 1) % 3; *t2 = (d + 2) % 3; }

/* ------------------------------------------------------------------ */
/* 1D state algebra (Eqs. 5-7)                                         */
/* ------------------------------------------------------------------ */
static double total_energy(const double w[7], double bn, double gam) {
  /* Eq. 5 */
  return w[4] / (gam - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) +
         0.5 * (bn * bn + w[5] * w[5] + w[6] * w[6]);
}

static void w_to_u(const double w[7], double bn, double gam, double u[7]) {
  u[0] = w[0];
  u[1] = w[0] * w[1];
  u[2] = w[0] * w[2];
  u[3] = w[0] * w[3];
  u[4] = total_energy(w, bn, gam);
  u[5] = w[5];
  u[6] = w[6];
}

static void u_to_w(const double u[7], double bn, double gam, double w[7]) {
  w[0] = u[0];
  w[1] = u[1] / u[0];
  w[2] = u[2] / u[0];
  w[3] = u[3] / u[0];
  w[5] = u[5];
  w[6] = u[6];
  w[4] = (gam - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0] -
                        0.5 * (bn * bn + u[5] * u[5] + u[6] * u[6]));
}

/* physical flux along n, Eq. 7 written in the face frame */
static void phys_flux(const double w[7], double bn, double gam, double f[7]) {
  double d = w[0], vn = w[1], v1 = w[2], v2 = w[3], p = w[4], b1 = w[5], b2 = w[6];
  double pt = p + 0.5 * (bn * bn + b1 * b1 + b2 * b2);   /* P* */
  double e = total_energy(w, bn, gam);
  double vb = vn * bn + v1 * b1 + v2 * b2;
  f[0] = d * vn;
  f[1] = d * vn * vn + pt - bn * bn;
  f[2] = d * vn * v1 - bn * b1;
  f[3] = d * vn * v2 - bn * b2;
  f[4] = (e + pt) * vn - bn * vb;
  f[5] = b1 * vn - bn * v1;
  f[6] = b2 * vn - bn * v2;
}

/* fast magnetosonic speed along n:
 * cf^2 = (a^2 + b^2 + sqrt((a^2 - b^2)^2 + 4 a^2 bt^2)) / 2, the
 * cancellation-free form of the textbook root; a^2 = gam p / rho,
 * b^2 = |B|^2 / rho, bt^2 = (|B|^2 - bn^2) / rho. */
static double fast_speed(double d, double p, double bn, double b1, double b2, double gam) {
  double asq = gam * p / d;
  double btsq = (b1 * b1 + b2 * b2) / d;
  double bsq = bn * bn / d + btsq;
  double diff = asq - bsq;
  return sqrt(0.5 * (asq + bsq + sqrt(diff * diff + 4.0 * asq * btsq)));
}

/* ------------------------------------------------------------------ */
/* Riemann solvers                                                     */
/* ------------------------------------------------------------------ */

/* HLLE with Davis wave-speed bounds. */
static void riemann_hlle(const double wl[7], const double wr[7], double bn, double gam, double f[7]) {
  double cfl = fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gam);
  double cfr = fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gam);
  double sl = fmin(wl[1] - cfl, wr[1] - cfr);
  double sr = fmax(wl[1] + cfl, wr[1] + cfr);
  double fl[7], fr[7], ul[7], ur[7];
  phys_flux(wl, bn, gam, fl);
  phys_flux(wr, bn, gam, fr);
  if (sl >= 0.0) { memcpy(f, fl, sizeof fl); return; }
  if (sr <= 0.0) { memcpy(f, fr, sizeof fr); return; }
  w_to_u(wl, bn, gam, ul);
  w_to_u(wr, bn, gam, ur);
  for (int m = 0; m < 7; ++m)
    f[m] = (sr * fl[m] - sl * fr[m] + sl * sr * (ur[m] - ul[m])) / (sr - sl);
}

/* Roe-averaged eigen-system of the linearised 1D problem.
 *
 * Averages: sqrt(rho)-weighted velocity and total enthalpy H = (e + P*)/rho,
 * geometric-mean density, transverse field weighted with the opposite
 * side's sqrt(rho) (Cargo & Gallice 1997).  With these, the Roe matrix is
 * the flux Jacobian at the averaged state except that the density
 * derivative of P* carries -(gam-2) X, X = |dBt|^2 / (2 (sqrt rhoL +
 * sqrt rhoR)^2); hence the modified sound speed
 *   a~^2 = (gam-1)(H - |v|^2/2 - |B|^2/rho) - (gam-2) X
 * and the entropy-wave energy |v|^2/2 + (gam-2) X/(gam-1).
 * Right eigenvectors use the Roe & Balsara (1996) normalisation.
 * Waves are ordered u-cf, u-ca, u-cs, u, u+cs, u+ca, u+cf.
 * R is row-major R[component][wave]. */
static void roe_eigensystem(const double wl[7], const double wr[7], double bn, double gam,
                            double lam[7], double R[7][7]) {
  const double g1 = gam - 1.0, g2 = gam - 2.0;
  double sl = sqrt(wl[0]), sr = sqrt(wr[0]);
  double isum = 1.0 / (sl + sr);
  double d = sl * sr;
  double vx = (sl * wl[1] + sr * wr[1]) * isum;
  double vy = (sl * wl[2] + sr * wr[2]) * isum;
  double vz = (sl * wl[3] + sr * wr[3]) * isum;
  double hl = (total_energy(wl, bn, gam) + wl[4] + 0.5 * (bn * bn + wl[5] * wl[5] + wl[6] * wl[6])) / wl[0];
  double hr = (total_energy(wr, bn, gam) + wr[4] + 0.5 * (bn * bn + wr[5] * wr[5] + wr[6] * wr[6])) / wr[0];
  double h = (sl * hl + sr * hr) * isum;
  double by = (sr * wl[5] + sl * wr[5]) * isum;
  double bz = (sr * wl[6] + sl * wr[6]) * isum;
  double dby = wr[5] - wl[5], dbz = wr[6] - wl[6];
  double X = 0.5 * (dby * dby + dbz * dbz) * isum * isum;

  double vsq = vx * vx + vy * vy + vz * vz;
  double btsq = by * by + bz * bz;
  double casq = bn * bn / d;
  double hp = h - (casq + btsq / d);          /* H minus magnetic enthalpy */
  double asq = g1 * (hp - 0.5 * vsq) - g2 * X; /* a~^2 */
  if (asq < 0.0) asq = 0.0;
  double ctsq = btsq / d;
  double sum = casq + ctsq + asq;
  double dif = casq + ctsq - asq;
  double root = sqrt(dif * dif + 4.0 * asq * ctsq);
  double cfsq = 0.5 * (sum + root);
  double cssq = (cfsq > 0.0) ? asq * casq / cfsq : 0.0;
  double cf = sqrt(cfsq), cs = sqrt(cssq), ca = sqrt(casq);
  double bt = sqrt(btsq);
  double b2, b3;
  if (bt > 0.0) { b2 = by / bt; b3 = bz / bt; }
  else { b2 = 1.0 / sqrt(2.0); b3 = 1.0 / sqrt(2.0); }
  double af, as;
  if (cfsq - cssq <= 0.0) { af = 1.0; as = 0.0; }
  else if (asq - cssq <= 0.0) { af = 0.0; as = 1.0; }
  else if (cfsq - asq <= 0.0) { af = 1.0; as = 0.0; }
  else { af = sqrt((asq - cssq) / (cfsq - cssq)); as = sqrt((cfsq - asq) / (cfsq - cssq)); }
  double sqd = sqrt(d), isqd = 1.0 / sqd;
  double s = (bn >= 0.0) ? 1.0 : -1.0;
  double a = sqrt(asq);
  double qf = cf * af * s, qs = cs * as * s;
  double afp = af * a * isqd, asp = as * a * isqd;
  double vbet = vy * b2 + vz * b3;
  double afpb = afp * bt, aspb = asp * bt;   /* |beta| = 1 */

  lam[0] = vx - cf; lam[1] = vx - ca; lam[2] = vx - cs; lam[3] = vx;
  lam[4] = vx + cs; lam[5] = vx + ca; lam[6] = vx + cf;

  /* fast, u - cf */
  R[0][0] = af; R[1][0] = af * (vx - cf); R[2][0] = af * vy + qs * b2; R[3][0] = af * vz + qs * b3;
  R[4][0] = af * (hp - vx * cf) + qs * vbet + aspb; R[5][0] = asp * b2; R[6][0] = asp * b3;
  /* Alfven, u - ca */
  R[0][1] = 0.0; R[1][1] = 0.0; R[2][1] = -b3; R[3][1] = b2;
  R[4][1] = -(vy * b3 - vz * b2); R[5][1] = -s * b3 * isqd; R[6][1] = s * b2 * isqd;
  /* slow, u - cs */
  R[0][2] = as; R[1][2] = as * (vx - cs); R[2][2] = as * vy - qf * b2; R[3][2] = as * vz - qf * b3;
  R[4][2] = as * (hp - vx * cs) - qf * vbet - afpb; R[5][2] = -afp * b2; R[6][2] = -afp * b3;
  /* entropy, u */
  R[0][3] = 1.0; R[1][3] = vx; R[2][3] = vy; R[3][3] = vz;
  R[4][3] = 0.5 * vsq + g2 * X / g1; R[5][3] = 0.0; R[6][3] = 0.0;
  /* slow, u + cs */
  R[0][4] = as; R[1][4] = as * (vx + cs); R[2][4] = as * vy + qf * b2; R[3][4] = as * vz + qf * b3;
  R[4][4] = as * (hp + vx * cs) + qf * vbet - afpb; R[5][4] = -afp * b2; R[6][4] = -afp * b3;
  /* Alfven, u + ca */
  R[0][5] = 0.0; R[1][5] = 0.0; R[2][5] = b3; R[3][5] = -b2;
  R[4][5] = (vy * b3 - vz * b2); R[5][5] = -s * b3 * isqd; R[6][5] = s * b2 * isqd;
  /* fast, u + cf */
  R[0][6] = af; R[1][6] = af * (vx + cf); R[2][6] = af * vy - qs * b2; R[3][6] = af * vz - qs * b3;
  R[4][6] = af * (hp + vx * cf) - qs * vbet + aspb; R[5][6] = asp * b2; R[6][6] = asp * b3;
}

/* Solve A x = b for a 7x7 system by Gaussian elimination with partial
 * pivoting (A and b are overwritten).  Returns 0, or -1 if singular. */
static int solve7(double A[7][7], double b[7], double x[7]) {
  for (int c = 0; c < 7; ++c) {
    int piv = c;
    for (int r = c + 1; r < 7; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (A[piv][c] == 0.0) return -1;
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
  return 0;
}

/* Roe flux F = (F_L + F_R)/2 - (1/2) sum_k |lam_k| alpha_k r_k, with the wave
 * strengths alpha found by solving R alpha = U_R - U_L.  If any state between
 * the waves has rho <= 0 or p <= 0, the HLLE flux is used instead.
 * Returns 1 when the fallback was taken, 0 otherwise. */
static int riemann_roe(const double wl[7], const double wr[7], double bn, double gam, double f[7]) {
  double lam[7], R[7][7], A[7][7], du[7], alpha[7], ul[7], ur[7], fl[7], fr[7];
  roe_eigensystem(wl, wr, bn, gam, lam, R);
  w_to_u(wl, bn, gam, ul);
  w_to_u(wr, bn, gam, ur);
  for (int m = 0; m < 7; ++m) du[m] = ur[m] - ul[m];
  memcpy(A, R, sizeof A);
  if (solve7(A, du, alpha) != 0) { riemann_hlle(wl, wr, bn, gam, f); return 1; }
  /* positivity of the intermediate states */
  double us[7];
  memcpy(us, ul, sizeof us);
  for (int k = 0; k < 6; ++k) {
    for (int m = 0; m < 7; ++m) us[m] += alpha[k] * R[m][k];
    double p = (gam - 1.0) * (us[4] - 0.5 * (us[1] * us[1] + us[2] * us[2] + us[3] * us[3]) / us[0] -
                              0.5 * (bn * bn + us[5] * us[5] + us[6] * us[6]));
    if (us[0] <= 0.0 || p <= 0.0) { riemann_hlle(wl, wr, bn, gam, f); return 1; }
  }
  phys_flux(wl, bn, gam, fl);
  phys_flux(wr, bn, gam, fr);
  for (int m = 0; m < 7; ++m) {
    double diss = 0.0;
    for (int k = 0; k < 7; ++k) diss += fabs(lam[k]) * alpha[k] * R[m][k];
    f[m] = 0.5 * (fl[m] + fr[m]) - 0.5 * diss;
  }
  return 0;
}

/* HLLD (Miyoshi & Kusano 2005): five-wave approximate solver with outer
 * speeds S_L = min(uL, uR) - max(cfL, cfR), S_R = max(uL, uR) + max(cfL, cfR),
 * contact speed S_M, Alfven speeds S*_{L,R} = S_M -/+ |Bn| / sqrt(rho*). */
static void hlld_star(const double w[7], const double u[7], double bn, double S, double SM,
                      double ptstar, double ustar[7]) {
  double d = w[0], vn = w[1];
  double ds = d * (S - vn) / (S - SM);
  double den = d * (S - vn) * (S - SM) - bn * bn;
  double v1s, v2s, b1s, b2s;
  if (fabs(den) <= 1e-12 * (fabs(d * (S - vn) * (S - SM)) + bn * bn)) {
    /* degenerate: the Alfven and fast waves coincide, no transverse jump */
    v1s = w[2]; v2s = w[3]; b1s = w[5]; b2s = w[6];
  } else {
    double mfac = bn * (SM - vn) / den;
    double bfac = (d * (S - vn) * (S - vn) - bn * bn) / den;
    v1s = w[2] - w[5] * mfac;
    v2s = w[3] - w[6] * mfac;
    b1s = w[5] * bfac;
    b2s = w[6] * bfac;
  }
  double pt = w[4] + 0.5 * (bn * bn + w[5] * w[5] + w[6] * w[6]);
  double vb = vn * bn + w[2] * w[5] + w[3] * w[6];
  double vbs = SM * bn + v1s * b1s + v2s * b2s;
  double es = ((S - vn) * u[4] - pt * vn + ptstar * SM + bn * (vb - vbs)) / (S - SM);
  ustar[0] = ds; ustar[1] = ds * SM; ustar[2] = ds * v1s; ustar[3] = ds * v2s;
  ustar[4] = es; ustar[5] = b1s; ustar[6] = b2s;
}

static void riemann_hlld(const double wl[7], const double wr[7], double bn, double gam, double f[7]) {
  double fl[7], fr[7], ul[7], ur[7];
  phys_flux(wl, bn, gam, fl);
  phys_flux(wr, bn, gam, fr);
  double cfl = fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gam);
  double cfr = fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gam);
  double cmax = fmax(cfl, cfr);
  double SL = fmin(wl[1], wr[1]) - cmax;
  double SR = fmax(wl[1], wr[1]) + cmax;
  if (SL >= 0.0) { memcpy(f, fl, sizeof fl); return; }
  if (SR <= 0.0) { memcpy(f, fr, sizeof fr); return; }
  w_to_u(wl, bn, gam, ul);
  w_to_u(wr, bn, gam, ur);
  double ptl = wl[4] + 0.5 * (bn * bn + wl[5] * wl[5] + wl[6] * wl[6]);
  double ptr = wr[4] + 0.5 * (bn * bn + wr[5] * wr[5] + wr[6] * wr[6]);
  double ml = wl[0] * (SL - wl[1]);   /* rho (S - u) on each side */
  double mr = wr[0] * (SR - wr[1]);
  double SM = (mr * wr[1] - ml * wl[1] - ptr + ptl) / (mr - ml);
  double ptstar = ptl + ml * (SM - wl[1]);
  double usl[7], usr[7];
  hlld_star(wl, ul, bn, SL, SM, ptstar, usl);
  hlld_star(wr, ur, bn, SR, SM, ptstar, usr);
  double sdl = sqrt(usl[0]), sdr = sqrt(usr[0]);
  double SLs = SM - fabs(bn) / sdl;
  double SRs = SM + fabs(bn) / sdr;
  double fsl[7], fsr[7];
  for (int m = 0; m < 7; ++m) {
    fsl[m] = fl[m] + SL * (usl[m] - ul[m]);
    fsr[m] = fr[m] + SR * (usr[m] - ur[m]);
  }
  if (SLs >= 0.0) { memcpy(f, fsl, sizeof fsl); return; }
  if (SRs <= 0.0) { memcpy(f, fsr, sizeof fsr); return; }
  /* double-star states, shared velocity and transverse field */
  double sgn = (bn >= 0.0) ? 1.0 : -1.0;
  double iden = 1.0 / (sdl + sdr);
  double v1l = usl[2] / usl[0], v2l = usl[3] / usl[0];
  double v1r = usr[2] / usr[0], v2r = usr[3] / usr[0];
  double v1ss = (sdl * v1l + sdr * v1r + (usr[5] - usl[5]) * sgn) * iden;
  double v2ss = (sdl * v2l + sdr * v2r + (usr[6] - usl[6]) * sgn) * iden;
  double b1ss = (sdl * usr[5] + sdr * usl[5] + sdl * sdr * (v1r - v1l) * sgn) * iden;
  double b2ss = (sdl * usr[6] + sdr * usl[6] + sdl * sdr * (v2r - v2l) * sgn) * iden;
  double vbss = SM * bn + v1ss * b1ss + v2ss * b2ss;
  if (SM >= 0.0) {
    double vbl = SM * bn + v1l * usl[5] + v2l * usl[6];
    double uss[7] = {usl[0], usl[0] * SM, usl[0] * v1ss, usl[0] * v2ss,
                     usl[4] - sdl * (vbl - vbss) * sgn, b1ss, b2ss};
    for (int m = 0; m < 7; ++m) f[m] = fsl[m] + SLs * (uss[m] - usl[m]);
  } else {
    double vbr = SM * bn + v1r * usr[5] + v2r * usr[6];
    double uss[7] = {usr[0], usr[0] * SM, usr[0] * v1ss, usr[0] * v2ss,
                     usr[4] + sdr * (vbr - vbss) * sgn, b1ss, b2ss};
    for (int m = 0; m < 7; ++m) f[m] = fsr[m] + SRs * (uss[m] - usr[m]);
  }
}

static int riemann(int solver, const double wl[7], const double wr[7], double bn, double gam, double f[7]) {
  switch (solver) {
    case OR_ROE: return riemann_roe(wl, wr, bn, gam, f);
    case OR_HLLE: riemann_hlle(wl, wr, bn, gam, f); return 0;
    case OR_HLLD: riemann_hlld(wl, wr, bn, gam, f); return 0;
    default: return -1;
  }
}

/* ------------------------------------------------------------------ */
/* grid operations                                                     */
/* ------------------------------------------------------------------ */

/* Primitive cell state.  W has 8 components: rho, vx, vy, vz, p,
 * Bcx, Bcy, Bcz, where the cell-centred field is the mean of the two
 * opposite face values. */
static void primitives(const grid_t* g, const double* U, const double* B, double* W) {
  size_t N = ncell(g);
  const double gam = g->gam;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        size_t c = at(g, i, j, k);
        double bc[3];
        for (int a = 0; a < 3; ++a) bc[a] = 0.5 * (B[a * N + c] + B[a * N + at_shift(g, i, j, k, a, 1)]);
        double d = U[c];
        double vx = U[N + c] / d, vy = U[2 * N + c] / d, vz = U[3 * N + c] / d;
        double p = (gam - 1.0) * (U[4 * N + c] - 0.5 * d * (vx * vx + vy * vy + vz * vz) -
                                  0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]));
        W[c] = d; W[N + c] = vx; W[2 * N + c] = vy; W[3 * N + c] = vz; W[4 * N + c] = p;
        W[5 * N + c] = bc[0]; W[6 * N + c] = bc[1]; W[7 * N + c] = bc[2];
      }
}

/* 1D primitive state of cell c in the frame of direction d */
static void cell_w1d(const double* W, size_t N, size_t c, int d, double w[7]) {
  int n, t1, t2;
  frame(d, &n, &t1, &t2);
  w[0] = W[c];
  w[1] = W[(1 + n) * N + c];
  w[2] = W[(1 + t1) * N + c];
  w[3] = W[(1 + t2) * N + c];
  w[4] = W[4 * N + c];
  w[5] = W[(5 + t1) * N + c];
  w[6] = W[(5 + t2) * N + c];
}

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (a > 0.0) ? fmin(a, b) : fmax(a, b);
}

/* Face fluxes of one direction d.  Face (i,j,k) of F[d] is the lower face
 * of cell (i,j,k).  Stored components: 0 mass, 1..3 momentum x,y,z, 4 energy,
 * 5 E_t1, 6 E_t2 (the edge-parallel EMFs carried by the face:
 * E_t1 = F_n[B_t2], E_t2 = -F_n[B_t1], from E = -V x B).
 * recon: OR_FIRST_ORDER uses the two cell states, OR_PLM minmod-limited
 * linear states in primitive variables, OR_PPM the limited parabolas of
 * Colella & Woodward (the upper edge value of the left cell and the lower
 * edge value of the right cell, in primitive variables, no tracing: the VL
 * predictor already centres the data in time). */
static void face_fluxes(const grid_t* g, int d, int recon, int solver, const double* W,
                        const double* B, double* F, int* nfallback) {
  size_t N = ncell(g);
  int n, t1, t2;
  frame(d, &n, &t1, &t2);
  int fb = 0;
#pragma omp parallel for schedule(static) reduction(+ : fb)
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        size_t cR = at(g, i, j, k);
        size_t cL = at_shift(g, i, j, k, d, -1);
        double wl[7], wr[7];
        cell_w1d(W, N, cL, d, wl);
        cell_w1d(W, N, cR, d, wr);
        if (recon == OR_PPM) {
          /* cells -3 .. 2 relative to the face's upper cell */
          double c6[6][7];
          for (int s = -3; s <= 2; ++s) cell_w1d(W, N, at_shift(g, i, j, k, d, s), d, c6[s + 3]);
          for (int m = 0; m < 7; ++m) {
            double lo, hi;
            double ql[5] = {c6[0][m], c6[1][m], c6[2][m], c6[3][m], c6[4][m]};
            double qr[5] = {c6[1][m], c6[2][m], c6[3][m], c6[4][m], c6[5][m]};
            or_ppm_edges(ql, &lo, &hi);
            wl[m] = hi;                       /* upper edge of the left cell */
            or_ppm_edges(qr, &lo, &hi);
            wr[m] = lo;                       /* lower edge of the right cell */
          }
        } else if (recon == OR_PLM || recon == OR_PLM_UNLIMITED) {
          double wll[7], wrr[7];
          cell_w1d(W, N, at_shift(g, i, j, k, d, -2), d, wll);
          cell_w1d(W, N, at_shift(g, i, j, k, d, 1), d, wrr);
          for (int m = 0; m < 7; ++m) {
            double sL, sR;
            if (recon == OR_PLM) {
              sL = minmod(wl[m] - wll[m], wr[m] - wl[m]);
              sR = minmod(wr[m] - wl[m], wrr[m] - wr[m]);
            } else { /* central slopes, no limiter: an order-of-accuracy probe only */
              sL = 0.5 * (wr[m] - wll[m]);
              sR = 0.5 * (wrr[m] - wl[m]);
            }
            wl[m] = wl[m] + 0.5 * sL;
            wr[m] = wr[m] - 0.5 * sR;
          }
        }
        double bn = B[d * N + cR];
        double f[7];
        fb += riemann(solver, wl, wr, bn, g->gam, f);
        F[cR] = f[0];
        F[(1 + n) * N + cR] = f[1];
        F[(1 + t1) * N + cR] = f[2];
        F[(1 + t2) * N + cR] = f[3];
        F[4 * N + cR] = f[4];
        F[5 * N + cR] = f[6];    /* E_t1 */
        F[6 * N + cR] = -f[5];   /* E_t2 */
      }
  if (nfallback) *nfallback += fb;
}

/* cell-centre reference EMF component a: -(V x B)_a with cell B */
static double ref_emf(const double* W, size_t N, size_t c, int a) {
  int b = (a + 1) % 3, cc = (a + 2) % 3;
  /* (V x B)_a = v_b B_c - v_c B_b */
  return -(W[(1 + b) * N + c] * W[(5 + cc) * N + c] - W[(1 + cc) * N + c] * W[(5 + b) * N + c]);
}

static double upwind(double m, double if_pos, double if_neg) {
  if (m > 0.0) return if_pos;
  if (m < 0.0) return if_neg;
  return 0.5 * (if_pos + if_neg);
}

/* Edge EMFs (Gardiner & Stone 2005, upwind "CT-contact" average).
 * E_a on the edge at the lower (b, c) corner of cell p, (a, b, c) cyclic.
 * The four faces around the edge carry E_a: faces normal to b at c-1 and c
 * (frame (b, c, a): E_a is their E_t2) and faces normal to c at b-1 and b
 * (frame (c, a, b): E_a is their E_t1).  The plain average of the four is
 * corrected by the difference of upwinded derivatives between face and
 * cell-centre values; upwinding follows the sign of the mass flux through
 * the face (contact wave), with the mean of both sides at zero. */
static void edge_emfs(const grid_t* g, const double* const F[3], const double* W, double* E) {
  size_t N = ncell(g);
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    const double* Fb = F[b];
    const double* Fc = F[c];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->n[2]; ++k)
      for (int j = 0; j < g->n[1]; ++j)
        for (int i = 0; i < g->n[0]; ++i) {
          size_t p = at(g, i, j, k);
          size_t pb = at_shift(g, i, j, k, b, -1);                  /* p - e_b */
          size_t pc = at_shift(g, i, j, k, c, -1);                  /* p - e_c */
          int q[3] = {i, j, k};
          q[b] -= 1; q[c] -= 1;
          size_t pbc = at(g, q[0], q[1], q[2]);                     /* p - e_b - e_c */
          double eb0 = Fb[6 * N + pc], eb1 = Fb[6 * N + p];         /* faces normal b at c-1, c */
          double ec0 = Fc[5 * N + pb], ec1 = Fc[5 * N + p];         /* faces normal c at b-1, b */
          double mb0 = Fb[pc], mb1 = Fb[p], mc0 = Fc[pb], mc1 = Fc[p];
          double r00 = ref_emf(W, N, pbc, a), r10 = ref_emf(W, N, pc, a);
          double r01 = ref_emf(W, N, pb, a), r11 = ref_emf(W, N, p, a);
          /* Upwinded one-sided differences (derivative times dx/2) along
           * each face, taken in the half cell next to the edge:
           *   dc1: along c on face b at c, between the edge and the face centre,
           *   dc0: along c on face b at c-1, between the face centre and the edge,
           *   db1, db0: the same along b on faces c at b and b-1.
           * Each face value is extrapolated to the edge with its derivative:
           * edge = e(b at c) - dc1 = e(b at c-1) + dc0, and likewise in b. */
          double dc1 = upwind(mb1, r01 - ec0, r11 - ec1);
          double dc0 = upwind(mb0, ec0 - r00, ec1 - r10);
          double db1 = upwind(mc1, r10 - eb0, r11 - eb1);
          double db0 = upwind(mc0, eb0 - r00, eb1 - r01);
          E[a * N + p] = 0.25 * (eb0 + eb1 + ec0 + ec1) + 0.25 * ((dc0 - dc1) + (db0 - db1));
        }
  }
}

/* Conservative update (Eq. 10) of the cell variables and CT update (Eq. 13)
 * of the face field over time tau: Uo = U - tau div F, Bo = B - tau curl E.
 * Flux differences are applied in the order x, y, z. */
static void apply_update(const grid_t* g, const double* U, const double* B, const double* const F[3],
                         const double* E, double tau, double* Uo, double* Bo) {
  size_t N = ncell(g);
  double r = tau / g->dx;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        size_t p = at(g, i, j, k);
        size_t px = at(g, i + 1, j, k), py = at(g, i, j + 1, k), pz = at(g, i, j, k + 1);
        for (int m = 0; m < 5; ++m) {
          double v = U[m * N + p];
          v -= r * (F[0][m * N + px] - F[0][m * N + p]);
          v -= r * (F[1][m * N + py] - F[1][m * N + p]);
          v -= r * (F[2][m * N + pz] - F[2][m * N + p]);
          Uo[m * N + p] = v;
        }
        const double* Ex = E;
        const double* Ey = E + N;
        const double* Ez = E + 2 * N;
        Bo[p] = B[p] - r * (Ez[py] - Ez[p]) + r * (Ey[pz] - Ey[p]);
        Bo[N + p] = B[N + p] - r * (Ex[pz] - Ex[p]) + r * (Ez[px] - Ez[p]);
        Bo[2 * N + p] = B[2 * N + p] - r * (Ey[px] - Ey[p]) + r * (Ex[py] - Ex[p]);
      }
}

/* ------------------------------------------------------------------ */
/* PPM reconstruction and CTU characteristic tracing                   */
/* (filled in mhd_oracle_ctu.c)                                        */
/* ------------------------------------------------------------------ */
int or_ctu_step_impl(int nx, int ny, int nz, double dx, double gam, int recon, int solver,
                     const double* U, const double* B, double dt, double* Uo, double* Bo,
                     int* nfallback, double* Fout, double* Eout);

/* ------------------------------------------------------------------ */
/* the VL (MUSCL-Hancock) step, paper Sec. 3.2, VL steps 1-7           */
/* ------------------------------------------------------------------ */
static int vl_step(const grid_t* g, int recon, int solver, const double* U, const double* B,
                   double dt, double* Uo, double* Bo, int* nfallback, double* Fout, double* Eout) {
  size_t N = ncell(g);
  double* W = malloc(8 * N * sizeof(double));
  double* Fd[3];
  for (int d = 0; d < 3; ++d) Fd[d] = malloc(7 * N * sizeof(double));
  double* E = malloc(3 * N * sizeof(double));
  double* Uh = malloc(5 * N * sizeof(double));
  double* Bh = malloc(3 * N * sizeof(double));
  if (!W || !Fd[0] || !Fd[1] || !Fd[2] || !E || !Uh || !Bh) return -2;
  const double* F[3] = {Fd[0], Fd[1], Fd[2]};

  /* 1. first-order fluxes with the face-centred normal field */
  primitives(g, U, B, W);
  for (int d = 0; d < 3; ++d) face_fluxes(g, d, OR_FIRST_ORDER, solver, W, B, Fd[d], nfallback);
  /* 2. edge EMFs with the time-n cell-centre reference */
  edge_emfs(g, F, W, E);
  /* 3. half-step update of U and the face field */
  apply_update(g, U, B, F, E, 0.5 * dt, Uh, Bh);
  /* 4. reconstruction at the half step, 5. Riemann fluxes */
  primitives(g, Uh, Bh, W);
  for (int d = 0; d < 3; ++d) face_fluxes(g, d, recon, solver, W, Bh, Fd[d], nfallback);
  /* 6. edge EMFs with the half-step reference */
  edge_emfs(g, F, W, E);
  /* 7. full update from time n */
  apply_update(g, U, B, F, E, dt, Uo, Bo);
  or__copy_final(N, F, E, Fout, Eout);

  free(W); free(Fd[0]); free(Fd[1]); free(Fd[2]); free(E); free(Uh); free(Bh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* ------------------------------------------------------------------ */
static grid_t mkgrid(int nx, int ny, int nz, double dx, double gam) {
  grid_t g;
  g.n[0] = nx; g.n[1] = ny; g.n[2] = nz; g.dx = dx; g.gam = gam;
  return g;
}

int or_version(void) { return 1; }

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_prim_to_cons(int nx, int ny, int nz, double gam, const double* W5, const double* B, double* U) {
  grid_t g = mkgrid(nx, ny, nz, 1.0, gam);
  size_t N = ncell(&g);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = at(&g, i, j, k);
        double bc[3];
        for (int a = 0; a < 3; ++a) bc[a] = 0.5 * (B[a * N + c] + B[a * N + at_shift(&g, i, j, k, a, 1)]);
        double d = W5[c], vx = W5[N + c], vy = W5[2 * N + c], vz = W5[3 * N + c], p = W5[4 * N + c];
        U[c] = d;
        U[N + c] = d * vx;
        U[2 * N + c] = d * vy;
        U[3 * N + c] = d * vz;
        U[4 * N + c] = p / (gam - 1.0) + 0.5 * d * (vx * vx + vy * vy + vz * vz) +
                       0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
      }
}

void or_cons_to_prim(int nx, int ny, int nz, double gam, const double* U, const double* B, double* W8) {
  grid_t g = mkgrid(nx, ny, nz, 1.0, gam);
  primitives(&g, U, B, W8);
}

/* CFL time step (Sec. 3.2; Courant factor 1/2 in Sec. 5):
 *   dt = courant * dx / max over cells of sum_d (|v_d| + c_f,d),
 * with the cell-centred field.  The Courant number is the sum over the three
 * directions: the unsplit update is stable for a summed number up to 1.
 * Returns -1 if any cell is non-physical. */
double or_cfl_dt(int nx, int ny, int nz, double dx, double gam, double courant,
                 const double* U, const double* B) {
  grid_t g = mkgrid(nx, ny, nz, dx, gam);
  size_t N = ncell(&g);
  double* W = malloc(8 * N * sizeof(double));
  primitives(&g, U, B, W);
  double smax = 0.0;
  int bad = 0;
  for (size_t c = 0; c < N; ++c) {
    double d = W[c], p = W[4 * N + c];
    if (!(d > 0.0) || !(p > 0.0)) { bad = 1; continue; }
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
      int b = (a + 1) % 3, cc = (a + 2) % 3;
      double cf = fast_speed(d, p, W[(5 + a) * N + c], W[(5 + b) * N + c], W[(5 + cc) * N + c], gam);
      s += fabs(W[(1 + a) * N + c]) + cf;
    }
    if (s > smax) smax = s;
  }
  free(W);
  if (bad) return -1.0;
  return courant * dx / smax;
}

/* discrete divergence, Eq. 16, per cell */
void or_divb(int nx, int ny, int nz, double dx, const double* B, double* div) {
  grid_t g = mkgrid(nx, ny, nz, dx, 1.0);
  size_t N = ncell(&g);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = at(&g, i, j, k);
        div[c] = (B[at(&g, i + 1, j, k)] - B[c]) / dx + (B[N + at(&g, i, j + 1, k)] - B[N + c]) / dx +
                 (B[2 * N + at(&g, i, j, k + 1)] - B[2 * N + c]) / dx;
      }
}

/* volume totals: mass, Mx, My, Mz, total energy, magnetic energy
 * (cell-centred field), kinetic energy; serial sums in storage order */
void or_sums(int nx, int ny, int nz, double dx, const double* U, const double* B, double out[7]) {
  grid_t g = mkgrid(nx, ny, nz, dx, 1.0);
  size_t N = ncell(&g);
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  double dv = dx * dx * dx;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = at(&g, i, j, k);
        for (int m = 0; m < 5; ++m) s[m] += U[m * N + c];
        double bx = 0.5 * (B[c] + B[at(&g, i + 1, j, k)]);
        double by = 0.5 * (B[N + c] + B[N + at(&g, i, j + 1, k)]);
        double bz = 0.5 * (B[2 * N + c] + B[2 * N + at(&g, i, j, k + 1)]);
        s[5] += 0.5 * (bx * bx + by * by + bz * bz);
        double mx = U[N + c], my = U[2 * N + c], mz = U[3 * N + c];
        s[6] += 0.5 * (mx * mx + my * my + mz * mz) / U[c];
      }
  for (int m = 0; m < 7; ++m) out[m] = s[m] * dv;
}

int or_step(int nx, int ny, int nz, double dx, double gam, int scheme, int recon, int solver,
            const double* U, const double* B, double dt, double* Uo, double* Bo, int* nfallback) {
  return or_step_ex(nx, ny, nz, dx, gam, scheme, recon, solver, U, B, dt, Uo, Bo, nfallback, NULL, NULL);
}

int or_step_ex(int nx, int ny, int nz, double dx, double gam, int scheme, int recon, int solver,
               const double* U, const double* B, double dt, double* Uo, double* Bo, int* nfallback,
               double* Fout, double* Eout) {
  grid_t g = mkgrid(nx, ny, nz, dx, gam);
  int fb = 0;
  int rc;
  if (scheme == OR_VL) {
    /* no unlimited PPM: without limiting or tracing both sides of a face
     * take the same interface value, a central scheme without dissipation */
    if (recon != OR_PLM && recon != OR_FIRST_ORDER && recon != OR_PLM_UNLIMITED && recon != OR_PPM) return -1;
    rc = vl_step(&g, recon, solver, U, B, dt, Uo, Bo, &fb, Fout, Eout);
  } else if (scheme == OR_CTU) {
    rc = or_ctu_step_impl(nx, ny, nz, dx, gam, recon, solver, U, B, dt, Uo, Bo, &fb, Fout, Eout);
  } else {
    return -1;
  }
  if (nfallback) *nfallback = fb;
  return rc;
}

/* ---- 1D entry points for unit tests ---- */
void or_phys_flux(double gam, const double* w, double bn, double* f) { phys_flux(w, bn, gam, f); }
void or_w_to_u(double gam, const double* w, double bn, double* u) { w_to_u(w, bn, gam, u); }
void or_u_to_w(double gam, const double* u, double bn, double* w) { u_to_w(u, bn, gam, w); }
double or_fast_speed(double gam, const double* w, double bn) {
  return fast_speed(w[0], w[4], bn, w[5], w[6], gam);
}
int or_riemann(int solver, double gam, const double* wl, const double* wr, double bn, double* f) {
  return riemann(solver, wl, wr, bn, gam, f);
}
void or_roe_eigen(double gam, const double* wl, const double* wr, double bn, double* lam, double* R) {
  double Rm[7][7];
  roe_eigensystem(wl, wr, bn, gam, lam, Rm);
  memcpy(R, Rm, sizeof Rm);
}

/* internal helpers exposed to the CTU translation unit */
void or__primitives(int nx, int ny, int nz, double dx, double gam, const double* U, const double* B, double* W) {
  grid_t g = mkgrid(nx, ny, nz, dx, gam);
  primitives(&g, U, B, W);
}
int or__riemann(int solver, const double* wl, const double* wr, double bn, double gam, double* f) {
  return riemann(solver, wl, wr, bn, gam, f);
}
void or__edge_emfs(int nx, int ny, int nz, double dx, const double* const F[3], const double* W, double* E) {
  grid_t g = mkgrid(nx, ny, nz, dx, 1.0);
  edge_emfs(&g, F, W, E);
}
void or__apply_update(int nx, int ny, int nz, double dx, const double* U, const double* B,
                      const double* const F[3], const double* E, double tau, double* Uo, double* Bo) {
  grid_t g = mkgrid(nx, ny, nz, dx, 1.0);
  apply_update(&g, U, B, F, E, tau, Uo, Bo);
}
/* the hydro components of the update's fluxes and its edge EMFs, if asked for */
void or__copy_final(size_t N, const double* const F[3], const double* E, double* Fout, double* Eout) {
  if (Fout)
    for (int d = 0; d < 3; ++d) memcpy(Fout + (size_t)d * 5 * N, F[d], 5 * N * sizeof(double));
  if (Eout) memcpy(Eout, E, 3 * N * sizeof(double));
}
