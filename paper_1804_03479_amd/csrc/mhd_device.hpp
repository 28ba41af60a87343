// mhd_device.hpp -- device building blocks of the unsplit MHD update for
// gfx950: equation of state, physical flux, Riemann solvers and limited
// reconstruction.  Everything is templated on the arithmetic type T
// (double or float) and inlined into the stage kernels.
//
// A one-dimensional state along a face normal n uses the cyclic frame
// (n, t1, t2): x-faces (x, y, z), y-faces (y, z, x), z-faces (z, x, y).
//   primitive  w = (rho, vn, vt1, vt2, p, Bt1, Bt2), normal field bn apart
//   flux       f = (rho, Mn, Mt1, Mt2, e, Bt1, Bt2) components of Eqs. 7-9.
#pragma once
#include <hip/hip_runtime.h>

namespace mhd {

template <typename T> __device__ __forceinline__ T dsqrt(T x);
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }
// 1/sqrt(x): one v_rsq in float (1 ulp), the divided square root in double
template <typename T> __device__ __forceinline__ T drsqrt(T x);
template <> __device__ __forceinline__ double drsqrt<double>(double x) { return 1.0 / sqrt(x); }
template <> __device__ __forceinline__ float drsqrt<float>(float x) { return rsqrtf(x); }
template <typename T> __device__ __forceinline__ T dabs(T x) { return x < T(0) ? -x : x; }
template <typename T> __device__ __forceinline__ T dmin(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ __forceinline__ T dmax(T a, T b) { return a > b ? a : b; }

// total energy density, Eq. 5
template <typename T>
__device__ __forceinline__ T energy(const T w[7], T bn, T gm1inv) {
  return w[4] * gm1inv + T(0.5) * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) +
         T(0.5) * (bn * bn + w[5] * w[5] + w[6] * w[6]);
}

// conserved state and physical flux of a 1D primitive state (Eqs. 6-7)
template <typename T>
__device__ __forceinline__ void state_and_flux(const T w[7], T bn, T gm1inv, T u[7], T f[7]) {
  const T d = w[0], vn = w[1], v1 = w[2], v2 = w[3], p = w[4], b1 = w[5], b2 = w[6];
  const T pt = p + T(0.5) * (bn * bn + b1 * b1 + b2 * b2);
  const T e = energy(w, bn, gm1inv);
  const T vb = vn * bn + v1 * b1 + v2 * b2;
  u[0] = d; u[1] = d * vn; u[2] = d * v1; u[3] = d * v2; u[4] = e; u[5] = b1; u[6] = b2;
  f[0] = d * vn;
  f[1] = d * vn * vn + pt - bn * bn;
  f[2] = d * vn * v1 - bn * b1;
  f[3] = d * vn * v2 - bn * b2;
  f[4] = (e + pt) * vn - bn * vb;
  f[5] = b1 * vn - bn * v1;
  f[6] = b2 * vn - bn * v2;
}

// fast magnetosonic speed along the normal, cancellation-free root
template <typename T>
__device__ __forceinline__ T fast_speed(T d, T p, T bn, T b1, T b2, T gam) {
  const T id = T(1) / d;
  const T asq = gam * p * id;
  const T btsq = (b1 * b1 + b2 * b2) * id;
  const T bsq = bn * bn * id + btsq;
  const T df = asq - bsq;
  return dsqrt(T(0.5) * (asq + bsq + dsqrt(df * df + T(4) * asq * btsq)));
}

// ---------------------------------------------------------------- HLLE
template <typename T>
__device__ __forceinline__ void hlle_from(const T wl[7], const T wr[7], const T ul[7], const T ur[7],
                                          const T fl[7], const T fr[7], T bn, T gam, T f[7]) {
  const T cfl = fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gam);
  const T cfr = fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gam);
  const T sl = dmin(wl[1] - cfl, wr[1] - cfr);
  const T sr = dmax(wl[1] + cfl, wr[1] + cfr);
  if (sl >= T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fl[m];
  } else if (sr <= T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fr[m];
  } else {
    const T inv = T(1) / (sr - sl);
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = (sr * fl[m] - sl * fr[m] + sl * sr * (ur[m] - ul[m])) * inv;
  }
}

template <typename T>
__device__ __forceinline__ void riemann_hlle(const T wl[7], const T wr[7], T bn, T gam, T f[7]) {
  const T gm1inv = T(1) / (gam - T(1));
  T ul[7], ur[7], fl[7], fr[7];
  state_and_flux(wl, bn, gm1inv, ul, fl);
  state_and_flux(wr, bn, gm1inv, ur, fr);
  hlle_from(wl, wr, ul, ur, fl, fr, bn, gam, f);
}

// ---------------------------------------------------------------- Roe
// Linearisation with sqrt(rho)-weighted velocity and enthalpy, geometric
// density and opposite-side-weighted transverse field (Cargo & Gallice
// 1997); the Roe matrix is the Jacobian at that state with the density
// derivative of P* shifted by -(gam-2) X.  Right eigenvectors with the
// Roe & Balsara (1996) normalisation, left eigenvectors their analytic
// inverse.  Wave strengths alpha_k = l_k . (U_R - U_L) are formed wave by
// wave, so neither matrix is ever held in registers.  If a state between
// waves has rho <= 0 or p <= 0 the HLLE flux is returned (fallback = 1).
template <typename T>
__device__ __forceinline__ int riemann_roe(const T wl[7], const T wr[7], T bn, T gam, T f[7]) {
  const T g1 = gam - T(1), g2 = gam - T(2);
  const T gm1inv = T(1) / g1;
  T ul[7], ur[7], fl[7], fr[7];
  state_and_flux(wl, bn, gm1inv, ul, fl);
  state_and_flux(wr, bn, gm1inv, ur, fr);

  const T sl = dsqrt(wl[0]), sr = dsqrt(wr[0]);
  const T isum = T(1) / (sl + sr);
  const T d = sl * sr;
  const T vx = (sl * wl[1] + sr * wr[1]) * isum;
  const T vy = (sl * wl[2] + sr * wr[2]) * isum;
  const T vz = (sl * wl[3] + sr * wr[3]) * isum;
  const T ptl = wl[4] + T(0.5) * (bn * bn + wl[5] * wl[5] + wl[6] * wl[6]);
  const T ptr = wr[4] + T(0.5) * (bn * bn + wr[5] * wr[5] + wr[6] * wr[6]);
  const T h = (sl * ((ul[4] + ptl) / wl[0]) + sr * ((ur[4] + ptr) / wr[0])) * isum;
  const T by = (sr * wl[5] + sl * wr[5]) * isum;
  const T bz = (sr * wl[6] + sl * wr[6]) * isum;
  const T dby = wr[5] - wl[5], dbz = wr[6] - wl[6];
  const T X = T(0.5) * (dby * dby + dbz * dbz) * isum * isum;

  const T vsq = vx * vx + vy * vy + vz * vz;
  const T btsq = by * by + bz * bz;
  const T id = T(1) / d;
  const T casq = bn * bn * id;
  const T hp = h - (casq + btsq * id);
  const T asq = g1 * (hp - T(0.5) * vsq) - g2 * X;
  if (!(asq > T(0))) {
    hlle_from(wl, wr, ul, ur, fl, fr, bn, gam, f);
    return 1;
  }
  const T ctsq = btsq * id;
  const T sum = casq + ctsq + asq;
  const T dif = casq + ctsq - asq;
  const T cfsq = T(0.5) * (sum + dsqrt(dif * dif + T(4) * asq * ctsq));
  const T cssq = asq * casq / cfsq;
  const T cf = dsqrt(cfsq), cs = dsqrt(cssq), ca = dsqrt(casq);
  const T bt = dsqrt(btsq);
  T b2, b3;
  if (bt > T(0)) {
    const T ibt = T(1) / bt;
    b2 = by * ibt;
    b3 = bz * ibt;
  } else {
    b2 = T(0.70710678118654752440);
    b3 = T(0.70710678118654752440);
  }
  T af, as;
  if (cfsq - cssq <= T(0)) { af = T(1); as = T(0); }
  else if (asq - cssq <= T(0)) { af = T(0); as = T(1); }
  else if (cfsq - asq <= T(0)) { af = T(1); as = T(0); }
  else {
    const T inv = T(1) / (cfsq - cssq);
    af = dsqrt((asq - cssq) * inv);
    as = dsqrt((cfsq - asq) * inv);
  }
  const T sqd = dsqrt(d), isqd = T(1) / sqd;
  const T s = bn >= T(0) ? T(1) : T(-1);
  const T a = dsqrt(asq);
  // right-eigenvector coefficients
  const T qf = cf * af * s, qs = cs * as * s;
  const T afp = af * a * isqd, asp = as * a * isqd;
  const T vbet = vy * b2 + vz * b3;
  const T afpb = afp * bt, aspb = asp * bt;
  // left-eigenvector coefficients
  const T nrm = T(0.5) / asq;
  const T Cff = nrm * af * cf, Css = nrm * as * cs;
  const T Qf = nrm * qf, Qs = nrm * qs;
  const T Af = nrm * af * a * sqd, As = nrm * as * a * sqd;
  const T lafpb = nrm * afpb, laspb = nrm * aspb;
  const T gf = g1 * nrm * af, gs = g1 * nrm * as;
  const T hvd = vsq - hp;
  const T nn = T(1) / asq;

  T du[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) du[m] = ur[m] - ul[m];
  T diss[7], us[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) { diss[m] = T(0); us[m] = ul[m]; }
  int bad = 0;

  auto wave = [&](int k, T lam, const T l[7], const T r[7]) {
    T alpha = T(0);
#pragma unroll
    for (int m = 0; m < 7; ++m) alpha += l[m] * du[m];
    const T c = dabs(lam) * alpha;
#pragma unroll
    for (int m = 0; m < 7; ++m) diss[m] += c * r[m];
    if (k < 6) {
#pragma unroll
      for (int m = 0; m < 7; ++m) us[m] += alpha * r[m];
      const T pint = g1 * (us[4] - T(0.5) * (us[1] * us[1] + us[2] * us[2] + us[3] * us[3]) / us[0] -
                           T(0.5) * (bn * bn + us[5] * us[5] + us[6] * us[6]));
      if (!(us[0] > T(0)) || !(pint > T(0))) bad = 1;
    }
  };
  {  // u - cf
    const T l[7] = {gf * hvd + Cff * (cf + vx) - Qs * vbet - laspb, -gf * vx - Cff, -gf * vy + Qs * b2,
                    -gf * vz + Qs * b3, gf, As * b2 - gf * by, As * b3 - gf * bz};
    const T r[7] = {af, af * (vx - cf), af * vy + qs * b2, af * vz + qs * b3,
                    af * (hp - vx * cf) + qs * vbet + aspb, asp * b2, asp * b3};
    wave(0, vx - cf, l, r);
  }
  {  // u - ca
    const T l[7] = {T(0.5) * (vy * b3 - vz * b2), T(0), T(-0.5) * b3, T(0.5) * b2, T(0),
                    T(-0.5) * sqd * b3 * s, T(0.5) * sqd * b2 * s};
    const T r[7] = {T(0), T(0), -b3, b2, -(vy * b3 - vz * b2), -s * b3 * isqd, s * b2 * isqd};
    wave(1, vx - ca, l, r);
  }
  {  // u - cs
    const T l[7] = {gs * hvd + Css * (cs + vx) + Qf * vbet + lafpb, -gs * vx - Css, -gs * vy - Qf * b2,
                    -gs * vz - Qf * b3, gs, -Af * b2 - gs * by, -Af * b3 - gs * bz};
    const T r[7] = {as, as * (vx - cs), as * vy - qf * b2, as * vz - qf * b3,
                    as * (hp - vx * cs) - qf * vbet - afpb, -afp * b2, -afp * b3};
    wave(2, vx - cs, l, r);
  }
  {  // u (entropy)
    const T l[7] = {T(1) - nn * (T(0.5) * g1 * vsq - g2 * X), nn * g1 * vx, nn * g1 * vy, nn * g1 * vz,
                    -nn * g1, nn * g1 * by, nn * g1 * bz};
    const T r[7] = {T(1), vx, vy, vz, T(0.5) * vsq + g2 * X / g1, T(0), T(0)};
    wave(3, vx, l, r);
  }
  {  // u + cs
    const T l[7] = {gs * hvd + Css * (cs - vx) - Qf * vbet + lafpb, -gs * vx + Css, -gs * vy + Qf * b2,
                    -gs * vz + Qf * b3, gs, -Af * b2 - gs * by, -Af * b3 - gs * bz};
    const T r[7] = {as, as * (vx + cs), as * vy + qf * b2, as * vz + qf * b3,
                    as * (hp + vx * cs) + qf * vbet - afpb, -afp * b2, -afp * b3};
    wave(4, vx + cs, l, r);
  }
  {  // u + ca
    const T l[7] = {T(-0.5) * (vy * b3 - vz * b2), T(0), T(0.5) * b3, T(-0.5) * b2, T(0),
                    T(-0.5) * sqd * b3 * s, T(0.5) * sqd * b2 * s};
    const T r[7] = {T(0), T(0), b3, -b2, (vy * b3 - vz * b2), -s * b3 * isqd, s * b2 * isqd};
    wave(5, vx + ca, l, r);
  }
  {  // u + cf
    const T l[7] = {gf * hvd + Cff * (cf - vx) + Qs * vbet - laspb, -gf * vx + Cff, -gf * vy - Qs * b2,
                    -gf * vz - Qs * b3, gf, As * b2 - gf * by, As * b3 - gf * bz};
    const T r[7] = {af, af * (vx + cf), af * vy - qs * b2, af * vz - qs * b3,
                    af * (hp + vx * cf) - qs * vbet + aspb, asp * b2, asp * b3};
    wave(6, vx + cf, l, r);
  }
  if (bad) {
    hlle_from(wl, wr, ul, ur, fl, fr, bn, gam, f);
    return 1;
  }
#pragma unroll
  for (int m = 0; m < 7; ++m) f[m] = T(0.5) * (fl[m] + fr[m]) - T(0.5) * diss[m];
  return 0;
}

// ---------------------------------------------------------------- HLLD
// Miyoshi & Kusano (2005).  Outer speeds S_L = min(uL, uR) - max(cfL, cfR),
// S_R = max(uL, uR) + max(cfL, cfR); contact S_M; rotational speeds
// S*_{L,R} = S_M -/+ |bn| / sqrt(rho*).
template <typename T>
__device__ __forceinline__ void hlld_star(const T w[7], const T u[7], T bn, T S, T SM, T pts, T us[7]) {
  const T d = w[0], vn = w[1];
  const T sv = S - vn, sm = S - SM;
  const T ism = T(1) / sm;
  const T ds = d * sv * ism;
  const T q = d * sv * sm;
  const T den = q - bn * bn;
  T v1, v2, b1, b2;
  // degenerate switch (S = S*, Miyoshi & Kusano 2005): set well above the
  // arithmetic's rounding level, which q - bn^2 inherits from S and SM -- in
  // float a relative 1e-12 is below the noise and the division amplifies it
  const T eps = sizeof(T) == 4 ? T(1e-5) : T(1e-12);
  if (dabs(den) <= eps * (dabs(q) + bn * bn)) {
    v1 = w[2]; v2 = w[3]; b1 = w[5]; b2 = w[6];
  } else {
    const T iden = T(1) / den;
    const T mf = bn * (SM - vn) * iden;
    const T bf = (d * sv * sv - bn * bn) * iden;
    v1 = w[2] - w[5] * mf;
    v2 = w[3] - w[6] * mf;
    b1 = w[5] * bf;
    b2 = w[6] * bf;
  }
  const T pt = w[4] + T(0.5) * (bn * bn + w[5] * w[5] + w[6] * w[6]);
  const T vb = vn * bn + w[2] * w[5] + w[3] * w[6];
  const T vbs = SM * bn + v1 * b1 + v2 * b2;
  const T es = (sv * u[4] - pt * vn + pts * SM + bn * (vb - vbs)) * ism;
  us[0] = ds; us[1] = ds * SM; us[2] = ds * v1; us[3] = ds * v2; us[4] = es; us[5] = b1; us[6] = b2;
}

template <typename T>
__device__ __forceinline__ void riemann_hlld(const T wl[7], const T wr[7], T bn, T gam, T f[7]) {
  const T gm1inv = T(1) / (gam - T(1));
  T ul[7], ur[7], fl[7], fr[7];
  state_and_flux(wl, bn, gm1inv, ul, fl);
  state_and_flux(wr, bn, gm1inv, ur, fr);
  const T cmax = dmax(fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gam),
                      fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gam));
  const T SL = dmin(wl[1], wr[1]) - cmax;
  const T SR = dmax(wl[1], wr[1]) + cmax;
  if (SL >= T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fl[m];
    return;
  }
  if (SR <= T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fr[m];
    return;
  }
  const T ptl = wl[4] + T(0.5) * (bn * bn + wl[5] * wl[5] + wl[6] * wl[6]);
  const T ptr = wr[4] + T(0.5) * (bn * bn + wr[5] * wr[5] + wr[6] * wr[6]);
  const T ml = wl[0] * (SL - wl[1]);
  const T mr = wr[0] * (SR - wr[1]);
  const T SM = (mr * wr[1] - ml * wl[1] - ptr + ptl) / (mr - ml);
  const T pts = ptl + ml * (SM - wl[1]);
  T usl[7], usr[7];
  hlld_star(wl, ul, bn, SL, SM, pts, usl);
  hlld_star(wr, ur, bn, SR, SM, pts, usr);
  const T isdl = drsqrt(usl[0]), isdr = drsqrt(usr[0]);
  const T sdl = usl[0] * isdl, sdr = usr[0] * isdr;
  const T SLs = SM - dabs(bn) * isdl;
  const T SRs = SM + dabs(bn) * isdr;
  if (SLs >= T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fl[m] + SL * (usl[m] - ul[m]);
    return;
  }
  if (SRs <= T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fr[m] + SR * (usr[m] - ur[m]);
    return;
  }
  const T sgn = bn >= T(0) ? T(1) : T(-1);
  const T iden = T(1) / (sdl + sdr);
  const T idl = isdl * isdl, idr = isdr * isdr;
  const T v1l = usl[2] * idl, v2l = usl[3] * idl;
  const T v1r = usr[2] * idr, v2r = usr[3] * idr;
  const T v1ss = (sdl * v1l + sdr * v1r + (usr[5] - usl[5]) * sgn) * iden;
  const T v2ss = (sdl * v2l + sdr * v2r + (usr[6] - usl[6]) * sgn) * iden;
  const T b1ss = (sdl * usr[5] + sdr * usl[5] + sdl * sdr * (v1r - v1l) * sgn) * iden;
  const T b2ss = (sdl * usr[6] + sdr * usl[6] + sdl * sdr * (v2r - v2l) * sgn) * iden;
  const T vbss = SM * bn + v1ss * b1ss + v2ss * b2ss;
  if (SM >= T(0)) {
    const T vbl = SM * bn + v1l * usl[5] + v2l * usl[6];
    const T uss[7] = {usl[0], usl[0] * SM, usl[0] * v1ss, usl[0] * v2ss,
                      usl[4] - sdl * (vbl - vbss) * sgn, b1ss, b2ss};
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fl[m] + SL * (usl[m] - ul[m]) + SLs * (uss[m] - usl[m]);
  } else {
    const T vbr = SM * bn + v1r * usr[5] + v2r * usr[6];
    const T uss[7] = {usr[0], usr[0] * SM, usr[0] * v1ss, usr[0] * v2ss,
                      usr[4] + sdr * (vbr - vbss) * sgn, b1ss, b2ss};
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fr[m] + SR * (usr[m] - ur[m]) + SRs * (uss[m] - usr[m]);
  }
}

template <int SOLVER, typename T>
__device__ __forceinline__ int riemann(const T wl[7], const T wr[7], T bn, T gam, T f[7]) {
  if constexpr (SOLVER == 0) {
    return riemann_roe(wl, wr, bn, gam, f);
  } else if constexpr (SOLVER == 1) {
    riemann_hlle(wl, wr, bn, gam, f);
    return 0;
  } else {
    riemann_hlld(wl, wr, bn, gam, f);
    return 0;
  }
}

// minmod limiter: 0 if the one-sided differences differ in sign (or one is
// zero), else the smaller in magnitude -- the median of a, b and 0: one
// v_med3_f32 in float; in double the sum of max(min(a, b), 0) and
// min(max(a, b), 0), of which one term is exactly zero (no compare and
// select chains)
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
  } else {
    return fmax(fmin(a, b), T(0)) + fmin(fmax(a, b), T(0));
  }
}

// monotonised-central slope of q0 between neighbours qm and qp: 0 where the
// one-sided differences dl, dr differ in sign, else the central difference
// dc limited to twice the smaller one-sided one -- minmod(dc, 2 minmod(dl,
// dr)), since dc has the sign of dl and dr where they agree
template <typename T>
__device__ __forceinline__ T mc_slope(T qm, T q0, T qp) {
  const T dl = q0 - qm, dr = qp - q0;
  const T dc = T(0.5) * (qp - qm);
  return minmod(dc, T(2) * minmod(dl, dr));
}

// PPM (Colella & Woodward 1984) interface value between cells a and b (a
// below) from their values and MC-limited slopes
template <typename T>
__device__ __forceinline__ T ppm_interface(T qa, T qb, T sa, T sb) {
  return T(0.5) * (qa + qb) - (sb - sa) * T(1.0 / 6.0);
}

// median of three values (one v_med3_f32 in float)
template <typename T>
__device__ __forceinline__ T med3(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_amdgcn_fmed3f(a, b, c);
  } else {
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
  }
}

// PPM monotonicity constraints on a cell's parabola (centre value c, edge
// values l and r): flat at an extremum, otherwise an edge more than twice as
// far from c as the other is pulled in to 3c - 2(other edge), so the
// parabola takes no value outside [l, r].  Written as medians: l becomes the
// median of l, c and c - 2 (r - c), r likewise -- at an extremum (l and r on
// the same side of c) both medians are c; otherwise the median keeps l
// unless it lies beyond c - 2 (r - c).  (The usual form compares
// (r - l)(c - (l + r)/2) with (r - l)^2 / 6; the two tests are the same
// inequality.)
template <typename T>
__device__ __forceinline__ void ppm_limit(T c, T& l, T& r) {
  const T l0 = l, r0 = r;
  l = med3(l0, c, c - T(2) * (r0 - c));
  r = med3(r0, c, c - T(2) * (l0 - c));
}

// PPM edge values of the centre of q0..q4: interface values from
// MC-limited slopes, then the monotonicity constraints
template <typename T>
__device__ __forceinline__ void ppm_edges(T q0, T q1, T q2, T q3, T q4, T& ql, T& qr) {
  const T dm = mc_slope(q0, q1, q2), d0 = mc_slope(q1, q2, q3), dp = mc_slope(q2, q3, q4);
  T l = ppm_interface(q1, q2, dm, d0);
  T r = ppm_interface(q2, q3, d0, dp);
  ppm_limit(q2, l, r);
  ql = l;
  qr = r;
}

// Characteristic tracing of one cell for the CTU predictor (Colella 1990):
// c holds the cell's 1D primitive state, sl / sr its reconstructed lower and
// upper edge values on entry (the profile's two ends) and the traced edge
// states on return, (bn_lo, bn_hi) the cell's two normal-face fields.  Each
// edge state starts at the reconstructed edge value; every wave moving
// toward that edge subtracts its share of the profile's average over its
// domain of dependence during dt (xi = lam dt/dx).  ALLW (the HLL-family
// solvers, which do not resolve every wave): waves moving away are traced as
// well, with the profile continued past the edge, so both states of a face
// are time-centred in every field.  Then the transverse field gets
// (dt/2) v_t dBn/dn.  A non-physical result falls back to the cell state.
template <typename T, bool ALLW>
__device__ __forceinline__ void trace_edges(const T c[7], T bn_lo, T bn_hi, T dtdx, T gam, T sl[7], T sr[7]) {
  T dq[7], q6[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    dq[m] = sr[m] - sl[m];
    q6[m] = T(6) * (c[m] - T(0.5) * (sl[m] + sr[m]));
  }
  // primitive eigen-system of the cell (Roe & Balsara normalisation)
  const T d = c[0], u = c[1], p = c[4], by = c[5], bz = c[6];
  const T bn = T(0.5) * (bn_lo + bn_hi);
  const T isd = drsqrt(d), sd = d * isd, id = isd * isd;
  const T asq = gam * p * id, a = dsqrt(asq);
  const T btsq = by * by + bz * bz;
  const T casq = bn * bn * id, ctsq = btsq * id;
  const T sum = asq + casq + ctsq, dif = casq + ctsq - asq;
  const T cfsq = T(0.5) * (sum + dsqrt(dif * dif + T(4) * asq * ctsq));
  const T cssq = asq * casq / cfsq;
  const T cf = dsqrt(cfsq), cs = dsqrt(cssq), ca = dabs(bn) * isd;
  T b2, b3;
  if (btsq > T(0)) {
    const T ib = drsqrt(btsq);
    b2 = by * ib;
    b3 = bz * ib;
  } else {
    b2 = T(0.70710678118654752440);
    b3 = T(0.70710678118654752440);
  }
  T af, as;
  if (cfsq - cssq <= T(0)) { af = T(1); as = T(0); }
  else if (asq - cssq <= T(0)) { af = T(0); as = T(1); }
  else if (cfsq - asq <= T(0)) { af = T(1); as = T(0); }
  else {
    const T inv = T(1) / (cfsq - cssq);
    af = dsqrt((asq - cssq) * inv);
    as = dsqrt((cfsq - asq) * inv);
  }
  const T sg = bn >= T(0) ? T(1) : T(-1);
  const T Cff = cf * af, Css = cs * as, Qf = cf * af * sg, Qs = cs * as * sg, Af = a * af * sd, As = a * as * sd;
  const T iasq = T(1) / asq, nrm = T(0.5) * iasq;
  // The left and right eigenvectors of the waves u -+ c (c = cf, ca, cs)
  // differ only in the sign of an antisymmetric part: l = S -+ A, r = Rs -+ Ra.
  // So each pair needs the projections S.x and A.x of x = dq, q6, and the
  // two waves' amplitudes enter each edge as (sum) Rs + (difference) Ra.
  // Transverse projections of the velocity (2, 3) and field (5, 6) parts:
  const T pv_d = b2 * dq[2] + b3 * dq[3], pb_d = b2 * dq[5] + b3 * dq[6];
  const T xv_d = b2 * dq[3] - b3 * dq[2], xb_d = b2 * dq[6] - b3 * dq[5];
  const T pv_6 = b2 * q6[2] + b3 * q6[3], pb_6 = b2 * q6[5] + b3 * q6[6];
  const T xv_6 = b2 * q6[3] - b3 * q6[2], xb_6 = b2 * q6[6] - b3 * q6[5];
  // amplitudes at the upper (R) and lower (L) edge of a wave with
  // xi = lam dt/dx and projections (ad, a6): zero for waves moving away,
  // or (ALLW) the profile continued past the edge for them too
  auto amps = [&](T lam, T ad, T a6, T& aR, T& aL) {
    const T xi = lam * dtdx;
    aR = T(0.5) * (ALLW ? xi : dmax(xi, T(0))) * (ad - (T(1) - T(2.0 / 3.0) * xi) * a6);
    aL = T(0.5) * (ALLW ? -xi : dmax(-xi, T(0))) * (ad + (T(1) + T(2.0 / 3.0) * xi) * a6);
  };
  // a wave pair (lam -+ c): returns the sums and differences of the amplitudes
  auto pair = [&](T c, T s_d, T a_d, T s_6, T a_6, T& sR, T& dR, T& sL, T& dL) {
    T rm, lm, rp, lp;
    amps(u - c, s_d - a_d, s_6 - a_6, rm, lm);
    amps(u + c, s_d + a_d, s_6 + a_6, rp, lp);
    sR = rm + rp; dR = rp - rm;
    sL = lm + lp; dL = lp - lm;
  };
  T fsR, fdR, fsL, fdL, ssR, sdR, ssL, sdL, asR, adR, asL, adL, eR, eL;
  pair(cf, nrm * (af * id * dq[4] + As * id * pb_d), nrm * (Cff * dq[1] - Qs * pv_d),
       nrm * (af * id * q6[4] + As * id * pb_6), nrm * (Cff * q6[1] - Qs * pv_6), fsR, fdR, fsL, fdL);
  pair(cs, nrm * (as * id * dq[4] - Af * id * pb_d), nrm * (Css * dq[1] + Qf * pv_d),
       nrm * (as * id * q6[4] - Af * id * pb_6), nrm * (Css * q6[1] + Qf * pv_6), ssR, sdR, ssL, sdL);
  pair(ca, T(0.5) * sg * isd * xb_d, T(-0.5) * xv_d, T(0.5) * sg * isd * xb_6, T(-0.5) * xv_6, asR, adR, asL,
       adL);
  amps(u, dq[0] - dq[4] * iasq, q6[0] - q6[4] * iasq, eR, eL);
  // edge += sign * sum over waves of amplitude * right eigenvector
  auto update = [&](T s[7], T sgn, T fS, T fD, T sS, T sD, T aS, T aD, T e) {
    const T ms = af * fS + as * sS, mv = Qf * sD - Qs * fD, mb = As * fS - Af * sS;
    s[0] += sgn * (d * ms + e);
    s[1] += sgn * (Cff * fD + Css * sD);
    s[2] += sgn * (b2 * mv + b3 * aD);
    s[3] += sgn * (b3 * mv - b2 * aD);
    s[4] += sgn * (d * asq * ms);
    s[5] += sgn * (b2 * mb - sg * sd * b3 * aS);
    s[6] += sgn * (b3 * mb + sg * sd * b2 * aS);
  };
  update(sr, T(-1), fsR, fdR, ssR, sdR, asR, adR, eR);
  update(sl, T(1), fsL, fdL, ssL, sdL, asL, adL, eL);
  // multidimensional source term of the transverse field
  const T hb = T(0.5) * dtdx * (bn_hi - bn_lo);   // (dt/2) dBn/dn
  sl[5] += hb * c[2];
  sl[6] += hb * c[3];
  sr[5] += hb * c[2];
  sr[6] += hb * c[3];
  if (!(sl[0] > T(0)) || !(sl[4] > T(0))) {
#pragma unroll
    for (int m = 0; m < 7; ++m) sl[m] = c[m];
  }
  if (!(sr[0] > T(0)) || !(sr[4] > T(0))) {
#pragma unroll
    for (int m = 0; m < 7; ++m) sr[m] = c[m];
  }
}

// trace_cell: the same from the primitive states q[s][m] of cells -2..2
// along the direction (RECON 0: minmod PLM edges, 1: PPM edges)
template <typename T, int RECON, bool ALLW>
__device__ __forceinline__ void trace_cell(const T q[5][7], T bn_lo, T bn_hi, T dtdx, T gam, T sl[7],
                                           T sr[7]) {
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    if (RECON == 1) {
      ppm_edges(q[0][m], q[1][m], q[2][m], q[3][m], q[4][m], sl[m], sr[m]);
    } else {
      const T s = minmod(q[2][m] - q[1][m], q[3][m] - q[2][m]);
      sl[m] = q[2][m] - T(0.5) * s;
      sr[m] = q[2][m] + T(0.5) * s;
    }
  }
  trace_edges<T, ALLW>(q[2], bn_lo, bn_hi, dtdx, gam, sl, sr);
}

}  // namespace mhd
