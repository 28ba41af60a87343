// mhd_mlp.hpp -- the learned interface flux: a 15 -> 64 -> 64 -> 7 GELU
// network that stands in for HLLD at smooth interfaces (HLLD stays in use
// where the pressure or density jump exceeds a threshold), its training
// kernels, and the capture of interface samples.  BF16 operands, FP32
// accumulation on the MFMA units (v_mfma_f32_16x16x16_bf16, and for the
// 64-deep layers of inference v_mfma_f32_16x16x32_bf16).
//
// Features: the mean of the two face-frame primitive states (rho, vn, vt1,
// vt2, p, Bt1, Bt2), the unit jump and the jump size s, and Bn, all in units
// of rho0 = (rhoL + rhoR)/2, p0 = (pL + pR)/2, v0 = sqrt(p0/rho0),
// B0 = sqrt(p0) (layout at mlp_features); outputs: the dissipative part of
// the flux, F - (F(wl) + F(wr))/2, divided by s (rho0 v0, p0, p0, p0, p0 v0,
// B0 v0, B0 v0); the central part is computed exactly.  Dividing by s keeps
// the BF16 operands of order one.  The normalisation follows the scaling
// symmetry of ideal MHD, under which HLLD is covariant.
//
// Parameters (FP32 master copy, packed): W1[15][64] b1[64] W2[64][64] b2[64]
// W3[64][7] b3[7], [in][out] row-major, 5639 values.
//
// MFMA 16x16x16 operand layout (lane l, 64 lanes): A fragment holds
// A[l % 16][4 (l / 16) + 0..3], B fragment B[4 (l / 16) + 0..3][l % 16],
// accumulator C[4 (l / 16) + 0..3][l % 16].
#pragma once
#include <hip/hip_runtime.h>

#include "mhd_device.hpp"

namespace mhd {

constexpr int kNin = 15, kNh = 64, kNout = 7;
constexpr float kTinyJump = 1e-4f;
constexpr int kParams = 15 * 64 + 64 + 64 * 64 + 64 + 64 * 7 + 7;
constexpr int oW1 = 0, ob1 = 960, oW2 = 1024, ob2 = 5120, oW3 = 5184, ob3 = 5632;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// round to the nearest bfloat16, ties to even (gfx950 converts in hardware,
// two values per v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned short f2bf(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ __forceinline__ unsigned f2bf2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2v));
}
// four floats to one MFMA BF16 operand fragment
__device__ __forceinline__ bf16x4 f2bf4(float a, float b, float c, float d) {
  return __builtin_bit_cast(bf16x4, u32x2{f2bf2(a, b), f2bf2(c, d)});
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// GELU, tanh form: 0.5 x (1 + tanh u) = x s with s = 1 / (1 + exp(-2u)),
// u = sqrt(2/pi) (x + 0.044715 x^3); exp(-2u) = 2^q with
// q = x (a + b x^2), a = -2 sqrt(2/pi) log2(e), b = 0.044715 a, so one GELU
// is three multiply-adds, v_exp_f32, an add, v_rcp_f32 and a multiply
// (the hardware reciprocal needs no range scaling: a denominator beyond
// 2^126 gives s = 0, the limit).  The derivative is
// s + 2 x s (1 - s) du/dx.
__device__ __forceinline__ float gelu_sig(float x) {
  const float a = -2.302208198144325f, b = -0.1029432395800235f;
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(x * __builtin_fmaf(b, x * x, a)));
}
__device__ __forceinline__ float gelu(float x) { return x * gelu_sig(x); }
__device__ __forceinline__ float gelu_prime(float x) {
  const float sg = gelu_sig(x);
  const float du2 = 1.5957691216057308f * (1.0f + 3.0f * 0.044715f * x * x);   // 2 du/dx
  return sg + x * sg * (1.0f - sg) * du2;
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// v_mfma_f32_16x16x32_bf16 (gfx950) on two 16-deep fragment pairs: lane l
// supplies k = 8 (l / 16) + 0..7, here the 4 values of the first pair's
// fragment followed by the 4 of the second.  Both operands take their k
// slots in that same order, so the product is the sum of the two 16-deep
// products: half the MFMA issues for the same contraction.
__device__ __forceinline__ f32x4 mfma32(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
  const bf16x8 a = __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
  const bf16x8 b = __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Inference weights as the kernels read them: transposed, BF16, padded.
//   W1t[64][16] (k = 15 zero), W2t[64][64], W3t[16][64] (rows >= 7 zero),
//   biases in FP32: b1[64], b2[64], b3[16].
struct MlpWeights {
  unsigned short W1t[64 * 16];
  unsigned short W2t[64 * 64];
  unsigned short W3t[16 * 64];
  float b1[64], b2[64], b3[16];
};

// FP32 master parameters -> inference layout
__global__ void __launch_bounds__(256) k_mlp_pack(const float* __restrict__ P, MlpWeights* __restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < 64 * 16) {
    const int n = t / 16, k = t % 16;
    out->W1t[t] = f2bf(k < kNin ? P[oW1 + k * kNh + n] : 0.0f);
  }
  if (t < 64 * 64) {
    const int n = t / 64, k = t % 64;
    out->W2t[t] = f2bf(P[oW2 + k * kNh + n]);
  }
  if (t < 16 * 64) {
    const int n = t / 64, k = t % 64;
    out->W3t[t] = f2bf(n < kNout ? P[oW3 + k * kNout + n] : 0.0f);
  }
  if (t < 64) {
    out->b1[t] = P[ob1 + t];
    out->b2[t] = P[ob2 + t];
  }
  if (t < 16) out->b3[t] = t < kNout ? P[ob3 + t] : 0.0f;
}

// Per-wave LDS staging of inference: the BF16 features of the wave's 64
// faces (one row per lane) and the 8 padded outputs of each face.
struct MlpStage {
  unsigned short X[64 * 16];
  float Y[64 * 8];
};
// LDS of one 256-thread block: the inference weights and four wave stages.
struct MlpShared {
  MlpWeights w;
  MlpStage st[4];
};

// Block-wide copy of the weights into LDS (a block barrier: every thread of
// the block calls it once, before any inference).
__device__ __forceinline__ void mlp_load_weights(MlpShared& sh, const MlpWeights* __restrict__ g) {
  const uint4* src = reinterpret_cast<const uint4*>(g);
  uint4* dst = reinterpret_cast<uint4*>(&sh.w);
  for (int t = threadIdx.x; t < (int)(sizeof(MlpWeights) / 16); t += blockDim.x) dst[t] = src[t];
  __syncthreads();
}

// ordering of LDS traffic between the lanes of one wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Normalised features of one interface (face frame) and the scales the
// network output is multiplied by.  With sc_w = (rho0, v0, v0, v0, p0, B0, B0)
// and d = (wR - wL) / sc_w, s = |d|:
//   x0 mean rho / rho0 (= 1), x1..x3 mean (vn, vt1, vt2) / v0, x4 = s,
//   x5, x6 mean (Bt1, Bt2) / B0, x7..x13 = d / s (0 when s = 0), x14 = Bn / B0;
//   osc = s * (rho0 v0, p0, p0, p0, p0 v0, B0 v0, B0 v0).
__device__ __forceinline__ void mlp_features(const float wl[7], const float wr[7], float bn, float x[16],
                                             float osc[7]) {
  const float rho0 = 0.5f * (wl[0] + wr[0]), p0 = 0.5f * (wl[4] + wr[4]);
  const float v0 = sqrtf(p0 / rho0), b0 = sqrtf(p0);
  const float inv[7] = {1.0f / rho0, 1.0f / v0, 1.0f / v0, 1.0f / v0, 1.0f / p0, 1.0f / b0, 1.0f / b0};
  float d[7], ss = 0.0f;
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    d[m] = (wr[m] - wl[m]) * inv[m];
    ss += d[m] * d[m];
  }
  const float sj = sqrtf(ss);
  const float is = sj > 0.0f ? 1.0f / sj : 0.0f;
  x[0] = 0.5f * (wl[0] + wr[0]) * inv[0];
  x[1] = 0.5f * (wl[1] + wr[1]) * inv[1];
  x[2] = 0.5f * (wl[2] + wr[2]) * inv[2];
  x[3] = 0.5f * (wl[3] + wr[3]) * inv[3];
  x[4] = sj;
  x[5] = 0.5f * (wl[5] + wr[5]) * inv[5];
  x[6] = 0.5f * (wl[6] + wr[6]) * inv[6];
#pragma unroll
  for (int m = 0; m < 7; ++m) x[7 + m] = d[m] * is;
  x[14] = bn * inv[5];
  x[15] = 0.0f;
  osc[0] = sj * rho0 * v0; osc[1] = sj * p0; osc[2] = sj * p0; osc[3] = sj * p0;
  osc[4] = sj * p0 * v0; osc[5] = sj * b0 * v0; osc[6] = sj * b0 * v0;
}

// Network output for the 64 faces of one wave (one face per lane).  All
// lanes of the wave call this together; lanes without a face pass zeros.
// The network runs transposed (H^T = W^T X^T): the weights are the A operand
// (lane (li, lk) reads W^T[16 t + li][16 s + 4 lk + 0..3] from LDS), so the
// accumulator tile of one layer is already the B operand of the next, and
// GELU and the BF16 rounding of each hidden layer act on it in registers.
// Per 16-face tile: 4 MFMA 16x16x16 (layer 1) and 8 + 2 MFMA 16x16x32.
__device__ __forceinline__ void mlp_forward_wave(MlpShared& sh, const float x[16], float y[7]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  MlpStage& S = sh.st[threadIdx.x >> 6];
  const MlpWeights& g = sh.w;
  {
    unsigned pk[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) pk[m] = f2bf2(x[2 * m], x[2 * m + 1]);
    uint4* dst = reinterpret_cast<uint4*>(S.X + lane * 16);
    dst[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    dst[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
  }
  wave_sync();
#pragma unroll 1
  for (int ft = 0; ft < 4; ++ft) {
    const bf16x4 xf = *reinterpret_cast<const bf16x4*>(S.X + (16 * ft + li) * 16 + 4 * lk);
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x4 wa = *reinterpret_cast<const bf16x4*>(g.W1t + (16 * t + li) * 16 + 4 * lk);
      const f32x4 z = mfma16(wa, xf, f32x4{0.f, 0.f, 0.f, 0.f});
      const float4 bb = *reinterpret_cast<const float4*>(g.b1 + 16 * t + 4 * lk);
      h1[t] = f2bf4(gelu(z[0] + bb.x), gelu(z[1] + bb.y), gelu(z[2] + bb.z), gelu(z[3] + bb.w));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        const unsigned short* wr = g.W2t + (16 * t + li) * 64 + 32 * kc + 4 * lk;
        z = mfma32(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16), h1[2 * kc],
                   h1[2 * kc + 1], z);
      }
      const float4 bb = *reinterpret_cast<const float4*>(g.b2 + 16 * t + 4 * lk);
      h2[t] = f2bf4(gelu(z[0] + bb.x), gelu(z[1] + bb.y), gelu(z[2] + bb.z), gelu(z[3] + bb.w));
    }
    f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const unsigned short* wr = g.W3t + li * 64 + 32 * kc + 4 * lk;
      o = mfma32(*reinterpret_cast<const bf16x4*>(wr), *reinterpret_cast<const bf16x4*>(wr + 16), h2[2 * kc],
                 h2[2 * kc + 1], o);
    }
    // lane (li, lk) holds outputs 4 lk + 0..3 of face 16 ft + li
    if (lk < 2) {
      const float4 b3 = *reinterpret_cast<const float4*>(g.b3 + 4 * lk);
      *reinterpret_cast<float4*>(S.Y + (16 * ft + li) * 8 + 4 * lk) =
          make_float4(o[0] + b3.x, o[1] + b3.y, o[2] + b3.z, o[3] + b3.w);
    }
  }
  wave_sync();
  const float4 y0 = *reinterpret_cast<const float4*>(S.Y + lane * 8);
  const float4 y1 = *reinterpret_cast<const float4*>(S.Y + lane * 8 + 4);
  y[0] = y0.x; y[1] = y0.y; y[2] = y0.z; y[3] = y0.w;
  y[4] = y1.x; y[5] = y1.y; y[6] = y1.z;
  wave_sync();   // the stage is rewritten by the next call
}

// Interface capture: (wl[7], wr[7], bn, flux[7]) of every stride-th face
struct Capture {
  float* buf;                    // [cap][22], nullptr = off
  long long cap;
  unsigned long long* count;     // device counter of attempted writes
  int stride;
};

// the record of a face (its states written), or nullptr when the face is not
// sampled or the buffer is full; capture_flux completes it
__device__ __forceinline__ float* capture_states(const Capture& cp, long long face, const float wl[7],
                                                 const float wr[7], float bn) {
  if (!cp.buf || face % cp.stride) return nullptr;
  const unsigned long long slot = atomicAdd(cp.count, 1ull);
  if ((long long)slot >= cp.cap) return nullptr;
  float* o = cp.buf + slot * 22;
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    o[m] = wl[m];
    o[7 + m] = wr[m];
  }
  o[14] = bn;
  return o;
}
__device__ __forceinline__ void capture_flux(float* o, const float f[7]) {
  if (!o) return;
#pragma unroll
  for (int m = 0; m < 7; ++m) o[15 + m] = f[m];
}
__device__ __forceinline__ void capture_face(const Capture& cp, long long face, const float wl[7], const float wr[7],
                                             float bn, const float f[7]) {
  capture_flux(capture_states(cp, face, wl, wr, bn), f);
}

// Learned flux with HLLD fallback for one face per lane (capture: face id
// `face` recorded with the flux used).  Returns 1 when the face used HLLD (a
// strong jump), 0 when it used the network.  Every lane of the wave calls it
// (lanes without a face pass active = false).  The fallback flux, or the
// exact central part, is computed before the network, so that only the flux
// and the output scales stay live across it.
__device__ __forceinline__ int mlp_or_hlld(MlpShared& sh, bool active, const float wl[7], const float wr[7], float bn,
                                           float gam, float dp, float drho, float f[7], const Capture& cp,
                                           long long face) {
  bool fall = true;
  float x[16], sc[7];
  if (active) {
    const float jp = fabsf(wr[4] - wl[4]) / fminf(wl[4], wr[4]);
    const float jr = fabsf(wr[0] - wl[0]) / fminf(wl[0], wr[0]);
    fall = (jp > dp) || (jr > drho);
  }
  float* rec = nullptr;
  if (active) rec = capture_states(cp, face, wl, wr, bn);
#pragma unroll
  for (int m = 0; m < 7; ++m) f[m] = 0.0f;
  if (active && !fall) {
    mlp_features(wl, wr, bn, x, sc);
    // the network gives the dissipative part; the central part is exact
    const float gm1inv = 1.0f / (gam - 1.0f);
    float ul[7], ur[7], fl[7], fr[7];
    state_and_flux(wl, bn, gm1inv, ul, fl);
    state_and_flux(wr, bn, gm1inv, ur, fr);
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = 0.5f * (fl[m] + fr[m]);
  } else {
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = 0.0f;
#pragma unroll
    for (int m = 0; m < 7; ++m) sc[m] = 0.0f;
    if (active) riemann_hlld(wl, wr, bn, gam, f);
  }
  float y[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // the network runs when any lane of the wave needs it (wave-uniform test)
  if (__ballot(active && !fall) != 0ull) mlp_forward_wave(sh, x, y);
  if (!active) return 0;
  if (!fall) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] += y[m] * sc[m];
  }
  capture_flux(rec, f);
  return fall ? 1 : 0;
}

// ------------------------------------------------------------ training
// Captured samples -> features X[n][15], targets T[n][7], fallback flags.
__global__ void __launch_bounds__(256) k_mlp_prepare(const float* __restrict__ S, int n, float gam, float dp,
                                                     float drho, float* __restrict__ X, float* __restrict__ T,
                                                     int* __restrict__ flag) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float* s = S + (long long)i * 22;
  float wl[7], wr[7], x[16], sc[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    wl[m] = s[m];
    wr[m] = s[7 + m];
  }
  mlp_features(wl, wr, s[14], x, sc);
  const float gm1inv = 1.0f / (gam - 1.0f);
  float ul[7], ur[7], fl[7], fr[7];
  state_and_flux(wl, s[14], gm1inv, ul, fl);
  state_and_flux(wr, s[14], gm1inv, ur, fr);
#pragma unroll
  for (int m = 0; m < kNin; ++m) X[(long long)i * kNin + m] = x[m];
#pragma unroll
  for (int m = 0; m < kNout; ++m)
    T[(long long)i * kNout + m] = sc[m] > 0.0f ? (s[15 + m] - 0.5f * (fl[m] + fr[m])) / sc[m] : 0.0f;
  const float jp = fabsf(wr[4] - wl[4]) / fminf(wl[4], wr[4]);
  const float jr = fabsf(wr[0] - wl[0]) / fminf(wl[0], wr[0]);
  // bit 0: strong jump (HLLD at run time); bit 1: jump below kTinyJump, whose
  // target is dominated by the float round-off of the flux difference
  flag[i] = ((jp > dp) || (jr > drho) ? 1 : 0) | (x[4] < kTinyJump ? 2 : 0);
}

// Epilogues of the training GEMM
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_PRIME = 3 };

// C[M x N] = A[M x K] . B[K x N] with A(m,k) = A[m*sam + k*sak] and
// B(k,n) = B[k*sbk + n*sbn] (FP32 in memory, rounded to BF16 on load,
// FP32 accumulation).  One wave per 16 x 16 tile of C.
//   EPI_STORE:      C
//   EPI_BIAS:       C + bias[n]
//   EPI_BIAS_GELU:  Z = C + bias[n] -> Z and H = gelu(Z)
//   EPI_GELU_PRIME: C * gelu'(Zin[m][n])
template <int EPI>
__global__ void __launch_bounds__(256) k_mlp_gemm(int M, int N, int K, const float* __restrict__ A, long long sam,
                                                  long long sak, const float* __restrict__ Bm, long long sbk,
                                                  long long sbn, const float* __restrict__ bias,
                                                  const float* __restrict__ Zin, float* __restrict__ C,
                                                  float* __restrict__ H, int ldc) {
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int tiles_n = (N + 15) / 16;
  const int tiles = ((M + 15) / 16) * tiles_n;
  if (wave >= tiles) return;
  const int m0 = (wave / tiles_n) * 16, n0 = (wave % tiles_n) * 16;
  f32x4 c = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * lk + q;
      const int m = m0 + li, n = n0 + li;
      const float av = (m < M && k < K) ? A[m * sam + k * sak] : 0.0f;
      const float bv = (n < N && k < K) ? Bm[k * sbk + n * sbn] : 0.0f;
      a[q] = (short)f2bf(av);
      b[q] = (short)f2bf(bv);
    }
    c = mfma16(a, b, c);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = m0 + 4 * lk + q, n = n0 + li;
    if (m >= M || n >= N) continue;
    const long long o = (long long)m * ldc + n;
    float v = c[q];
    if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) v += bias[n];
    if (EPI == EPI_GELU_PRIME) v *= gelu_prime(Zin[o]);
    C[o] = v;
    if (EPI == EPI_BIAS_GELU) H[o] = gelu(v);
  }
}

// Split-K form of EPI_STORE for the weight gradients (small M x N, K = the
// batch): wave w computes tile w % tiles over rows [kc (w / tiles), + kc) of
// K into part[chunk][M][N]; k_mlp_sum_parts adds the chunks in order.
__global__ void __launch_bounds__(256) k_mlp_gemm_part(int M, int N, int K, int kc, const float* __restrict__ A,
                                                       long long sam, long long sak, const float* __restrict__ Bm,
                                                       long long sbk, long long sbn, float* __restrict__ part) {
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int tiles_n = (N + 15) / 16;
  const int tiles = ((M + 15) / 16) * tiles_n;
  const int chunks = (K + kc - 1) / kc;
  if (wave >= tiles * chunks) return;
  const int tile = wave % tiles, chunk = wave / tiles;
  const int m0 = (tile / tiles_n) * 16, n0 = (tile % tiles_n) * 16;
  const int kb = chunk * kc, ke = min(K, kb + kc);
  f32x4 c = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * lk + q;
      const int m = m0 + li, n = n0 + li;
      const float av = (m < M && k < ke) ? A[m * sam + k * sak] : 0.0f;
      const float bv = (n < N && k < ke) ? Bm[k * sbk + n * sbn] : 0.0f;
      a[q] = (short)f2bf(av);
      b[q] = (short)f2bf(bv);
    }
    c = mfma16(a, b, c);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = m0 + 4 * lk + q, n = n0 + li;
    if (m < M && n < N) part[((long long)chunk * M + m) * N + n] = c[q];
  }
}

__global__ void __launch_bounds__(256) k_mlp_sum_parts(int M, int N, int chunks, const float* __restrict__ part,
                                                       float* __restrict__ C, int ldc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M * N) return;
  float acc = 0.0f;
  for (int ch = 0; ch < chunks; ++ch) acc += part[(long long)ch * M * N + i];
  C[(long long)(i / N) * ldc + i % N] = acc;
}

// column sums of a [M x N] matrix (bias gradients), fixed order
__global__ void __launch_bounds__(256) k_mlp_colsum(int M, int N, const float* __restrict__ S, float* __restrict__ out) {
  __shared__ float red[256];
  const int n = blockIdx.x;
  float acc = 0.0f;
  for (int m = threadIdx.x; m < M; m += 256) acc += S[(long long)m * N + n];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

// dY = 2 (Y - T) / (n * 7); per-block partial sums of (Y - T)^2
__global__ void __launch_bounds__(256) k_mlp_mse(long long total, const float* __restrict__ Y, const float* __restrict__ T,
                                                 float* __restrict__ dY, float* __restrict__ part) {
  __shared__ float red[256];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  float e = 0.0f;
  if (i < total) {
    const float d = Y[i] - T[i];
    dY[i] = 2.0f * d / (float)total;
    e = d * d;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mlp_loss(const float* __restrict__ part, int nb, long long total, float* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += part[b];
  *loss = s / (float)total;
}

// Adam (Kingma & Ba) on the FP32 master parameters
__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g, int n, float lr, float b1, float b2,
                                                  float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace mhd
