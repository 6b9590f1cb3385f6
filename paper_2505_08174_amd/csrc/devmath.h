// Device math and two-body kernel evaluation for gfx950 (VALU forms).
//
// tanh in FP32 uses the identity tanh(x) = 1 - 2 / (e^{2x} + 1) with the
// hardware base-2 exponential (v_exp_f32) and reciprocal (v_rcp_f32).
// tanh in FP64 uses tanh(|x|) = m / (m + 2) with m = e^{2|x|} - 1, where e^y
// is evaluated by Cody-Waite reduction y = k ln2 + r, |r| <= ln2/2, and the
// Taylor series of e^r (degree 13, truncation < 1e-17 relative); for small
// arguments m comes straight from the Taylor series of e^y - 1, which avoids
// the cancellation of e^y - 1.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

#define HH_PI 3.14159265358979323846

__device__ __forceinline__ float hh_tanh(float x) {
  float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // e^{2x} = 2^{2x log2 e}
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ double hh_expm1_taylor(double x) {
  // sum_{n=1}^{16} x^n / n!, Horner form; |x| <= 0.35 gives < 1e-19 truncation.
  double p = 1.0 / 20922789888000.0;  // 1/16!
  p = p * x + 1.0 / 1307674368000.0;  // 1/15!
  p = p * x + 1.0 / 87178291200.0;
  p = p * x + 1.0 / 6227020800.0;
  p = p * x + 1.0 / 479001600.0;
  p = p * x + 1.0 / 39916800.0;
  p = p * x + 1.0 / 3628800.0;
  p = p * x + 1.0 / 362880.0;
  p = p * x + 1.0 / 40320.0;
  p = p * x + 1.0 / 5040.0;
  p = p * x + 1.0 / 720.0;
  p = p * x + 1.0 / 120.0;
  p = p * x + 1.0 / 24.0;
  p = p * x + 1.0 / 6.0;
  p = p * x + 0.5;
  p = p * x + 1.0;
  return p * x;
}

__device__ __forceinline__ double hh_exp(double y) {
  // y = k ln2 + r with ln2 split so that k * LN2_HI is exact for |k| < 2^20.
  const double LN2_HI = 6.93147180369123816490e-01;
  const double LN2_LO = 1.90821492927058770002e-10;
  const double INV_LN2 = 1.44269504088896338700e+00;
  double k = rint(y * INV_LN2);
  double r = (y - k * LN2_HI) - k * LN2_LO;
  double er = 1.0 + hh_expm1_taylor(r);
  return ldexp(er, (int)k);
}

__device__ __forceinline__ double hh_tanh(double x) {
  double ax = fabs(x);
  if (ax >= 20.0) return copysign(1.0, x);  // 1 - tanh(20) < 1e-17
  double y = 2.0 * ax;
  double m = (y <= 0.34) ? hh_expm1_taylor(y) : hh_exp(y) - 1.0;
  return copysign(m / (m + 2.0), x);
}

__device__ __forceinline__ float hh_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double hh_rsqrt(double x) { return 1.0 / sqrt(x); }

// ------------------------------------------------------------------ RPY

// K(r) as a symmetric 3x3 (row-major 9 values) for spheres of radius a.
// c8 = 1/(8 pi mu), c6 = 1/(6 pi mu a).
template <class T>
__device__ __forceinline__ void rpy_entry(T rx, T ry, T rz, T a, T c8, T c6, T K[9]) {
  T d2 = rx * rx + ry * ry + rz * rz;
  T d = sqrt(d2);
  T ci, co;  // K = ci I + co r r^T / d^2
  if (d >= T(2) * a) {
    T id = T(1) / d;
    T a2d2 = a * a / d2;
    ci = (T(1) + T(2) / T(3) * a2d2) * c8 * id;
    co = (T(1) - T(2) * a2d2) * c8 * id;
  } else {
    ci = (T(1) - T(9) / T(32) * d / a) * c6;
    co = (T(3) / T(32) * d / a) * c6;
  }
  T s = co / d2;
  K[0] = ci + s * rx * rx; K[1] = s * rx * ry; K[2] = s * rx * rz;
  K[3] = K[1];             K[4] = ci + s * ry * ry; K[5] = s * ry * rz;
  K[6] = K[2];             K[7] = K[5];             K[8] = ci + s * rz * rz;
}

// The 6N Rotne-Prager mobility on its grid of 3x3 entries (Eq. (1)): row
// parity si = 0 is a translational velocity, 1 a rotational one; column
// parity sj = 0 a force, 1 a torque. r = x_i - x_j, d = |r|, c8 = 1/(8 pi mu):
//   (0, 0): the RPY tensor above;
//   (1, 0) and (0, 1): -(c8 / d^3) [r]_x, [r]_x u = r x u (half the curl of
//           the Stokeslet flow; the coupling block is the same function of r
//           in both places);
//   (1, 1): -(c8 / (2 d^3)) (I - 3 r r^T / d^2) (half the curl of the rotlet
//           flow).
// The rotational blocks are the forms for non-overlapping spheres (d >= 2a).
// d = 0 (the two rows of one particle) gives zeros: the self terms are added
// separately.
template <class T>
__device__ __forceinline__ void rpy6_entry(int si, int sj, T rx, T ry, T rz, T a, T c8, T c6,
                                           T K[9]) {
  if ((si | sj) == 0) {
    rpy_entry<T>(rx, ry, rz, a, c8, c6, K);
    return;
  }
  const T d2 = rx * rx + ry * ry + rz * rz;
  if (!(d2 > T(0))) {
#pragma unroll
    for (int e = 0; e < 9; ++e) K[e] = T(0);
    return;
  }
  const T id2 = T(1) / d2;
  const T id3 = id2 * sqrt(id2);
  if (si != sj) {
    const T s = c8 * id3;
    K[0] = T(0);   K[1] = s * rz;  K[2] = -s * ry;
    K[3] = -s * rz; K[4] = T(0);   K[5] = s * rx;
    K[6] = s * ry;  K[7] = -s * rx; K[8] = T(0);
  } else {
    const T ci = -T(0.5) * c8 * id3, co = T(1.5) * c8 * id3 * id2;
    K[0] = ci + co * rx * rx; K[1] = co * rx * ry;      K[2] = co * rx * rz;
    K[3] = K[1];              K[4] = ci + co * ry * ry; K[5] = co * ry * rz;
    K[6] = K[2];              K[7] = K[5];              K[8] = ci + co * rz * rz;
  }
}

// ------------------------------------------------------------- MLP (VALU)

// Raw outputs o[9] of the 3-64-64-64-9 tanh MLP at input v, parameters packed
// (see internal.h) in any address space P points to.
template <class T, class PT>
__device__ __forceinline__ void mlp_raw(const PT* __restrict__ P, T v0, T v1, T v2, T o[9]) {
  T h1[MLP_H], h2[MLP_H];
#pragma unroll
  for (int k = 0; k < MLP_H; ++k) {
    T z = T(P[OFF_B1 + k]) + T(P[OFF_W1 + 3 * k]) * v0 + T(P[OFF_W1 + 3 * k + 1]) * v1 +
          T(P[OFF_W1 + 3 * k + 2]) * v2;
    h1[k] = hh_tanh(z);
  }
#pragma unroll 4
  for (int o2 = 0; o2 < MLP_H; ++o2) {
    T z = T(P[OFF_B2 + o2]);
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z += T(P[OFF_W2 + MLP_H * o2 + k]) * h1[k];
    h2[o2] = hh_tanh(z);
  }
#pragma unroll 4
  for (int o3 = 0; o3 < MLP_H; ++o3) {
    T z = T(P[OFF_B3 + o3]);
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z += T(P[OFF_W3 + MLP_H * o3 + k]) * h2[k];
    h1[o3] = hh_tanh(z);
  }
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    T z = T(P[OFF_B4 + m]);
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z += T(P[OFF_W4 + MLP_H * m + k]) * h1[k];
    o[m] = z;
  }
}

// K(r) = (O + O^T)/2 / (8 pi |r|), O = reshape(MLP(v)) row-major.
template <class T, class PT>
__device__ __forceinline__ void mlp_entry(const PT* __restrict__ P, int input_mode, T rx, T ry,
                                          T rz, T K[9]) {
  T d2 = rx * rx + ry * ry + rz * rz;
  T id = hh_rsqrt(d2);
  T v0 = rx, v1 = ry, v2 = rz;
  if (input_mode == HH_MLP_INPUT_DIRECTION) { v0 *= id; v1 *= id; v2 *= id; }
  T o[9];
  mlp_raw<T>(P, v0, v1, v2, o);
  T s = id * T(1.0 / (16.0 * HH_PI));   // (1/2) * 1/(8 pi |r|)
  K[0] = T(2) * o[0] * s; K[1] = (o[1] + o[3]) * s; K[2] = (o[2] + o[6]) * s;
  K[3] = K[1];            K[4] = T(2) * o[4] * s;   K[5] = (o[5] + o[7]) * s;
  K[6] = K[2];            K[7] = K[5];              K[8] = T(2) * o[8] * s;
}

// Kernel parameters passed by value to device code.
struct KParams {
  int kind;
  int input_mode;
  // alpha1: self mobility of even rows; alpha2: of odd rows (the rotational
  // rows of a 6N kernel; equal to alpha1 for the 3N kernels)
  double a, c8, c6, alpha1, alpha2;
  const void* w;     // packed MLP parameters (double or float per T)
};

// Kernel parameters of a kernel handle, with the MLP weights of the FP64
// (fp64) or the FP32 copy.
KParams make_kparams(hh_kernel k, bool fp64);

// Entry K(r) between rows i and j; si, sj are their parities (i & 1, j & 1),
// which only the 6N kernel reads.
template <class T>
__device__ __forceinline__ void kernel_entry(const KParams& kp, const T* __restrict__ wl, T rx,
                                             T ry, T rz, T K[9], int si = 0, int sj = 0) {
  if (kp.kind == KIND_RPY)
    rpy_entry<T>(rx, ry, rz, T(kp.a), T(kp.c8), T(kp.c6), K);
  else if (kp.kind == KIND_RPY6)
    rpy6_entry<T>(si, sj, rx, ry, rz, T(kp.a), T(kp.c8), T(kp.c6), K);
  else
    mlp_entry<T, T>(wl, kp.input_mode, rx, ry, rz, K);
}

// Rows i and j belong to one particle (their pair term is not summed): the
// same row, or for the 6N kernel the two rows 2p, 2p + 1 of particle p.
__device__ __forceinline__ bool same_particle(int kind, int64_t i, int64_t j) {
  return kind == KIND_RPY6 ? (i >> 1) == (j >> 1) : i == j;
}

// ------------------------------------------------------- wave reductions

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Argmax with ties to the lowest index: (v, i) pairs.
template <class T>
__device__ __forceinline__ void wave_argmax(T& v, int& i) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T v2 = __shfl_xor(v, o, 64);
    int i2 = __shfl_xor(i, o, 64);
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
  }
}
