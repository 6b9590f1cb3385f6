// The seeded kernel MLP (3 -> 64 -> 64 -> 64 -> 9, tanh) on BF16 MFMA
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) for one wave-tile of 32 pairs.
//
// Lane l works on pair p = l % 32; lanes l and l + 32 hold the same pair and
// split the K dimension of every product (K slots 8 h .. 8 h + 7, h = l / 32).
// Hidden layers are computed transposed, H^T[64 x 32] = W[64 x 64] H_in^T, so
// the pairs are the MFMA columns. An MFMA result register v of lane l holds
// row 8 (v / 4) + 4 h + v % 4 of column p; the next layer's K index is
// permuted to exactly that order (the weights are stored pre-permuted), so a
// layer's tanh output is the next layer's B operand without any data motion:
// K step s (features 16 s .. 16 s + 15) takes result registers 8 (s % 2) ..
// 8 (s % 2) + 7 of M tile s / 2.
//
// Precision: every weight W is stored as W_hi + W_lo (two BF16 numbers) and
// multiplied in two MFMAs, which removes the systematic error of rounding
// the weights to BF16; activations are rounded to BF16 once (near field) or
// carried as BF16 hi + lo with a third MFMA per K step (ACA samples, whose
// error must stay far below the cross-approximation tolerance). Layer 1 takes
// the input v = v_hi + v_lo split the same way, with the bias in spare K
// slots (K = 16: v_hi W_hi, v_lo W_hi, b_hi, b_lo, v_hi W_lo). The biases of
// layers 2-4 enter through one extra K step whose B operand is the constant
// column (1, 1, 0, ...). Accumulation is FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "devmath.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Fragment table (16 bytes per lane and fragment) in LDS.
#define FR_L1 0                                // [mo 2][lane 64]
#define FR_L2 (FR_L1 + 2 * 64)                 // [mo 2][s 4][part 2][lane]; bias [mo 2][lane]
#define FR_L3 (FR_L2 + (2 * 4 * 2 + 2) * 64)
#define FR_L4 (FR_L3 + (2 * 4 * 2 + 2) * 64)   // [s 4][part 2][lane]; bias [lane]
#define FR_TOTAL (FR_L4 + (4 * 2 + 1) * 64)
#define FR_BYTES (FR_TOTAL * 16)

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// tanh of 8 consecutive result registers -> one BF16 B operand (and, for
// the accurate tile, the BF16 remainder as a second operand). Layers 1-3 are
// stored scaled by 2 log2(e), so a result register y holds 2 log2(e) times
// the pre-activation x and tanh(x) = 1 - 2 / (2^y + 1). The accurate tile
// adds the remainder t - hi, rounded to BF16. Values go in pairs through one
// two-way BF16 conversion.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float tanh_scaled(float y) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f);
}

template <bool ACC>
__device__ __forceinline__ void act8(const f32x16& a, int base, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int u = 0; u < 8; u += 2) {
    const f32x2 t = {tanh_scaled(a[base + u]), tanh_scaled(a[base + u + 1])};
    const bf16x2 h = __builtin_convertvector(t, bf16x2);
    hi[u] = h[0];
    hi[u + 1] = h[1];
    if (ACC) {
      const uint32_t hb = __builtin_bit_cast(uint32_t, h);
      const f32x2 r = {t[0] - __uint_as_float(hb << 16), t[1] - __uint_as_float(hb & 0xffff0000u)};
      const bf16x2 l = __builtin_convertvector(r, bf16x2);
      lo[u] = l[0];
      lo[u + 1] = l[1];
    }
  }
}

// One hidden layer (64 -> 64) of NT independent tiles: B[t][4] in, Bo[t][4]
// out (after tanh). Each weight fragment is read once for all NT tiles, and
// the tiles' MFMA chains are independent, so one tile's MFMAs overlap the
// other's activations. ACC adds the products of the activation remainders
// (W_hi a_lo), for samples whose error must stay far below the
// cross-approximation tolerance.
template <bool ACC, int NT>
__device__ __forceinline__ void hidden_layer(const bf16x8* __restrict__ fr, int base, int lane,
                                             const bf16x8 (&B)[NT][4], const bf16x8 (&Bl)[NT][4],
                                             const bf16x8& Bone, bf16x8 (&Bo)[NT][4],
                                             bf16x8 (&Bol)[NT][4]) {
#pragma unroll
  for (int mo = 0; mo < 2; ++mo) {
    f32x16 acc[NT];
    const bf16x8 wb = fr[base + (2 * 4 * 2) * 64 + mo * 64 + lane];   // bias
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16(wb, Bone, f32x16{});
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bf16x8 wh = fr[base + ((mo * 4 + s) * 2 + 0) * 64 + lane];
      const bf16x8 wl = fr[base + ((mo * 4 + s) * 2 + 1) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc[t] = mfma_bf16(wh, B[t][s], acc[t]);
        acc[t] = mfma_bf16(wl, B[t][s], acc[t]);
        if (ACC) acc[t] = mfma_bf16(wh, Bl[t][s], acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      act8<ACC>(acc[t], 0, Bo[t][2 * mo], Bol[t][2 * mo]);
      act8<ACC>(acc[t], 8, Bo[t][2 * mo + 1], Bol[t][2 * mo + 1]);
    }
  }
}

// Raw outputs o[t][0..8] of the MLP at inputs v[t] for this lane's pair of
// each of NT independent tiles. Must be called by all 64 lanes of the wave
// with lanes l and l+32 holding the same inputs. ACC = false: activations
// rounded to BF16 once (relative error ~1e-4 of a sample); ACC = true:
// activations carried as BF16 hi + lo (~3e-6), used where samples must
// resolve a 1e-4 cross-approximation.
template <bool ACC, int NT>
__device__ __forceinline__ void mlp_tiles_bf16(const bf16x8* __restrict__ fr,
                                               const float (&v)[NT][3], float (&o)[NT][9]) {
  // the fragments are re-read from LDS for every call: hoisting them out of
  // a caller's loop would pin 192 VGPRs and cut the occupancy to one wave
  __asm__ volatile("" ::: "memory");
  const int lane = threadIdx.x & 63;
  const bool h1 = lane >= 32;
  const __bf16 z = (__bf16)0.0f, one = (__bf16)1.0f;
  bf16x8 Bone;
#pragma unroll
  for (int u = 0; u < 8; ++u) Bone[u] = (!h1 && u < 2) ? one : z;
  // layer 1 input column: K slots (v_hi, v_lo, 1, 1 | v_hi, 0...)
  bf16x8 b1[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const __bf16 vh0 = (__bf16)v[t][0], vh1 = (__bf16)v[t][1], vh2 = (__bf16)v[t][2];
    b1[t][0] = vh0;
    b1[t][1] = vh1;
    b1[t][2] = vh2;
    b1[t][3] = h1 ? z : (__bf16)(v[t][0] - (float)vh0);
    b1[t][4] = h1 ? z : (__bf16)(v[t][1] - (float)vh1);
    b1[t][5] = h1 ? z : (__bf16)(v[t][2] - (float)vh2);
    b1[t][6] = h1 ? z : one;
    b1[t][7] = h1 ? z : one;
  }
  bf16x8 B[NT][4], Bn[NT][4], Bl[NT][4], Bnl[NT][4];
#pragma unroll
  for (int mo = 0; mo < 2; ++mo) {
    const bf16x8 w1 = fr[FR_L1 + mo * 64 + lane];
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16(w1, b1[t], f32x16{});
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      act8<ACC>(acc[t], 0, B[t][2 * mo], Bl[t][2 * mo]);
      act8<ACC>(acc[t], 8, B[t][2 * mo + 1], Bl[t][2 * mo + 1]);
    }
  }
  hidden_layer<ACC, NT>(fr, FR_L2, lane, B, Bl, Bone, Bn, Bnl);
  hidden_layer<ACC, NT>(fr, FR_L3, lane, Bn, Bnl, Bone, B, Bl);
  f32x16 acc[NT];
  const bf16x8 w4b = fr[FR_L4 + (4 * 2) * 64 + lane];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16(w4b, Bone, f32x16{});
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const bf16x8 wh = fr[FR_L4 + (s * 2 + 0) * 64 + lane];
    const bf16x8 wl = fr[FR_L4 + (s * 2 + 1) * 64 + lane];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[t] = mfma_bf16(wh, B[t][s], acc[t]);
      acc[t] = mfma_bf16(wl, B[t][s], acc[t]);
      if (ACC) acc[t] = mfma_bf16(wh, Bl[t][s], acc[t]);
    }
  }
  // rows 0-3 and 8 live in lanes 0-31 (registers 0-3, 4); rows 4-7 in 32-63
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const f32x16& c = acc[t];
    const float t0 = __shfl_xor(c[0], 32, 64), t1 = __shfl_xor(c[1], 32, 64);
    const float t2 = __shfl_xor(c[2], 32, 64), t3 = __shfl_xor(c[3], 32, 64);
    const float t4 = __shfl_xor(c[4], 32, 64);
    o[t][0] = h1 ? t0 : c[0]; o[t][1] = h1 ? t1 : c[1]; o[t][2] = h1 ? t2 : c[2];
    o[t][3] = h1 ? t3 : c[3]; o[t][4] = h1 ? c[0] : t0; o[t][5] = h1 ? c[1] : t1;
    o[t][6] = h1 ? c[2] : t2; o[t][7] = h1 ? c[3] : t3; o[t][8] = h1 ? t4 : c[4];
  }
}

// One tile of 32 pairs (see mlp_tiles_bf16).
template <bool ACC>
__device__ __forceinline__ void mlp_tile_bf16(const bf16x8* __restrict__ fr, float v0, float v1,
                                              float v2, float o[9]) {
  const float v[1][3] = {{v0, v1, v2}};
  float oo[1][9];
  mlp_tiles_bf16<ACC, 1>(fr, v, oo);
#pragma unroll
  for (int e = 0; e < 9; ++e) o[e] = oo[0][e];
}

// Stage the fragment table (global -> LDS) by the whole workgroup.
__device__ __forceinline__ void stage_frags(bf16x8* __restrict__ lds, const uint4* __restrict__ g,
                                            int nthreads) {
  uint4* d = reinterpret_cast<uint4*>(lds);
  for (int i = threadIdx.x; i < FR_TOTAL; i += nthreads) d[i] = g[i];
}

// ------------------------------------------------------------ FP32 MFMA tile
//
// The same MLP for one wave-tile of 32 pairs on FP32 MFMA
// (v_mfma_f32_32x32x2_f32: FP32 operands and accumulation, the plain FP32
// form). Lane l works on pair l % 32 and supplies K slot h = l / 32 of every
// product. A result register r of lane l holds row 8 (r / 4) + 4 h + r % 4
// of its M tile; K step (mo, r) of the next layer contracts the two features
// 32 mo + 8 (r / 4) + r % 4 + 4 h, h = 0, 1, which are exactly what the two
// halves of the wave hold in register r, so a layer's tanh output is the next
// layer's B operand with no data motion (the weights are stored permuted to
// that order, one float per lane and step). Layer 1 contracts (v0, v1) and
// (v2, 1), the 1 carrying the bias; layers 2-4 take their bias through one
// extra step whose B operand is (1, 0). Layers 1-3 are stored scaled by
// 2 log2(e) (see tanh_scaled).
#define F32_L1 0                               // [mo 2][step 2]
#define F32_L2 (F32_L1 + 4)                    // [mo' 2][mo 2][r 16], bias [mo' 2]
#define F32_L3 (F32_L2 + 66)
#define F32_L4 (F32_L3 + 66)                   // [mo 2][r 16], bias
#define F32_FRAGS (F32_L4 + 33)
#define F32_BYTES (F32_FRAGS * 64 * 4)

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// One hidden layer (64 -> 64, then tanh) from h[2][16] into g[2][16]; the two
// output M tiles are two independent MFMA chains.
__device__ __forceinline__ void hidden_f32(const float* __restrict__ fr, int base, int lane,
                                           float bone, const float (&h)[2][16],
                                           float (&g)[2][16]) {
  f32x16 a0 = mfma_f32(fr[(base + 64) * 64 + lane], bone, f32x16{});
  f32x16 a1 = mfma_f32(fr[(base + 65) * 64 + lane], bone, f32x16{});
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      a0 = mfma_f32(fr[(base + (0 * 2 + mo) * 16 + r) * 64 + lane], h[mo][r], a0);
      a1 = mfma_f32(fr[(base + (1 * 2 + mo) * 16 + r) * 64 + lane], h[mo][r], a1);
    }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    g[0][r] = tanh_scaled(a0[r]);
    g[1][r] = tanh_scaled(a1[r]);
  }
}

// Raw outputs o[0..8] of the MLP at input (v0, v1, v2) for this lane's pair.
// Must be called by all 64 lanes with lanes l and l + 32 holding the same
// input. fr: the FP32 fragment table (F32_FRAGS x 64 floats).
__device__ __forceinline__ void mlp_tile_f32(const float* __restrict__ fr, float v0, float v1,
                                             float v2, float o[9]) {
  __asm__ volatile("" ::: "memory");
  const int lane = threadIdx.x & 63;
  const bool h1 = lane >= 32;
  const float bone = h1 ? 0.0f : 1.0f;
  float h[2][16], g[2][16];
  {
    const float b0 = h1 ? v1 : v0, b1 = h1 ? 1.0f : v2;
#pragma unroll
    for (int mo = 0; mo < 2; ++mo) {
      f32x16 a = mfma_f32(fr[(F32_L1 + 2 * mo) * 64 + lane], b0, f32x16{});
      a = mfma_f32(fr[(F32_L1 + 2 * mo + 1) * 64 + lane], b1, a);
#pragma unroll
      for (int r = 0; r < 16; ++r) h[mo][r] = tanh_scaled(a[r]);
    }
  }
  hidden_f32(fr, F32_L2, lane, bone, h, g);
  hidden_f32(fr, F32_L3, lane, bone, g, h);
  // layer 4: two chains (features of M tile 0 and 1), summed at the end
  f32x16 c0 = mfma_f32(fr[(F32_L4 + 32) * 64 + lane], bone, f32x16{});
  f32x16 c1 = f32x16{};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    c0 = mfma_f32(fr[(F32_L4 + r) * 64 + lane], h[0][r], c0);
    c1 = mfma_f32(fr[(F32_L4 + 16 + r) * 64 + lane], h[1][r], c1);
  }
  // rows 0-3 and 8 live in lanes 0-31 (registers 0-3, 4); rows 4-7 in 32-63
  float c[5];
#pragma unroll
  for (int e = 0; e < 5; ++e) c[e] = c0[e] + c1[e];
  const float t0 = __shfl_xor(c[0], 32, 64), t1 = __shfl_xor(c[1], 32, 64);
  const float t2 = __shfl_xor(c[2], 32, 64), t3 = __shfl_xor(c[3], 32, 64);
  const float t4 = __shfl_xor(c[4], 32, 64);
  o[0] = h1 ? t0 : c[0]; o[1] = h1 ? t1 : c[1]; o[2] = h1 ? t2 : c[2];
  o[3] = h1 ? t3 : c[3]; o[4] = h1 ? c[0] : t0; o[5] = h1 ? c[1] : t1;
  o[6] = h1 ? c[2] : t2; o[7] = h1 ? c[3] : t3; o[8] = h1 ? t4 : c[4];
}

// Symmetrised kernel entry K(r) = (O + O^T)/2 / (8 pi |r|) of this lane's
// pair from the FP32 tile, r given in FP64 and rounded to FP32 (all 64 lanes
// call it; lanes l and l + 32 hold the same r). The ACA samples and their
// replay both come from here, so a replay reproduces a build bit for bit.
__device__ __forceinline__ void entry_f32tile(const float* __restrict__ fr, int mode, double dx,
                                              double dy, double dz, float K[9]) {
  const float rx = (float)dx, ry = (float)dy, rz = (float)dz;
  const float rs = hh_rsqrt(rx * rx + ry * ry + rz * rz);
  const float sc = mode == HH_MLP_INPUT_DIRECTION ? rs : 1.0f;
  float o[9];
  mlp_tile_f32(fr, rx * sc, ry * sc, rz * sc, o);
  const float s = rs * (float)(1.0 / (16.0 * HH_PI));
  K[0] = 2.0f * o[0] * s; K[1] = (o[1] + o[3]) * s; K[2] = (o[2] + o[6]) * s;
  K[3] = K[1];            K[4] = 2.0f * o[4] * s;   K[5] = (o[5] + o[7]) * s;
  K[6] = K[2];            K[7] = K[5];              K[8] = 2.0f * o[8] * s;
}

// Stage the FP32 fragment table (global -> LDS) by the whole workgroup.
__device__ __forceinline__ void stage_frags_f32(float* __restrict__ lds,
                                                const float4* __restrict__ g, int nthreads) {
  float4* d = reinterpret_cast<float4*>(lds);
  for (int i = threadIdx.x; i < F32_FRAGS * 16; i += nthreads) d[i] = g[i];
}
