// Back-propagation of kernel-MLP samples on FP32 MFMA (the FP32 backward).
//
// A tile is 32 pairs (i, j) with cotangents G_ij of their kernel entries
// K(x_i - x_j); lane l works on pair l % 32 (lanes l and l + 32 hold the same
// pair), as in the FP32 forward tile (mlp_mfma.h). Per tile:
//   forward: the three hidden activations H1, H2, H3 (64 x 32 each, kept in
//            the result-register layout) and the outputs o;
//   output cotangent d4 = s g, s = 1/(8 pi |r|), g the symmetric part of G;
//   deltas: D3 = (W4^T d4) * (1 - H3^2), D2 = (W3^T D3) * (1 - H2^2),
//           D1 = (W2^T D2) * (1 - H1^2), as MFMA chains on a table of the
//           transposed weights permuted like the forward one, so each delta
//           feeds the next product with no data motion;
//   parameter gradients: dW_l += D_l H_{l-1}^T is a product over the tile's
//           32 pairs (K = pairs); D_l and H_{l-1} go through a per-wave LDS
//           buffer ([feature][pair]) to bring the pairs into the K slots, and
//           the MFMA accumulators of the four weight matrices persist across
//           tiles (FP32 over at most FLUSH tiles, then added into the wave's
//           own FP64 slot; slots are summed in a fixed order afterwards);
//           biases and W1 (64 x 3) by each lane for its own feature;
//   input cotangent dL/dv = W1^T D1, then dL/dr through the direction input
//           and through s.
// Near pairs: work unit = 32 targets of a leaf against every source of its
// near list (one source per tile, as the forward near field); the source's
// dX is the wave sum of its 32 pairs, added with one atomic per component.
// Far pairs: the samples of every ACA term of a block, 32 per tile; a column
// term's samples share x_j and a row term's share x_i, so that side is also
// summed over the tile before its atomic.
#include <algorithm>

#include "devmath.h"
#include "internal.h"
#include "mlp_mfma.h"

// Transposed-weight table of the FP32 backward (one float per lane and step):
// BW4: [mo' 2][s 5] W4[2 s + h][32 mo' + lane % 32] (0 past row 8);
// BW3, BW2: [mo' 2][mo 2][r 16] W[f(mo, r, h)][32 mo' + lane % 32];
// BW1: [d 3][feature 64] W1[feature][d] (read by feature, not by lane).
#define BW4 0
#define BW3 (BW4 + 10)
#define BW2 (BW3 + 64)
#define BW1 (BW2 + 64)
#define BW_FRAGS (BW1 + 3)

namespace {

constexpr int VB = 256;        // four waves per workgroup
constexpr int XS = 33;         // row stride (floats) of the per-wave LDS buffers
constexpr int FLUSH = 64;      // tiles between flushes of the FP32 accumulators

// feature held in result register r of M tile mo by lane half h
__device__ __forceinline__ int feat(int mo, int r, int h) {
  return 32 * mo + 8 * (r / 4) + 4 * h + (r % 4);
}

struct VjpAcc {
  f32x16 w3[2][2], w2[2][2];
  float b1, b2, b3, b4, w1[3], w4[9];   // w4[m]: W4[m][feature = lane]
};

__device__ __forceinline__ void acc_zero(VjpAcc& A) {
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      A.w3[a][b] = f32x16{};
      A.w2[a][b] = f32x16{};
    }
  }
  A.b1 = A.b2 = A.b3 = A.b4 = 0.0f;
  A.w1[0] = A.w1[1] = A.w1[2] = 0.0f;
#pragma unroll
  for (int m = 0; m < 9; ++m) A.w4[m] = 0.0f;
}

// Adds the accumulators into the wave's FP64 slot (every parameter has one
// owner lane and register) and clears them.
__device__ __forceinline__ void acc_flush(VjpAcc& A, double* __restrict__ slot) {
  const int lane = threadIdx.x & 63, h = lane >> 5, p = lane & 31;
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int no = 0; no < 2; ++no)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = feat(mo, r, h), col = 32 * no + p;
        slot[OFF_W3 + MLP_H * row + col] += (double)A.w3[mo][no][r];
        slot[OFF_W2 + MLP_H * row + col] += (double)A.w2[mo][no][r];
      }
#pragma unroll
  for (int m = 0; m < 9; ++m) slot[OFF_W4 + MLP_H * m + lane] += (double)A.w4[m];
  slot[OFF_B3 + lane] += (double)A.b3;
  slot[OFF_B2 + lane] += (double)A.b2;
  slot[OFF_B1 + lane] += (double)A.b1;
#pragma unroll
  for (int d = 0; d < 3; ++d) slot[OFF_W1 + 3 * lane + d] += (double)A.w1[d];
  if (lane < 9) slot[OFF_B4 + lane] += (double)A.b4;
  acc_zero(A);
}

// Writes a 64 x 32 block held in the result-register layout to LDS as
// [feature][pair].
__device__ __forceinline__ void put_block(float* __restrict__ X, const float (&v)[2][16]) {
  const int lane = threadIdx.x & 63, h = lane >> 5, p = lane & 31;
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int r = 0; r < 16; ++r) X[feat(mo, r, h) * XS + p] = v[mo][r];
}

// LDS accesses of one wave are processed in order; this keeps the compiler
// from moving them across the phase boundary.
__device__ __forceinline__ void lds_phase() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
  __asm__ volatile("" ::: "memory");
}

// dW += D H^T over the 32 pairs of the tile (D rows = output features, H rows
// = input features), D and H in XD and XH; and the bias sum of D's rows.
__device__ __forceinline__ void grad_block(const float* __restrict__ XD,
                                           const float* __restrict__ XH, f32x16 (&W)[2][2],
                                           float& bias) {
  const int lane = threadIdx.x & 63, h = lane >> 5, p = lane & 31;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const float a0 = XD[p * XS + 2 * s + h], a1 = XD[(32 + p) * XS + 2 * s + h];
    const float b0 = XH[p * XS + 2 * s + h], b1 = XH[(32 + p) * XS + 2 * s + h];
    W[0][0] = mfma_f32(a0, b0, W[0][0]);
    W[0][1] = mfma_f32(a0, b1, W[0][1]);
    W[1][0] = mfma_f32(a1, b0, W[1][0]);
    W[1][1] = mfma_f32(a1, b1, W[1][1]);
  }
  float sb = 0.0f;
#pragma unroll
  for (int q = 0; q < 32; ++q) sb += XD[lane * XS + q];
  bias += sb;
}

// The transposed product T^T of one layer (64 -> 64) applied to D (result
// layout), times (1 - H^2): the next delta.
__device__ __forceinline__ void delta_hidden(const float* __restrict__ bw, int base, int lane,
                                             const float (&D)[2][16], const float (&H)[2][16],
                                             float (&out)[2][16]) {
  f32x16 a0 = f32x16{}, a1 = f32x16{};
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      a0 = mfma_f32(bw[(base + (0 * 2 + mo) * 16 + r) * 64 + lane], D[mo][r], a0);
      a1 = mfma_f32(bw[(base + (1 * 2 + mo) * 16 + r) * 64 + lane], D[mo][r], a1);
    }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    out[0][r] = a0[r] * (1.0f - H[0][r] * H[0][r]);
    out[1][r] = a1[r] * (1.0f - H[1][r] * H[1][r]);
  }
}

// One tile: pair input v (direction or displacement), symmetric cotangent g
// (zero for a lane that adds nothing), s = 1/(8 pi |r|). Returns dL/dv (both
// halves combined) and og = sum_m o_m g_m; accumulates the parameter
// gradients into A. XD, XH: this wave's LDS buffers (64 x XS floats each).
__device__ __forceinline__ void vjp_tile_f32(const float* __restrict__ fw,
                                             const float* __restrict__ bw, float* __restrict__ XD,
                                             float* __restrict__ XH, VjpAcc& A, float v0, float v1,
                                             float v2, const float (&g)[9], float s,
                                             float (&gv)[3], float& og) {
  const int lane = threadIdx.x & 63, h = lane >> 5, p = lane & 31;
  const bool h1 = h == 1;
  const float bone = h1 ? 0.0f : 1.0f;
  float H1[2][16], H2[2][16], H3[2][16], D[2][16], E[2][16];
  // ---- forward
  {
    const float b0 = h1 ? v1 : v0, b1 = h1 ? 1.0f : v2;
#pragma unroll
    for (int mo = 0; mo < 2; ++mo) {
      f32x16 a = mfma_f32(fw[(F32_L1 + 2 * mo) * 64 + lane], b0, f32x16{});
      a = mfma_f32(fw[(F32_L1 + 2 * mo + 1) * 64 + lane], b1, a);
#pragma unroll
      for (int r = 0; r < 16; ++r) H1[mo][r] = tanh_scaled(a[r]);
    }
  }
  hidden_f32(fw, F32_L2, lane, bone, H1, H2);
  hidden_f32(fw, F32_L3, lane, bone, H2, H3);
  float o[9];
  {
    f32x16 c0 = mfma_f32(fw[(F32_L4 + 32) * 64 + lane], bone, f32x16{});
    f32x16 c1 = f32x16{};
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      c0 = mfma_f32(fw[(F32_L4 + r) * 64 + lane], H3[0][r], c0);
      c1 = mfma_f32(fw[(F32_L4 + 16 + r) * 64 + lane], H3[1][r], c1);
    }
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
  float d4[10];
  og = 0.0f;
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    og += o[m] * g[m];
    d4[m] = s * g[m];
  }
  d4[9] = 0.0f;
  // ---- dW4, db4: rows 0..8 of XD hold d4 of the tile's pairs, XH holds H3
  if (!h1) {
#pragma unroll
    for (int m = 0; m < 9; ++m) XD[m * XS + p] = d4[m];
  }
  put_block(XH, H3);
  lds_phase();
  {
    // lane = feature k: W4[m][k] += sum over pairs of d4[m] H3[k] (9 x 64)
#pragma unroll 4
    for (int q = 0; q < 32; ++q) {
      const float hk = XH[lane * XS + q];
#pragma unroll
      for (int m = 0; m < 9; ++m) A.w4[m] += XD[m * XS + q] * hk;
    }
    float sb = 0.0f;
    if (lane < 9) {
#pragma unroll
      for (int q = 0; q < 32; ++q) sb += XD[lane * XS + q];
    }
    A.b4 += sb;
  }
  lds_phase();
  // ---- D3 = (W4^T d4) (1 - H3^2)
  {
    f32x16 a0 = f32x16{}, a1 = f32x16{};
#pragma unroll
    for (int s2 = 0; s2 < 5; ++s2) {
      const float b = h1 ? d4[2 * s2 + 1] : d4[2 * s2];
      a0 = mfma_f32(bw[(BW4 + s2) * 64 + lane], b, a0);
      a1 = mfma_f32(bw[(BW4 + 5 + s2) * 64 + lane], b, a1);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      D[0][r] = a0[r] * (1.0f - H3[0][r] * H3[0][r]);
      D[1][r] = a1[r] * (1.0f - H3[1][r] * H3[1][r]);
    }
  }
  // ---- dW3, db3
  put_block(XD, D);
  put_block(XH, H2);
  lds_phase();
  grad_block(XD, XH, A.w3, A.b3);
  lds_phase();
  // ---- D2, then dW2, db2
  delta_hidden(bw, BW3, lane, D, H2, E);
  put_block(XD, E);
  put_block(XH, H1);
  lds_phase();
  grad_block(XD, XH, A.w2, A.b2);
  lds_phase();
  // ---- D1, then dW1, db1 and dL/dv
  delta_hidden(bw, BW2, lane, E, H1, D);
  put_block(XD, D);
  if (!h1) {
    XH[0 * XS + p] = v0;
    XH[1 * XS + p] = v1;
    XH[2 * XS + p] = v2;
  }
  lds_phase();
  {
    float sb = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const float d = XD[lane * XS + q];
      sb += d;
      s0 += d * XH[0 * XS + q];
      s1 += d * XH[1 * XS + q];
      s2 += d * XH[2 * XS + q];
    }
    A.b1 += sb;
    A.w1[0] += s0;
    A.w1[1] += s1;
    A.w1[2] += s2;
  }
  lds_phase();
  float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f;
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = feat(mo, r, h);
      q0 += bw[(BW1 + 0) * 64 + f] * D[mo][r];
      q1 += bw[(BW1 + 1) * 64 + f] * D[mo][r];
      q2 += bw[(BW1 + 2) * 64 + f] * D[mo][r];
    }
  gv[0] = q0 + __shfl_xor(q0, 32, 64);
  gv[1] = q1 + __shfl_xor(q1, 32, 64);
  gv[2] = q2 + __shfl_xor(q2, 32, 64);
}

// dL/dr of a pair from dL/dv and og (see the file comment).
__device__ __forceinline__ void pair_dr(bool dir, float rx, float ry, float rz, float rs,
                                        float v0, float v1, float v2, const float (&gv)[3],
                                        float og, float (&dr)[3]) {
  float g0 = gv[0], g1 = gv[1], g2 = gv[2];
  if (dir) {
    const float vg = v0 * g0 + v1 * g1 + v2 * g2;
    g0 = (g0 - v0 * vg) * rs;
    g1 = (g1 - v1 * vg) * rs;
    g2 = (g2 - v2 * vg) * rs;
  }
  const float c3 = og * rs * rs * rs * (float)(1.0 / (8.0 * HH_PI));
  dr[0] = g0 - rx * c3;
  dr[1] = g1 - ry * c3;
  dr[2] = g2 - rz * c3;
}

// Sum over the 32 lanes of half 0 (every lane active), in every lane.
__device__ __forceinline__ float half0_sum(float v) {
  v = (threadIdx.x & 32) ? 0.0f : v;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct VjpArgs {
  const float* fw;      // forward table (F32_FRAGS x 64)
  const float* bw;      // transposed table (BW_FRAGS x 64)
  const int4* nodes;
  const double* xs;
  double* dXs;
  double* slots;        // FP64 [waves][MLP_NP]
  int input_mode;
};

__device__ __forceinline__ void stage_tables(float* fw, float* bw, const VjpArgs& a) {
  for (int i = threadIdx.x; i < F32_FRAGS * 64; i += VB) fw[i] = a.fw[i];
  for (int i = threadIdx.x; i < BW_FRAGS * 64; i += VB) bw[i] = a.bw[i];
}

// Near pairs: persistent waves over the work units (fixed assignment, so the
// slot sums are reproducible).
__global__ __launch_bounds__(VB) void k_near_vjp_f32(VjpArgs a, const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ near_ptr,
                                                     const int2* __restrict__ H,
                                                     const int2* __restrict__ units,
                                                     int64_t n_units, const float* __restrict__ Fs,
                                                     const float* __restrict__ ws) {
  __shared__ float fw[F32_FRAGS * 64];
  __shared__ float bw[BW_FRAGS * 64];
  __shared__ float xbuf[VB / 64][2][64 * XS];
  stage_tables(fw, bw, a);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, p = lane & 31;
  float* XD = xbuf[w][0];
  float* XH = xbuf[w][1];
  const int64_t wave = (int64_t)blockIdx.x * (VB / 64) + w, nw = (int64_t)gridDim.x * (VB / 64);
  double* slot = a.slots + wave * MLP_NP;
  const bool dir = a.input_mode == HH_MLP_INPUT_DIRECTION;
  const float c8 = (float)(1.0 / (8.0 * HH_PI));
  VjpAcc A;
  acc_zero(A);
  int tiles = 0;
  for (int64_t u = wave; u < n_units; u += nw) {
    const int2 un = units[u];
    const int4 nt = a.nodes[leaves[un.x]];
    const int i = nt.x + 32 * un.y + p;
    const bool act = i < nt.y;
    const int ii = act ? i : nt.x;
    const double xi0 = a.xs[3 * (int64_t)ii], xi1 = a.xs[3 * (int64_t)ii + 1],
                 xi2 = a.xs[3 * (int64_t)ii + 2];
    const float w0 = ws[3 * (int64_t)ii], w1 = ws[3 * (int64_t)ii + 1], w2 = ws[3 * (int64_t)ii + 2];
    double t0 = 0, t1 = 0, t2 = 0;
    for (int pp = near_ptr[un.x]; pp < near_ptr[un.x + 1]; ++pp) {
      const int4 ns = a.nodes[H[pp].y];
      for (int j = ns.x; j < ns.y; ++j) {
        float rx = (float)(xi0 - a.xs[3 * (int64_t)j]);
        float ry = (float)(xi1 - a.xs[3 * (int64_t)j + 1]);
        float rz = (float)(xi2 - a.xs[3 * (int64_t)j + 2]);
        const bool skip = (j == ii) || !act;
        if (j == ii) { rx = 1.0f; ry = 0.0f; rz = 0.0f; }
        const float rs = hh_rsqrt(rx * rx + ry * ry + rz * rz);
        const float sv = dir ? rs : 1.0f;
        const float v0 = rx * sv, v1 = ry * sv, v2 = rz * sv;
        const float f0 = Fs[3 * (int64_t)j], f1 = Fs[3 * (int64_t)j + 1],
                    f2 = Fs[3 * (int64_t)j + 2];
        const float u0 = skip ? 0.0f : w0, u1 = skip ? 0.0f : w1, u2 = skip ? 0.0f : w2;
        // symmetric part of the cotangent w_i F_j^T
        const float g[9] = {u0 * f0, 0.5f * (u0 * f1 + u1 * f0), 0.5f * (u0 * f2 + u2 * f0),
                            0.5f * (u1 * f0 + u0 * f1), u1 * f1, 0.5f * (u1 * f2 + u2 * f1),
                            0.5f * (u2 * f0 + u0 * f2), 0.5f * (u2 * f1 + u1 * f2), u2 * f2};
        float gv[3], og, dr[3];
        vjp_tile_f32(fw, bw, XD, XH, A, v0, v1, v2, g, rs * c8, gv, og);
        pair_dr(dir, rx, ry, rz, rs, v0, v1, v2, gv, og, dr);
        if (!skip) { t0 += dr[0]; t1 += dr[1]; t2 += dr[2]; }
        const float s0 = half0_sum(skip ? 0.0f : dr[0]);
        const float s1 = half0_sum(skip ? 0.0f : dr[1]);
        const float s2 = half0_sum(skip ? 0.0f : dr[2]);
        if (lane == 0) {
          atomicAdd(a.dXs + 3 * (int64_t)j, -(double)s0);
          atomicAdd(a.dXs + 3 * (int64_t)j + 1, -(double)s1);
          atomicAdd(a.dXs + 3 * (int64_t)j + 2, -(double)s2);
        }
        if (++tiles == FLUSH) {
          acc_flush(A, slot);
          tiles = 0;
        }
      }
    }
    if (act && lane < 32) {
      atomicAdd(a.dXs + 3 * (int64_t)i, t0);
      atomicAdd(a.dXs + 3 * (int64_t)i + 1, t1);
      atomicAdd(a.dXs + 3 * (int64_t)i + 2, t2);
    }
  }
  acc_flush(A, slot);
}

// Sampled far pairs: the column samples (i, j_k) and row samples (i_k, j) of
// every term k of every admissible block, with the cotangents the ACA
// adjoint left in the pool; persistent waves over the blocks [b0, b1).
__global__ __launch_bounds__(VB) void k_far_vjp_f32(VjpArgs a, const int2* __restrict__ G,
                                                    int64_t b0, int64_t b1,
                                                    const int32_t* __restrict__ rank,
                                                    const int32_t* __restrict__ flag,
                                                    const int32_t* __restrict__ piv,
                                                    const int64_t* __restrict__ goff,
                                                    const float* __restrict__ gpool) {
  __shared__ float fw[F32_FRAGS * 64];
  __shared__ float bw[BW_FRAGS * 64];
  __shared__ float xbuf[VB / 64][2][64 * XS];
  stage_tables(fw, bw, a);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, p = lane & 31;
  float* XD = xbuf[w][0];
  float* XH = xbuf[w][1];
  const int64_t wave = (int64_t)blockIdx.x * (VB / 64) + w, nw = (int64_t)gridDim.x * (VB / 64);
  double* slot = a.slots + wave * MLP_NP;
  const bool dir = a.input_mode == HH_MLP_INPUT_DIRECTION;
  const float c8 = (float)(1.0 / (8.0 * HH_PI));
  VjpAcc A;
  acc_zero(A);
  int tiles = 0;
  for (int64_t b = b0 + wave; b < b1; b += nw) {
    if (flag[b] || rank[b] == 0) continue;
    const int2 gb = G[b];
    const int4 nt = a.nodes[gb.x], ns = a.nodes[gb.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x, l = rank[b];
    for (int k = 0; k < l; ++k) {
      const int ik = piv[b * 2 * LMAX_CAP + k], jk = piv[b * 2 * LMAX_CAP + LMAX_CAP + k];
      const float* gc = gpool + goff[b] + 9 * (int64_t)k * (c + q);
      const float* gr = gc + 9 * (int64_t)c;
      for (int t0 = 0; t0 < c + q; t0 += 32) {
        const int t = t0 + p;
        const bool ok = t < c + q;
        const int tt = ok ? t : 0;
        const bool colp = tt < c;
        const int i = colp ? nt.x + tt : nt.x + ik;
        const int j = colp ? ns.x + jk : ns.x + (tt - c);
        const float* gs = colp ? gc + 9 * (int64_t)tt : gr + 9 * (int64_t)(tt - c);
        float G9[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) G9[e] = ok ? gs[e] : 0.0f;
        const float g[9] = {G9[0], 0.5f * (G9[1] + G9[3]), 0.5f * (G9[2] + G9[6]),
                            0.5f * (G9[3] + G9[1]), G9[4], 0.5f * (G9[5] + G9[7]),
                            0.5f * (G9[6] + G9[2]), 0.5f * (G9[7] + G9[5]), G9[8]};
        const float rx = (float)(a.xs[3 * (int64_t)i] - a.xs[3 * (int64_t)j]);
        const float ry = (float)(a.xs[3 * (int64_t)i + 1] - a.xs[3 * (int64_t)j + 1]);
        const float rz = (float)(a.xs[3 * (int64_t)i + 2] - a.xs[3 * (int64_t)j + 2]);
        const float rs = hh_rsqrt(rx * rx + ry * ry + rz * rz);
        const float sv = dir ? rs : 1.0f;
        const float v0 = rx * sv, v1 = ry * sv, v2 = rz * sv;
        float gv[3], og, dr[3];
        vjp_tile_f32(fw, bw, XD, XH, A, v0, v1, v2, g, rs * c8, gv, og);
        pair_dr(dir, rx, ry, rz, rs, v0, v1, v2, gv, og, dr);
        // column samples share x_j (j = j_k), row samples share x_i (i = i_k):
        // those sides are summed over the tile first (one atomic each), the
        // other side is a distinct particle per lane
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float sc = half0_sum(ok && colp ? dr[d] : 0.0f);
          const float sr = half0_sum(ok && !colp ? dr[d] : 0.0f);
          if (lane == 0) {
            if (t0 < c) atomicAdd(a.dXs + 3 * (int64_t)(ns.x + jk) + d, -(double)sc);
            if (t0 + 32 > c) atomicAdd(a.dXs + 3 * (int64_t)(nt.x + ik) + d, (double)sr);
          }
          if (ok && lane < 32) {
            if (colp)
              atomicAdd(a.dXs + 3 * (int64_t)i + d, (double)dr[d]);
            else
              atomicAdd(a.dXs + 3 * (int64_t)j + d, -(double)dr[d]);
          }
        }
        if (++tiles == FLUSH) {
          acc_flush(A, slot);
          tiles = 0;
        }
      }
    }
  }
  acc_flush(A, slot);
}

}  // namespace

// Waves of the persistent MFMA back-propagation kernels (one workgroup of four
// waves per compute unit: the weight tables and the per-wave buffers take
// most of the LDS).
int64_t vjp_f32_waves(hh_ctx ctx) { return 4 * (int64_t)std::max(1, ctx->n_cu); }

static VjpArgs vjp_args(hh_tree t, hh_kernel k, double* dXs, double* slots) {
  VjpArgs a;
  a.fw = k->pf32.as<float>();
  a.bw = k->pf32t.as<float>();
  a.nodes = t->nodes.as<int4>();
  a.xs = t->xs.as<double>();
  a.dXs = dXs;
  a.slots = slots;
  a.input_mode = k->input_mode;
  return a;
}

// Near pairs: slots [vjp_f32_waves] x MLP_NP doubles (zeroed by the caller).
void launch_near_vjp_f32(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const float* Fs,
                         const float* ws, double* dXs, double* slots) {
  ensure_units(ctx, t);
  const VjpArgs a = vjp_args(t, k, dXs, slots);
  hipLaunchKernelGGL(k_near_vjp_f32, dim3((unsigned)(vjp_f32_waves(ctx) / 4)), dim3(VB), 0,
                     ctx->stream, a, t->leaves.as<int32_t>(), p->near_ptr.as<int32_t>(),
                     p->H.as<int2>(), t->units.as<int2>(), t->n_units, Fs, ws);
  HIP_OK(hipGetLastError());
}

// Sampled pairs of the blocks [b0, b1): slots as above (added to).
void launch_far_vjp_f32(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k,
                        int64_t b0, int64_t b1, const int64_t* goff, const float* gpool,
                        double* dXs, double* slots) {
  const VjpArgs a = vjp_args(t, k, dXs, slots);
  hipLaunchKernelGGL(k_far_vjp_f32, dim3((unsigned)(vjp_f32_waves(ctx) / 4)), dim3(VB), 0,
                     ctx->stream, a, p->G.as<int2>(), b0, b1, lr->rank.as<int32_t>(),
                     lr->flag.as<int32_t>(), lr->piv.as<int32_t>(), goff, gpool);
  HIP_OK(hipGetLastError());
}
