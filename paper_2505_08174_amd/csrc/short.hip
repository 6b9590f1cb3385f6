// Short-range many-body terms of the velocity (Eq. (6): M^(s,2) F + M^(t,3) F
// + M^(s,3) F; Eq. (2) with the normalisation of Eq. (4)):
//
//   U_i += sum_{j in N(i)} alpha_2^(s)(d_j) F_i
//        + sum_{k in N(i)} sum_{j in N(k), j != i} [alpha_3^(s) F_i + alpha_3^(t) F_j],
//
// d_j = x_j - x_i, N(i) the particles within the cut-off R_cut of particle i
// (Sec. 2.2), the inner double sum the 3-cliques (j, k, i) of Sec. 2.3.
//   alpha_2^(s) = sym(h_s(d_j / |d_j|)) / (8 pi |d_j|)
//   [alpha_3^(s) | alpha_3^(t)] = sym-blocks of g((d_j, d_k) / R_cut) / (8 pi |x_j - x_k| |x_k - x_i|)
// with h_s a 3-64-64-64-9 and g a 6-64-64-64-18 tanh MLP (seeded stand-ins
// for the trained networks of Sec. 2.4).
//
// Neighbours come from a uniform grid of cells of edge R_cut over the root box
// of the (single-system) tree: particles are sorted by cell (the radix sort of
// the tree), every particle scans the 27 cells around its own, and the
// neighbour lists are kept in CSR form in the tree's particle order. The
// product (FP64 form) is one thread per target particle, over its neighbours
// and then its 3-cliques, with both networks' weights in LDS. The FP32 forms
// run both networks on FP32 MFMA tiles with one wave per target particle:
// its neighbour pairs 32 at a time, then its 3-cliques packed 32 per tile
// across neighbours k (a prefix sum of the degrees of up to 64 neighbours
// maps a tile slot to its pair (k, j)). Each target's row is owned by one
// thread or wave, so the sums are deterministic and need no atomics.
#include <algorithm>

#include "api_guard.h"
#include "devmath.h"
#include "internal.h"
#include "mlp_mfma.h"

// FP32 MFMA fragment table (layout in mlp_mfma.h) of a packed two-body MLP
// (HH_MLP_NPARAM), context.hip.
std::vector<float> build_f32_frags(const double* P);

// Packed parameters of g (6-64-64-64-18), each W row-major [out][in].
#define G3_W1 0
#define G3_B1 (G3_W1 + MLP_H * 6)
#define G3_W2 (G3_B1 + MLP_H)
#define G3_B2 (G3_W2 + MLP_H * MLP_H)
#define G3_W3 (G3_B2 + MLP_H)
#define G3_B3 (G3_W3 + MLP_H * MLP_H)
#define G3_W4 (G3_B3 + MLP_H)
#define G3_B4 (G3_W4 + 18 * MLP_H)
#define G3_NP (G3_B4 + 18)
static_assert(G3_NP == HH_G3_NPARAM, "packed layout of the three-body network");

// The three-body network on the FP32 tile of mlp_mfma.h: the network 6 -> 64 -> 64 -> 64 -> 18 on the same FP32 tile: layer 1
// contracts (v0, v1), (v2, v3), (v4, v5) and (1, 0) (the bias), the hidden
// layers are those of the two-body tile (same table layout), and the output
// layer has 18 rows of one M tile. Layers 1-3 scaled by 2 log2(e).
#define G32_L1 0                               // [mo 2][step 4]
#define G32_L2 (G32_L1 + 8)
#define G32_L3 (G32_L2 + 66)
#define G32_L4 (G32_L3 + 66)                   // [mo 2][r 16], bias
#define G32_FRAGS (G32_L4 + 33)

// Raw outputs o[0..17] of the three-body network at input v[6] for this
// lane's pair (all 64 lanes; lanes l and l + 32 hold the same input).
__device__ __forceinline__ void mlp_tile_f32_g(const float* __restrict__ fr, const float (&v)[6],
                                               float (&o)[18]) {
  __asm__ volatile("" ::: "memory");
  const int lane = threadIdx.x & 63;
  const bool h1 = lane >= 32;
  const float bone = h1 ? 0.0f : 1.0f;
  float h[2][16], g[2][16];
  {
    const float b[4] = {h1 ? v[1] : v[0], h1 ? v[3] : v[2], h1 ? v[5] : v[4], bone};
#pragma unroll
    for (int mo = 0; mo < 2; ++mo) {
      f32x16 a = f32x16{};
#pragma unroll
      for (int st = 0; st < 4; ++st) a = mfma_f32(fr[(G32_L1 + 4 * mo + st) * 64 + lane], b[st], a);
#pragma unroll
      for (int r = 0; r < 16; ++r) h[mo][r] = tanh_scaled(a[r]);
    }
  }
  hidden_f32(fr, G32_L2, lane, bone, h, g);
  hidden_f32(fr, G32_L3, lane, bone, g, h);
  f32x16 c0 = mfma_f32(fr[(G32_L4 + 32) * 64 + lane], bone, f32x16{});
  f32x16 c1 = f32x16{};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    c0 = mfma_f32(fr[(G32_L4 + r) * 64 + lane], h[0][r], c0);
    c1 = mfma_f32(fr[(G32_L4 + 16 + r) * 64 + lane], h[1][r], c1);
  }
  // row 8 (r / 4) + 4 h + r % 4 of register r: rows 0-17 sit in registers 0-9
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const float mine = c0[r] + c1[r];
    const float other = __shfl_xor(mine, 32, 64);
    const int lo = 8 * (r / 4) + (r % 4), hi = lo + 4;
    if (lo < 18) o[lo] = h1 ? other : mine;
    if (hi < 18) o[hi] = h1 ? mine : other;
  }
}

// Fragment table of the three-body network on the FP32 tile (layout in
// mlp_mfma.h: G32_*), packed parameters as HH_G3_NPARAM: W1[64][6] b1[64]
// W2[64][64] b2[64] W3[64][64] b3[64] W4[18][64] b4[18].
static std::vector<float> build_g32_frags(const double* P0) {
  std::vector<float> fr((size_t)G32_FRAGS * 64, 0.0f);
  auto at = [&](int frag, int lane) -> float& { return fr[(size_t)frag * 64 + lane]; };
  const double S = 2.0 / log(2.0);
  const int W1 = 0, B1 = W1 + 64 * 6, W2 = B1 + 64, B2 = W2 + 64 * 64, W3 = B2 + 64,
            B3 = W3 + 64 * 64, W4 = B3 + 64, B4 = W4 + 18 * 64;
  auto feat = [](int mo, int r, int h) { return 32 * mo + 8 * (r / 4) + 4 * h + (r % 4); };
  for (int mo = 0; mo < 2; ++mo)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = 32 * mo + (lane & 31), h = lane >> 5;
      for (int st = 0; st < 3; ++st) at(G32_L1 + 4 * mo + st, lane) = (float)(S * P0[W1 + 6 * m + 2 * st + h]);
      at(G32_L1 + 4 * mo + 3, lane) = h == 0 ? (float)(S * P0[B1 + m]) : 0.0f;
    }
  auto hidden = [&](int base, int w, int b) {
    for (int mp = 0; mp < 2; ++mp)
      for (int lane = 0; lane < 64; ++lane) {
        const int m = 32 * mp + (lane & 31), h = lane >> 5;
        for (int mo = 0; mo < 2; ++mo)
          for (int r = 0; r < 16; ++r)
            at(base + (mp * 2 + mo) * 16 + r, lane) = (float)(S * P0[w + 64 * m + feat(mo, r, h)]);
        at(base + 64 + mp, lane) = h == 0 ? (float)(S * P0[b + m]) : 0.0f;
      }
  };
  hidden(G32_L2, W2, B2);
  hidden(G32_L3, W3, B3);
  for (int lane = 0; lane < 64; ++lane) {
    const int m = lane & 31, h = lane >> 5;
    if (m >= 18) continue;
    for (int mo = 0; mo < 2; ++mo)
      for (int r = 0; r < 16; ++r)
        at(G32_L4 + mo * 16 + r, lane) = (float)P0[W4 + 64 * m + feat(mo, r, h)];
    if (h == 0) at(G32_L4 + 32, lane) = (float)P0[B4 + m];
  }
  return fr;
}

struct hh_short_s {
  hh_ctx ctx = nullptr;
  hh_tree tree = nullptr;
  double r_cut = 5.0;
  int64_t n = 0, n_pairs = 0, n_cliques = 0;
  DevBuf nb_ptr;           // int64 [n + 1] CSR of N(i), tree order
  DevBuf nb;               // int32 [n_pairs] neighbour positions (tree order)
  DevBuf w2_64, w2_32;     // h_s parameters (HH_MLP_NPARAM)
  DevBuf w3_64, w3_32;     // g parameters (HH_G3_NPARAM)
  DevBuf ws_f;             // forces in tree order (workspace of a product)
  DevBuf fr_h, fr_g;       // FP32 MFMA fragment tables of h_s and g
};

namespace {

constexpr int TB = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + TB - 1) / TB); }

struct Grid {
  double lo[3];
  double inv;      // 1 / cell edge
  int64_t g[3];    // cells per axis
};

__device__ __forceinline__ int64_t cell_coord(double x, double lo, double inv, int64_t g) {
  int64_t c = (int64_t)floor((x - lo) * inv);
  return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

__global__ __launch_bounds__(TB) void k_cell_key(const double* __restrict__ xs, int64_t n,
                                                 Grid G, uint64_t* __restrict__ key,
                                                 uint32_t* __restrict__ val,
                                                 int64_t* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  const int64_t cx = cell_coord(xs[3 * s], G.lo[0], G.inv, G.g[0]);
  const int64_t cy = cell_coord(xs[3 * s + 1], G.lo[1], G.inv, G.g[1]);
  const int64_t cz = cell_coord(xs[3 * s + 2], G.lo[2], G.inv, G.g[2]);
  const int64_t c = (cz * G.g[1] + cy) * G.g[0] + cx;
  key[s] = (uint64_t)c;
  val[s] = (uint32_t)s;
  atomicAdd((unsigned long long*)&cnt[c], 1ull);
}

// Neighbours of particle s (tree order) by the 27 cells around its own:
// counts them (out == nullptr) or writes them at out. The cut-off test is
// (dx^2 + dy^2) + dz^2 < r_cut^2 in FP64 with every operation rounded.
#pragma clang fp contract(off)
__device__ __forceinline__ int64_t scan_cells(const double* __restrict__ xs, int64_t s, Grid G,
                                              double rc2, const int64_t* __restrict__ cstart,
                                              const uint32_t* __restrict__ cval,
                                              int32_t* __restrict__ out) {
  const double x0 = xs[3 * s], x1 = xs[3 * s + 1], x2 = xs[3 * s + 2];
  const int64_t cx = cell_coord(x0, G.lo[0], G.inv, G.g[0]);
  const int64_t cy = cell_coord(x1, G.lo[1], G.inv, G.g[1]);
  const int64_t cz = cell_coord(x2, G.lo[2], G.inv, G.g[2]);
  int64_t m = 0;
  for (int64_t z = max(cz - 1, (int64_t)0); z <= min(cz + 1, G.g[2] - 1); ++z)
    for (int64_t y = max(cy - 1, (int64_t)0); y <= min(cy + 1, G.g[1] - 1); ++y)
      for (int64_t x = max(cx - 1, (int64_t)0); x <= min(cx + 1, G.g[0] - 1); ++x) {
        const int64_t c = (z * G.g[1] + y) * G.g[0] + x;
        for (int64_t p = cstart[c]; p < cstart[c + 1]; ++p) {
          const int64_t j = cval[p];
          if (j == s) continue;
          const double d0 = xs[3 * j] - x0, d1 = xs[3 * j + 1] - x1, d2 = xs[3 * j + 2] - x2;
          if (d0 * d0 + d1 * d1 + d2 * d2 < rc2) {
            if (out) out[m] = (int32_t)j;
            ++m;
          }
        }
      }
  return m;
}

#pragma clang fp contract(on)

__global__ __launch_bounds__(TB) void k_nb_count(const double* __restrict__ xs, int64_t n, Grid G,
                                                 double rc2, const int64_t* __restrict__ cstart,
                                                 const uint32_t* __restrict__ cval,
                                                 int64_t* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  cnt[s] = scan_cells(xs, s, G, rc2, cstart, cval, nullptr);
}

__global__ __launch_bounds__(TB) void k_nb_fill(const double* __restrict__ xs, int64_t n, Grid G,
                                                double rc2, const int64_t* __restrict__ cstart,
                                                const uint32_t* __restrict__ cval,
                                                const int64_t* __restrict__ ptr,
                                                int32_t* __restrict__ nb) {
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  scan_cells(xs, s, G, rc2, cstart, cval, nb + ptr[s]);
}

// 3-cliques with target s: sum over k in N(s) of |N(k)| - 1 (j runs over
// N(k) without s, and s is in N(k) because the relation is symmetric).
__global__ __launch_bounds__(TB) void k_clique_count(const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ nb, int64_t n,
                                                     int64_t* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  int64_t m = 0;
  for (int64_t p = ptr[s]; p < ptr[s + 1]; ++p) {
    const int k = nb[p];
    m += ptr[k + 1] - ptr[k] - 1;
  }
  cnt[s] = m;
}

template <class TI, class T>
__global__ __launch_bounds__(TB) void k_gather_f(const TI* __restrict__ F,
                                                 const int32_t* __restrict__ perm, int64_t n,
                                                 T* __restrict__ Fs) {
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  const int64_t o = perm[s];
  Fs[3 * s] = (T)F[3 * o];
  Fs[3 * s + 1] = (T)F[3 * o + 1];
  Fs[3 * s + 2] = (T)F[3 * o + 2];
}

// Raw outputs o[18] of g at input v (6 values).
template <class T>
__device__ __forceinline__ void g3_raw(const T* __restrict__ P, const T (&v)[6], T o[18]) {
  T h1[MLP_H], h2[MLP_H];
#pragma unroll
  for (int k = 0; k < MLP_H; ++k) {
    T z = P[G3_B1 + k];
#pragma unroll
    for (int d = 0; d < 6; ++d) z += P[G3_W1 + 6 * k + d] * v[d];
    h1[k] = hh_tanh(z);
  }
#pragma unroll 4
  for (int a = 0; a < MLP_H; ++a) {
    T z = P[G3_B2 + a];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z += P[G3_W2 + MLP_H * a + k] * h1[k];
    h2[a] = hh_tanh(z);
  }
#pragma unroll 4
  for (int a = 0; a < MLP_H; ++a) {
    T z = P[G3_B3 + a];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z += P[G3_W3 + MLP_H * a + k] * h2[k];
    h1[a] = hh_tanh(z);
  }
#pragma unroll
  for (int m = 0; m < 18; ++m) {
    T z = P[G3_B4 + m];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z += P[G3_W4 + MLP_H * m + k] * h1[k];
    o[m] = z;
  }
}

// u += sym(O) f for the row-major 3x3 O given as o[0..8] (sym(O) = (O + O^T)/2)
template <class T>
__device__ __forceinline__ void add_sym(const T* o, T s, T f0, T f1, T f2, double& u0,
                                        double& u1, double& u2) {
  const T a01 = T(0.5) * (o[1] + o[3]), a02 = T(0.5) * (o[2] + o[6]),
          a12 = T(0.5) * (o[5] + o[7]);
  u0 += (double)(s * (o[0] * f0 + a01 * f1 + a02 * f2));
  u1 += (double)(s * (a01 * f0 + o[4] * f1 + a12 * f2));
  u2 += (double)(s * (a02 * f0 + a12 * f1 + o[8] * f2));
}

template <class T, class TU>
__global__ __launch_bounds__(TB) void k_short(const double* __restrict__ xs,
                                              const int32_t* __restrict__ perm, int64_t n,
                                              const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ nb,
                                              const T* __restrict__ w2, const T* __restrict__ w3,
                                              double inv_rc, const T* __restrict__ Fs,
                                              TU* __restrict__ U) {
  __shared__ T l2[MLP_NP];
  __shared__ T l3[G3_NP];
  for (int i = threadIdx.x; i < MLP_NP; i += TB) l2[i] = w2[i];
  for (int i = threadIdx.x; i < G3_NP; i += TB) l3[i] = w3[i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  const double x0 = xs[3 * s], x1 = xs[3 * s + 1], x2 = xs[3 * s + 2];
  const T f0 = Fs[3 * s], f1 = Fs[3 * s + 1], f2 = Fs[3 * s + 2];
  double u0 = 0, u1 = 0, u2 = 0;
  const int64_t p0 = ptr[s], p1 = ptr[s + 1];
  // two-body self term: sum_j alpha_2^(s)(x_j - x_i) F_i
  for (int64_t p = p0; p < p1; ++p) {
    const int64_t j = nb[p];
    T K[9];
    mlp_entry<T, T>(l2, HH_MLP_INPUT_DIRECTION, (T)(xs[3 * j] - x0), (T)(xs[3 * j + 1] - x1),
                    (T)(xs[3 * j + 2] - x2), K);
    u0 += (double)(K[0] * f0 + K[1] * f1 + K[2] * f2);
    u1 += (double)(K[3] * f0 + K[4] * f1 + K[5] * f2);
    u2 += (double)(K[6] * f0 + K[7] * f1 + K[8] * f2);
  }
  // three-body terms over the 3-cliques (j, k, s)
  for (int64_t p = p0; p < p1; ++p) {
    const int64_t k = nb[p];
    const double k0 = xs[3 * k] - x0, k1 = xs[3 * k + 1] - x1, k2 = xs[3 * k + 2] - x2;
    const double rki = sqrt(k0 * k0 + k1 * k1 + k2 * k2);
    for (int64_t q = ptr[k]; q < ptr[k + 1]; ++q) {
      const int64_t j = nb[q];
      if (j == s) continue;
      const double j0 = xs[3 * j] - x0, j1 = xs[3 * j + 1] - x1, j2 = xs[3 * j + 2] - x2;
      const double e0 = j0 - k0, e1 = j1 - k1, e2 = j2 - k2;
      const double rjk = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      const T v[6] = {(T)(j0 * inv_rc), (T)(j1 * inv_rc), (T)(j2 * inv_rc),
                      (T)(k0 * inv_rc), (T)(k1 * inv_rc), (T)(k2 * inv_rc)};
      T o[18];
      g3_raw<T>(l3, v, o);
      const T sc = (T)(1.0 / (8.0 * HH_PI * rjk * rki));
      add_sym<T>(o, sc, f0, f1, f2, u0, u1, u2);
      add_sym<T>(o + 9, sc, Fs[3 * j], Fs[3 * j + 1], Fs[3 * j + 2], u0, u1, u2);
    }
  }
  const int64_t o = perm[s];
  U[3 * o] = (TU)((double)U[3 * o] + u0);
  U[3 * o + 1] = (TU)((double)U[3 * o + 1] + u1);
  U[3 * o + 2] = (TU)((double)U[3 * o + 2] + u2);
}

constexpr int SB = 512;   // eight waves per workgroup

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Short-range terms of the FP32 forms on FP32 MFMA tiles, one wave per target
// particle s (tree order), persistent waves with a fixed assignment.
template <class TU>
__global__ __launch_bounds__(SB) void k_short_f32(const double* __restrict__ xs,
                                                  const int32_t* __restrict__ perm, int64_t n,
                                                  const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ nb,
                                                  const float4* __restrict__ frh,
                                                  const float4* __restrict__ frg, double inv_rc,
                                                  const float* __restrict__ Fs,
                                                  TU* __restrict__ U) {
  __shared__ float fh[F32_FRAGS * 64];
  __shared__ float fg[G32_FRAGS * 64];
  __shared__ int pref[SB / 64][65];
  __shared__ int kk[SB / 64][64];
  stage_frags_f32(fh, frh, SB);
  {
    float4* d = reinterpret_cast<float4*>(fg);
    for (int i = threadIdx.x; i < G32_FRAGS * 16; i += SB) d[i] = frg[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, p = lane & 31;
  const bool h0 = lane < 32;
  const int64_t wave = (int64_t)blockIdx.x * (SB / 64) + w, nw = (int64_t)gridDim.x * (SB / 64);
  const double c8 = 1.0 / (8.0 * HH_PI);
  for (int64_t s = wave; s < n; s += nw) {
    const double x0 = xs[3 * s], x1 = xs[3 * s + 1], x2 = xs[3 * s + 2];
    const float f0 = Fs[3 * s], f1 = Fs[3 * s + 1], f2 = Fs[3 * s + 2];
    const int64_t p0 = ptr[s], p1 = ptr[s + 1];
    double u0 = 0, u1 = 0, u2 = 0;
    // two-body self term: sum_j alpha_2^(s)(x_j - x_i) F_i, 32 neighbours per tile
    for (int64_t t0 = p0; t0 < p1; t0 += 32) {
      const int64_t q = t0 + p;
      const bool ok = q < p1;
      const int64_t j = nb[ok ? q : p0];
      float K[9];
      entry_f32tile(fh, HH_MLP_INPUT_DIRECTION, xs[3 * j] - x0, xs[3 * j + 1] - x1,
                    xs[3 * j + 2] - x2, K);
      if (ok && h0) {
        u0 += (double)(K[0] * f0 + K[1] * f1 + K[2] * f2);
        u1 += (double)(K[3] * f0 + K[4] * f1 + K[5] * f2);
        u2 += (double)(K[6] * f0 + K[7] * f1 + K[8] * f2);
      }
    }
    // three-body terms over the 3-cliques (j, k, s), up to 64 neighbours k at a time
    for (int64_t g0 = p0; g0 < p1; g0 += 64) {
      const int64_t pk = g0 + lane;
      const bool okk = pk < p1;
      const int k = okk ? nb[pk] : 0;
      const int dk = okk ? (int)(ptr[k + 1] - ptr[k]) : 0;
      const int incl = wave_incl_scan(dk);
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
      pref[w][lane + 1] = incl;
      kk[w][lane] = k;
      if (lane == 0) pref[w][0] = 0;
      const int tot = __shfl(incl, 63, 64);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
      for (int t0 = 0; t0 < tot; t0 += 32) {
        const int t1 = t0 + p;
        const bool okt = t1 < tot;
        const int t = okt ? t1 : 0;
        int lo = 0, hi = 64;   // pref[lo] <= t < pref[hi]
#pragma unroll
        for (int it = 0; it < 6; ++it) {
          const int mid = (lo + hi) >> 1;
          if (pref[w][mid] <= t) lo = mid; else hi = mid;
        }
        const int kv = kk[w][lo];
        const int64_t j = nb[ptr[kv] + (t - pref[w][lo])];
        const bool valid = okt && j != s;
        const double k0 = xs[3 * (int64_t)kv] - x0, k1 = xs[3 * (int64_t)kv + 1] - x1,
                     k2 = xs[3 * (int64_t)kv + 2] - x2;
        const double j0 = xs[3 * j] - x0, j1 = xs[3 * j + 1] - x1, j2 = xs[3 * j + 2] - x2;
        const double e0 = j0 - k0, e1 = j1 - k1, e2 = j2 - k2;
        const double rki = sqrt(k0 * k0 + k1 * k1 + k2 * k2);
        const double rjk = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        const float v[6] = {(float)(j0 * inv_rc), (float)(j1 * inv_rc), (float)(j2 * inv_rc),
                            (float)(k0 * inv_rc), (float)(k1 * inv_rc), (float)(k2 * inv_rc)};
        float o[18];
        mlp_tile_f32_g(fg, v, o);
        if (valid && h0) {
          const float sc = (float)(c8 / (rjk * rki));
          add_sym<float>(o, sc, f0, f1, f2, u0, u1, u2);
          add_sym<float>(o + 9, sc, Fs[3 * j], Fs[3 * j + 1], Fs[3 * j + 2], u0, u1, u2);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();   // pref and kk are read before the next group
    }
    u0 = wave_sum_d(u0);
    u1 = wave_sum_d(u1);
    u2 = wave_sum_d(u2);
    if (lane == 0) {
      const int64_t o = perm[s];
      U[3 * o] = (TU)((double)U[3 * o] + u0);
      U[3 * o + 1] = (TU)((double)U[3 * o + 1] + u1);
      U[3 * o + 2] = (TU)((double)U[3 * o + 2] + u2);
    }
  }
}

template <class T>
void upload_params(hh_ctx ctx, DevBuf& d, const double* p, int np) {
  std::vector<T> v(p, p + np);
  d.alloc(ctx->stream, np * sizeof(T));
  HIP_OK(hipMemcpyAsync(d.p, v.data(), np * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  ctx_sync(ctx);   // v is freed on return
}

template <class T, class TI, class TU>
void short_matvec_t(hh_ctx ctx, hh_short_s* sh, const void* F, void* U) {
  hipStream_t st = ctx->stream;
  hh_tree t = sh->tree;
  const int64_t n = sh->n;
  sh->ws_f.ensure(st, 3 * n * sizeof(T));
  hipLaunchKernelGGL((k_gather_f<TI, T>), dim3(nblk(n)), dim3(TB), 0, st, (const TI*)F,
                     t->perm.as<int32_t>(), n, sh->ws_f.as<T>());
  if constexpr (sizeof(T) == 4) {
    const unsigned grid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((n + SB / 64 - 1) / (SB / 64), ctx->n_cu));
    hipLaunchKernelGGL((k_short_f32<TU>), dim3(grid), dim3(SB), 0, st, t->xs.as<double>(),
                       t->perm.as<int32_t>(), n, sh->nb_ptr.as<int64_t>(), sh->nb.as<int32_t>(),
                       sh->fr_h.as<float4>(), sh->fr_g.as<float4>(), 1.0 / sh->r_cut,
                       sh->ws_f.as<float>(), (TU*)U);
  } else {
    hipLaunchKernelGGL((k_short<T, TU>), dim3(nblk(n)), dim3(TB), 0, st, t->xs.as<double>(),
                       t->perm.as<int32_t>(), n, sh->nb_ptr.as<int64_t>(), sh->nb.as<int32_t>(),
                       sh->w2_64.as<T>(), sh->w3_64.as<T>(), 1.0 / sh->r_cut, sh->ws_f.as<T>(),
                       (TU*)U);
  }
  HIP_OK(hipGetLastError());
}

}  // namespace

extern "C" {

hh_status hh_short_create(hh_ctx ctx, hh_tree tree, const double* s2_params,
                          const double* g3_params, double r_cut, hh_short* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && tree && s2_params && g3_params, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(tree->ctx == ctx, HH_ERR_INVALID_ARG, "tree belongs to another context");
  HH_REQUIRE(tree->n_sys == 1 && !tree->six, HH_ERR_INVALID_ARG,
             "the short-range terms take a single-system tree of particles");
  HH_REQUIRE(r_cut > 0 && std::isfinite(r_cut), HH_ERR_INVALID_ARG, "r_cut must be > 0");
  for (int i = 0; i < MLP_NP; ++i)
    HH_REQUIRE(std::isfinite(s2_params[i]), HH_ERR_INVALID_ARG, "non-finite parameter");
  for (int i = 0; i < G3_NP; ++i)
    HH_REQUIRE(std::isfinite(g3_params[i]), HH_ERR_INVALID_ARG, "non-finite parameter");
  hipStream_t st = ctx->stream;
  PhaseTimer timer(ctx, HH_PHASE_SHORT);
  hh_short_s* sh = new hh_short_s();
  try {
    sh->ctx = ctx;
    sh->tree = tree;
    sh->r_cut = r_cut;
    const int64_t n = tree->n;
    sh->n = n;
    upload_params<double>(ctx, sh->w2_64, s2_params, MLP_NP);
    upload_params<float>(ctx, sh->w2_32, s2_params, MLP_NP);
    upload_params<double>(ctx, sh->w3_64, g3_params, G3_NP);
    upload_params<float>(ctx, sh->w3_32, g3_params, G3_NP);
    {
      const std::vector<float> fh = build_f32_frags(s2_params), fg = build_g32_frags(g3_params);
      sh->fr_h.alloc(st, fh.size() * sizeof(float));
      sh->fr_g.alloc(st, fg.size() * sizeof(float));
      HIP_OK(hipMemcpyAsync(sh->fr_h.p, fh.data(), fh.size() * sizeof(float),
                            hipMemcpyHostToDevice, st));
      HIP_OK(hipMemcpyAsync(sh->fr_g.p, fg.data(), fg.size() * sizeof(float),
                            hipMemcpyHostToDevice, st));
      ctx_sync(ctx);   // the host tables are freed on return
    }
    // cell grid over the root box (node 0)
    double bb[6];
    read_bytes(ctx, bb, tree->bbox.p, 6 * sizeof(double));
    Grid G;
    G.inv = 1.0 / r_cut;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
      G.lo[d] = bb[d];
      const double ext = (bb[3 + d] - bb[d]) / r_cut;
      HH_REQUIRE(ext < 2e6, HH_ERR_CAPACITY, "the cell grid would be too large");
      G.g[d] = (int64_t)floor(ext) + 1;
      ncell *= G.g[d];
    }
    HH_REQUIRE(ncell < (1ll << 31), HH_ERR_CAPACITY, "the cell grid would be too large");
    DevBuf key, val, cnt, cstart;
    key.alloc(st, n * sizeof(uint64_t));
    val.alloc(st, n * sizeof(uint32_t));
    cnt.alloc(st, (ncell + 1) * sizeof(int64_t));
    cstart.alloc(st, (ncell + 1) * sizeof(int64_t));
    zero_words(ctx, cnt.p, ncell + 1);
    hipLaunchKernelGGL(k_cell_key, dim3(nblk(n)), dim3(TB), 0, st, tree->xs.as<double>(), n, G,
                       key.as<uint64_t>(), val.as<uint32_t>(), cnt.as<int64_t>());
    HIP_OK(hipGetLastError());
    int bits = 1;
    while ((1ll << bits) < ncell) ++bits;
    radix_sort_u64(ctx, key.as<uint64_t>(), val.as<uint32_t>(), n, bits);
    scan_exclusive_i64(ctx, cnt.as<int64_t>(), cstart.as<int64_t>(), ncell + 1);
    const double rc2 = r_cut * r_cut;
    DevBuf ncnt;
    ncnt.alloc(st, (n + 1) * sizeof(int64_t));
    zero_words(ctx, ncnt.p, n + 1);
    hipLaunchKernelGGL(k_nb_count, dim3(nblk(n)), dim3(TB), 0, st, tree->xs.as<double>(), n, G,
                       rc2, cstart.as<int64_t>(), val.as<uint32_t>(), ncnt.as<int64_t>());
    sh->nb_ptr.alloc(st, (n + 1) * sizeof(int64_t));
    scan_exclusive_i64(ctx, ncnt.as<int64_t>(), sh->nb_ptr.as<int64_t>(), n + 1);
    sh->n_pairs = read_i64(ctx, sh->nb_ptr.as<int64_t>() + n);
    HH_REQUIRE(sh->n_pairs < (1ll << 40), HH_ERR_CAPACITY, "too many neighbour pairs");
    sh->nb.alloc(st, std::max<int64_t>(sh->n_pairs, 1) * sizeof(int32_t));
    hipLaunchKernelGGL(k_nb_fill, dim3(nblk(n)), dim3(TB), 0, st, tree->xs.as<double>(), n, G,
                       rc2, cstart.as<int64_t>(), val.as<uint32_t>(), sh->nb_ptr.as<int64_t>(),
                       sh->nb.as<int32_t>());
    zero_words(ctx, ncnt.p, n + 1);
    hipLaunchKernelGGL(k_clique_count, dim3(nblk(n)), dim3(TB), 0, st, sh->nb_ptr.as<int64_t>(),
                       sh->nb.as<int32_t>(), n, ncnt.as<int64_t>());
    scan_exclusive_i64(ctx, ncnt.as<int64_t>(), ncnt.as<int64_t>(), n + 1);
    sh->n_cliques = read_i64(ctx, ncnt.as<int64_t>() + n);
    HIP_OK(hipGetLastError());
  } catch (...) {
    delete sh;
    throw;
  }
  *out = sh;
  HH_API_END(ctx)
}

hh_status hh_short_matvec(hh_ctx ctx, hh_short s, hh_precision prec, const void* F, void* U) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(s && F && U, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(s->ctx == ctx, HH_ERR_INVALID_ARG, "handle belongs to another context");
  PhaseTimer timer(ctx, HH_PHASE_SHORT);
  if (prec == HH_FP64)
    short_matvec_t<double, double, double>(ctx, s, F, U);
  else if (prec == HH_FP32)
    short_matvec_t<float, float, float>(ctx, s, F, U);
  else if (is_bf16(prec))
    short_matvec_t<float, float, double>(ctx, s, F, U);
  else
    HH_REQUIRE(false, HH_ERR_INVALID_ARG, "unknown precision");
  HH_API_END(ctx)
}

hh_status hh_short_info(hh_short s, int64_t* n_pairs, int64_t* n_cliques) {
  if (!s) return HH_ERR_INVALID_ARG;
  if (n_pairs) *n_pairs = s->n_pairs;
  if (n_cliques) *n_cliques = s->n_cliques;
  return HH_OK;
}

void hh_short_free(hh_short s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  delete s;
}

}  // extern "C"
