// Adaptive cross approximation with 3x3 entries (Algorithm 2, Eqs. (8)-(10)).
//
// One wave (64 lanes) per admissible block, fetched from a global work
// counter (dynamic load balance; the results do not depend on the order).
// The rank loop runs inside the wave:
//   column j_k: a(i) = K(x_i - y_j) - sum_{m<k} c_m(i) q_m(j)
//   i_k = argmax over unused rows of the pivot magnitude, lowest index on ties
//   c_k(i) = a(i) P^-1, P = a(i_k)
//   row i_k:  q_k(j) = K(x_ik - y_j) - sum_{m<k} c_m(i_k) q_m(j)
//   j_{k+1} = argmax over unused columns of the pivot magnitude of q_k(j)
//   nu^2 = tr(A_kk B_kk), lambda^2 += nu^2 + 2 sum_{m<k} tr(A_mk B_km)
//   with A_mk = sum_i c_m(i)^T c_k(i), B_km = sum_j q_k(j) q_m(j)^T
//   stop when nu^2 <= eps^2 lambda^2 or after min(c, q) terms.
// Pivot magnitude: squared Frobenius norm in the FP64 form (Algorithm 2);
// |det| of the 3x3 entry in the FP32 and BF16 forms (the magnitude the text
// around Eq. (9) names), which avoids nearly singular pivots whose inverse
// would amplify single-precision rounding in c_k = a P^-1. The 6N kernel
// takes |det| in every form: its translation-rotation entries are singular
// (antisymmetric 3x3), and the Frobenius rule would pick them as pivots.
// Guards: a residual column with ||a||^2 <= 1e-30 lambda^2 ends as converged
// without a new term; |det P| <= s ||P||_F^3 ends with a dense fallback, with
// s = 1e-14 under the Frobenius rule (a singularity guard) and s = 1e-8 under
// the |det| rule: ||P||_F^3 / |det P| bounds the 2-norm condition number of a
// 3x3 P, and when the best-conditioned entry of the column exceeds 1e8 the
// inverse would carry FP64 rounding into c_k beyond 1e-8 relative. With FP32
// residuals (the FP32 and BF16 forms) s = 1e-6, about 16 units of FP32
// roundoff: a residual entry that is singular in exact arithmetic (the 6N
// grid's coupling entries and their Schur complements) comes out of FP32
// arithmetic with |det P| / ||P||_F^3 near the roundoff, and inverting it
// would fill c_k with rounding noise;
// l_max terms without convergence end with a dense fallback.
// Factors c_k (c entries) and q_k (q entries), 9 values each, are stored
// contiguously per step in a pool, followed by the pivot entry P_k (9 values);
// each step bump-allocates 9 (c + q + 1) values. In streamed mode the factors
// of a step take 9 (c + q) values of the worker's arena.
// Samples, residuals and factors are in the working type T; pivots, norms,
// the normalisation and Gram matrices in FP64 in every form (a lane's
// two-row share of Ghat_m is formed in T before the FP64 wave sum). In the
// BF16 form the samples come from the MFMA MLP tile (activations carried as
// BF16 hi + lo).
#include <algorithm>
#include <iterator>

#include "devmath.h"
#include "internal.h"
#include "mlp_mfma.h"

namespace {

constexpr int AW = 8;              // block workers (waves) per workgroup
constexpr int AW_T = 64 * AW;
constexpr int RCH = 2;             // rows per lane per chunk
constexpr int CH = 64 * RCH;       // rows per chunk

template <class T>
struct AcaArgs {
  const int2* G;
  int64_t nG;
  const int32_t* order;   // blocks of each launch range, largest first
  const int4* nodes;
  const double* xs;
  KParams kp;
  double eps2;
  int l_max;
  int32_t* rank;
  int32_t* flag;
  int32_t* piv;      // [nG][2][LMAX_CAP]
  int64_t* fptr;     // [nG][LMAX_CAP]
  T* pool;
  int64_t pool_elems;
  T* arena;             // per-wave factor arenas (streamed mode)
  int64_t arena_elems;  // elements per wave arena; a workgroup team owns AW of them
  T* huge;              // arenas of the workgroups that take the huge blocks
  // huge blocks in tiers of one size class each, largest first (streamed
  // mode): tier t is order[b0 + tier_b[t] .. b0 + tier_b[t+1]); workgroups
  // [tier_wg[t], tier_wg[t+1]) own arenas of tier_cap[t] elements starting at
  // huge + tier_off[t], take tier t and then the smaller tiers
  int ntier;
  int tier_wg[ACA_MAX_TIERS + 1];
  int64_t tier_b[ACA_MAX_TIERS + 1];
  int64_t tier_cap[ACA_MAX_TIERS];
  int64_t tier_off[ACA_MAX_TIERS];
  int64_t slot0_w;      // first worker slot (Gram history, arena) of the single waves
  unsigned long long* pool_top;
  int* overflow;
  int* work;         // dynamic block counter (blocks worked on by single waves)
  int* work_big;     // dynamic block counter (blocks worked on by whole workgroups)
  int* work_huge;    // dynamic block counters, one per huge tier (streamed mode)
  int64_t nhuge;     // order[b0 .. b0 + nhuge) are huge (streamed mode)
  int64_t nbig;      // then order[.. + nbig) go to whole workgroups
  int64_t b0, b1;    // block range of this launch
  // fused apply (streamed mode): Fs != nullptr
  const T* Fs;       // sorted forces
  double* ublk;      // per-block output rows [c][3], at uoff[pos] - uoff[b0]
  const int64_t* uoff;   // prefix sums of c over the work order (streamed mode)
  const uint4* frags;   // BF16 MFMA weight fragments (BF16 sampling)
  const float4* frags32;   // FP32 MFMA weight fragments (FP32 sampling)
  int det_pivot;        // pivot magnitude |det| (else squared Frobenius norm)
  double* gram;         // Gram history A (gram_half doubles) and cross-wave
  int64_t gram_stride;  // partials, gram_stride doubles per worker
  int64_t gram_half;
};

template <class NT, class T>
__device__ __forceinline__ NT det3(const T* K) {
  return fabs((NT)K[0] * ((NT)K[4] * (NT)K[8] - (NT)K[5] * (NT)K[7]) -
              (NT)K[1] * ((NT)K[3] * (NT)K[8] - (NT)K[5] * (NT)K[6]) +
              (NT)K[2] * ((NT)K[3] * (NT)K[7] - (NT)K[4] * (NT)K[6]));
}

// MFMA sampling of the kernel MLP: MFK = 1 BF16 tiles (hi + lo activations),
// MFK = 2 FP32 tiles; fr is the matching fragment table in LDS.
enum { MF_NONE = 0, MF_BF16 = 1, MF_F32 = 2 };

// K(x_i - y_j) from NT independent MFMA MLP tiles: symmetrised 3x3 entries
// of this lane's pair of each tile.
template <int NT, int MFK>
__device__ __forceinline__ void mfma_entries(const void* fr, int mode, const double (&d)[NT][3],
                                             float (&K)[NT][9]) {
  if constexpr (MFK == MF_F32) {
#pragma unroll
    for (int t = 0; t < NT; ++t) entry_f32tile((const float*)fr, mode, d[t][0], d[t][1], d[t][2], K[t]);
    return;
  }
  float v[NT][3], rs[NT], o[NT][9];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const float rx = (float)d[t][0], ry = (float)d[t][1], rz = (float)d[t][2];
    rs[t] = hh_rsqrt(rx * rx + ry * ry + rz * rz);
    const float sc = mode == HH_MLP_INPUT_DIRECTION ? rs[t] : 1.0f;
    v[t][0] = rx * sc;
    v[t][1] = ry * sc;
    v[t][2] = rz * sc;
  }
  mlp_tiles_bf16<true, NT>((const bf16x8*)fr, v, o);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const float s = rs[t] * (float)(1.0 / (16.0 * HH_PI));
    K[t][0] = 2.0f * o[t][0] * s; K[t][1] = (o[t][1] + o[t][3]) * s; K[t][2] = (o[t][2] + o[t][6]) * s;
    K[t][3] = K[t][1];            K[t][4] = 2.0f * o[t][4] * s;       K[t][5] = (o[t][5] + o[t][7]) * s;
    K[t][6] = K[t][2];            K[t][7] = K[t][5];                  K[t][8] = 2.0f * o[t][8] * s;
  }
}

template <int MFK>
__device__ __forceinline__ void mfma_entry(const void* fr, int mode, double dx, double dy,
                                           double dz, float K[9]) {
  const double d[1][3] = {{dx, dy, dz}};
  float k1[1][9];
  mfma_entries<1, MFK>(fr, mode, d, k1);
#pragma unroll
  for (int e = 0; e < 9; ++e) K[e] = k1[0][e];
}

__device__ __forceinline__ int tri(int m) { return m * (m + 1) / 2; }

// Orders the wave's earlier global and LDS writes before its later reads by
// other lanes (all lanes of one wave share the CU's L1 and LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// v + (v of the source lane given by a DPP control), 0 where the source lane
// is outside the row or the row is masked off
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int slo, shi;
  if (ROW_MASK == 0xf) {   // every row written; invalid source lanes read 0
    slo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, true);
    shi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, true);
  } else {                 // rows masked off keep the 0 they start from
    slo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
    shi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
  }
  return v + __hiloint2double(shi, slo);
}

// Sum over the wave of each p[e], returned in every lane: scans by row shifts 1, 2,
// 4, 8 inside each 16-lane row (lane 15 of a row then holds the row sum), row
// 0 into row 1 and row 2 into row 3 (lane 15 broadcast), rows 0-1 into rows
// 2-3 (lane 31 broadcast), so lane 63 holds the total. No LDS traffic.
template <int N>
__device__ __forceinline__ void wave_sumv(double (&p)[N]) {
#pragma unroll
  for (int e = 0; e < N; ++e) {
    double v = p[e];
    v = dpp_add<0x111, 0xf>(v);   // row_shr:1
    v = dpp_add<0x112, 0xf>(v);   // row_shr:2
    v = dpp_add<0x114, 0xf>(v);   // row_shr:4
    v = dpp_add<0x118, 0xf>(v);   // row_shr:8
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    p[e] = __hiloint2double(hi, lo);
  }
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// K -= A B (3x3, row-major)
template <class T>
__device__ __forceinline__ void sub_mm(T K[9], const T A[9], const T B[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      K[3 * r + cc] -= A[3 * r] * B[cc] + A[3 * r + 1] * B[3 + cc] + A[3 * r + 2] * B[6 + cc];
}

__device__ __forceinline__ void mul_mm(const double A[9], const double B[9], double O[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      O[3 * r + cc] = A[3 * r] * B[cc] + A[3 * r + 1] * B[3 + cc] + A[3 * r + 2] * B[6 + cc];
}

// 3x3 history matrix of the Gram store, transposed when lo > hi
__device__ __forceinline__ void load_hist(const double* __restrict__ h, int m1, int m2,
                                          double M[9]) {
  if (m1 <= m2) {
    const double* s = h + 9 * (tri(m2) + m1);
#pragma unroll
    for (int e = 0; e < 9; ++e) M[e] = s[e];
  } else {
    const double* s = h + 9 * (tri(m1) + m2);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) M[3 * r + cc] = s[3 * cc + r];
  }
}

// Entries 9 i .. 9 i + 8 of f for the rows i = i0 + 64 r (r < RCH), zero past n.
template <class T>
__device__ __forceinline__ void load_rows(const T* __restrict__ f, int i0, int n, T (&v)[RCH][9]) {
#pragma unroll
  for (int r = 0; r < RCH; ++r) {
    const int i = i0 + 64 * r;
#pragma unroll
    for (int e = 0; e < 9; ++e) v[r][e] = i < n ? f[9 * (int64_t)i + e] : T(0);
  }
}

// Scratch of one worker team (TW waves) for the block it approximates.
template <class T>
struct TeamSh {
  T qc[LMAX_CAP * 9];     // q_m(j_k) in the column pass, c_m(i_k) in the row pass
  int64_t off[LMAX_CAP];  // pool offset of factor m
  int pi[LMAX_CAP];
  int pj[LMAX_CAP + 1];
  double am[LMAX_CAP * 9];  // A_mk = sum_i c_m(i)^T c_k(i), m < k (row pass)
  int64_t bo;             // broadcast: claimed block, pool offset
  int ovf;                // broadcast: pool overflow
};

// Cross-wave partial results of a team of AW waves (one per workgroup).
struct TeamRed {
  double v[AW][16];
  int i[AW];
};

template <int TW>
__device__ __forceinline__ void team_sync() {
  if constexpr (TW == 1)
    wave_sync();
  else
    __syncthreads();
}

// Raw samples K(sgn (p_i - y)) for rows i in [0, n) of `pts`, written to
// slot[9 i ..]: 32-row MFMA tiles, lanes l and l + 32 share a row, the tiles
// spread over the TW waves of the team.
template <int NT, int MFK>
__device__ __forceinline__ void sample_tiles(const void* fr, int mode, const double* pts, int n,
                                             double y0, double y1, double y2, double sgn,
                                             float* slot, int t0, int step) {
  const int lane = threadIdx.x & 63;
  double d[NT][3];
  int row[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int tb = t0 + t * step;
    const int i = tb + (lane & 31);
    row[t] = i;
    const int ii = i < n ? i : tb;
    d[t][0] = sgn * (pts[3 * ii] - y0);
    d[t][1] = sgn * (pts[3 * ii + 1] - y1);
    d[t][2] = sgn * (pts[3 * ii + 2] - y2);
  }
  float K[NT][9];
  mfma_entries<NT, MFK>(fr, mode, d, K);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int i = row[t];
    if (i < n) {
      if (lane < 32) {
#pragma unroll
        for (int e = 0; e < 5; ++e) slot[9 * (int64_t)i + e] = K[t][e];
      } else {
#pragma unroll
        for (int e = 5; e < 9; ++e) slot[9 * (int64_t)i + e] = K[t][e];
      }
    }
  }
}

template <int TW, int MFK>
__device__ __forceinline__ void sample_mfma(const void* fr, int mode, const double* pts, int n,
                                            double y0, double y1, double y2, double sgn,
                                            float* slot, int wit) {
  // this wave's tiles t0, t0 + 32 TW, ... in pairs (two independent MFMA chains)
  const int step = 32 * TW;
  int t0 = 32 * wit;
#pragma unroll 1
  for (; t0 + step < n; t0 += 2 * step)
    sample_tiles<2, MFK>(fr, mode, pts, n, y0, y1, y2, sgn, slot, t0, step);
  if (t0 < n) sample_tiles<1, MFK>(fr, mode, pts, n, y0, y1, y2, sgn, slot, t0, step);
}

// Combines the per-wave results of a pass over the team: sums v[0..NV) in
// wave order, max of the two magnitudes, argmax (ties to the lowest index),
// and sums the per-m partials (lane m of every wave) through global scratch.
template <int TW, int NV>
__device__ __forceinline__ void team_combine(TeamRed* tr, double* gx, int wit, int k,
                                             double (&v)[NV], double& mx1, double& mx2,
                                             double& best, int& bi, double (&G)[9]) {
  if constexpr (TW > 1) {
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
      for (int e = 0; e < NV; ++e) tr->v[wit][e] = v[e];
      tr->v[wit][NV] = mx1;
      tr->v[wit][NV + 1] = mx2;
      tr->v[wit][NV + 2] = best;
      tr->i[wit] = bi;
    }
    if (lane < k) {
      double* d = gx + 9 * (64 * wit + lane);
#pragma unroll
      for (int e = 0; e < 9; ++e) d[e] = G[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      double s = 0;
      for (int w = 0; w < TW; ++w) s += tr->v[w][e];
      v[e] = s;
    }
    mx1 = tr->v[0][NV];
    mx2 = tr->v[0][NV + 1];
    best = tr->v[0][NV + 2];
    bi = tr->i[0];
    for (int w = 1; w < TW; ++w) {
      mx1 = tr->v[w][NV] > mx1 ? tr->v[w][NV] : mx1;
      mx2 = tr->v[w][NV + 1] > mx2 ? tr->v[w][NV + 1] : mx2;
      const double bw = tr->v[w][NV + 2];
      const int iw = tr->i[w];
      if (bw > best || (bw == best && iw < bi)) { best = bw; bi = iw; }
    }
    if (lane < k) {
#pragma unroll
      for (int e = 0; e < 9; ++e) G[e] = 0;
      for (int w = 0; w < TW; ++w) {
        const double* s = gx + 9 * (64 * w + lane);
#pragma unroll
        for (int e = 0; e < 9; ++e) G[e] += s[e];
      }
    }
    __syncthreads();
  }
}

// ACA of the blocks order[r0 .. r1) by teams of TW waves; `counter` hands out
// the blocks. Per step k:
//   column pass: raw column g(i) = K(x_i - y_j); residual
//     a(i) = g(i) - sum_{m<k} c_m(i) q_m(j_k), subtracting term by term
//     (partial residuals r_m = g - sum_{m'<m} ..., r_k = a); in the same pass
//     Ghat_m = sum_i c_m(i)^T r_m(i) (one wave reduction per m and chunk);
//   pivot i_k, c_k = a P^-1;
//   A_mk = sum_i c_m(i)^T c_k(i) = (Ghat_m - sum_{m<=m'<k} A_mm' q_m'(j_k)) P^-1
//     from the stored Gram history A_mm' (lane m works on m);
//   row pass: q_k(j) = h(j) - sum_m c_m(i_k) q_m(j), and in the same pass
//     V(j) = sum_{m<k} A_mk^T q_m(j), so that the cross terms
//     sum_{m<k} tr(A_mk B_km) = sum_j <V(j), q_k(j)>_F (B_km = sum_j q_k(j) q_m(j)^T)
//     take one scalar reduction; B_kk = sum_j q_k(j) q_k(j)^T;
//   nu^2 = tr(A_kk B_kk), lambda^2 += nu^2 + 2 sum_{m<k} tr(A_mk B_km).
// So the Gram terms cost no extra pass over the factors. Every wave of a team
// computes the per-step scalars itself from the same combined values, so all
// decisions are uniform over the team. Fused apply: u(i) += c_{k-1}(i) t_{k-1}
// rides on the next column pass (or a final pass).
template <class T, int KIND, int MF, int TW>
__device__ __forceinline__ void aca_worker(const AcaArgs<T>& a, const T* wl, const void* fr,
                                           TeamSh<T>& sh, TeamRed* tr, int wit, int64_t slot,
                                           int* counter, int64_t r0, int64_t r1, T* fbase,
                                           int64_t fcap) {
  using NT = double;
  const int lane = threadIdx.x & 63;
  const bool lead = wit == 0 && lane == 0;
  const int stride = 64 * TW;   // threads of the team
  const int tid = 64 * wit + lane;
  double* hA = a.gram + slot * a.gram_stride;
  double* gx = hA + a.gram_half;   // cross-wave partials, [AW][64][9]
#pragma unroll 1
  for (;;) {
    if (lead) sh.bo = atomicAdd(counter, 1);
    team_sync<TW>();
    const int64_t sb = sh.bo;
    if (r0 + sb >= r1) break;
    const int64_t pos = r0 + sb;
    const int64_t b = a.order[pos];
    const int2 g2 = a.G[b];
    const int4 nt = a.nodes[g2.x], ns = a.nodes[g2.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x;
    const double* xt = a.xs + 3 * (int64_t)nt.x;
    const double* xsr = a.xs + 3 * (int64_t)ns.x;
    const int kmax = min(min(c, q), a.l_max);
    // factor storage: the worker's own arena (fcap elements; offsets restart
    // with every block), or the shared pool, bump-allocated (fbase == null)
    const bool own = fbase != nullptr;
    T* const fb = own ? fbase : a.pool;
    int j = q / 2;
    int rank = 0;
    bool converged = false, fallback = false, pending = false;
    double lam2 = 0;
    const bool fuse = a.Fs != nullptr;
    double* ub = fuse ? a.ublk + 3 * (a.uoff[pos] - a.uoff[a.b0]) : nullptr;
    if (fuse)
#pragma unroll 1
      for (int i = tid; i < 3 * c; i += stride) ub[i] = 0.0;
    double tp0 = 0, tp1 = 0, tp2 = 0;   // t_{k-1} = sum_j q_{k-1}(j) F_j
#pragma unroll 1
    for (int k = 0; k < kmax; ++k) {
      team_sync<TW>();   // sh.bo and sh.qc of the previous step are consumed
      if (lead) {
        // c_k, q_k and (stored factors) the pivot entry P_k for the adjoint
        const unsigned long long need = 9ull * (unsigned long long)(c + q + (fuse ? 0 : 1));
        unsigned long long o;
        int ovf = 0;
        if (own) {
          o = (unsigned long long)k * need;
          ovf = (int64_t)(o + need) > fcap;
        } else {
          o = atomicAdd(a.pool_top, need);
          ovf = (int64_t)(o + need) > a.pool_elems;
        }
        if (ovf) atomicOr(a.overflow, 1);
        sh.bo = (int64_t)o;
        sh.ovf = ovf;
        sh.off[k] = (int64_t)o;
        sh.pj[k] = j;
        a.fptr[b * LMAX_CAP + k] = (int64_t)o;
      }
      team_sync<TW>();
      if (sh.ovf) { fallback = true; break; }
      const int64_t offv = sh.bo;
#pragma unroll 1
      for (int t = tid; t < 9 * k; t += stride) {
        const int m = t / 9, e = t - 9 * m;
        sh.qc[t] = fb[sh.off[m] + 9 * (int64_t)c + 9 * (int64_t)j + e];
      }
      T* Ck = fb + offv;
      T* Qk = Ck + 9 * (int64_t)c;
      const double yj0 = xsr[3 * j], yj1 = xsr[3 * j + 1], yj2 = xsr[3 * j + 2];
      if (MF) sample_mfma<TW, MF>(fr, a.kp.input_mode, xt, c, yj0, yj1, yj2, 1.0, (float*)Ck, wit);
      team_sync<TW>();
      // ---- column pass: residual, Ghat, pivot search, sum a^T a
      NT best = -1, bestf = -1, graw = 0;
      int bi = 0x7fffffff;
      double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
      for (int base = CH * wit; base < c; base += CH * TW) {
        T rs[RCH][9];
#pragma unroll
        for (int r = 0; r < RCH; ++r) {
          const int i = base + 64 * r + lane;
          if (i < c) {
            if (MF) {
#pragma unroll
              for (int e = 0; e < 9; ++e) rs[r][e] = Ck[9 * (int64_t)i + e];
            } else {
              kernel_entry<T>(a.kp, wl, (T)(xt[3 * i] - yj0), (T)(xt[3 * i + 1] - yj1),
                              (T)(xt[3 * i + 2] - yj2), rs[r], i & 1, j & 1);
            }
          } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) rs[r][e] = 0;
          }
          if (sizeof(T) == 4) {
            NT g2s = 0;
#pragma unroll
            for (int e = 0; e < 9; ++e) g2s += (NT)rs[r][e] * (NT)rs[r][e];
            graw = g2s > graw ? g2s : graw;
          }
        }
        // c_m(i) of the next m is loaded while m is worked on
        T cn[RCH][9];
        if (k > 0) load_rows<T>(fb + sh.off[0], base + lane, c, cn);
#pragma unroll 1
        for (int m = 0; m < k; ++m) {
          T cc[RCH][9];
#pragma unroll
          for (int r = 0; r < RCH; ++r)
#pragma unroll
            for (int e = 0; e < 9; ++e) cc[r][e] = cn[r][e];
          if (m + 1 < k) load_rows<T>(fb + sh.off[m + 1], base + lane, c, cn);
          T qv[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) qv[e] = sh.qc[9 * m + e];
          // this lane's rows of c_m(i)^T r_m(i): products of the working type
          // (FP32 in the single-precision forms), summed over the wave in FP64
          T pl[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
          for (int r = 0; r < RCH; ++r) {
            const int i = base + 64 * r + lane;
            const T* cv = cc[r];
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
              for (int y = 0; y < 3; ++y)
                pl[3 * x + y] += cv[x] * rs[r][y] + cv[3 + x] * rs[r][3 + y] + cv[6 + x] * rs[r][6 + y];
            sub_mm<T>(rs[r], cv, qv);
            if (fuse && m == k - 1 && i < c) {
              ub[3 * i] += (double)cv[0] * tp0 + (double)cv[1] * tp1 + (double)cv[2] * tp2;
              ub[3 * i + 1] += (double)cv[3] * tp0 + (double)cv[4] * tp1 + (double)cv[5] * tp2;
              ub[3 * i + 2] += (double)cv[6] * tp0 + (double)cv[7] * tp1 + (double)cv[8] * tp2;
            }
          }
          double p[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) p[e] = (double)pl[e];
          wave_sumv(p);
          if (lane == m) {
#pragma unroll
            for (int e = 0; e < 9; ++e) G[e] += p[e];
          }
        }
#pragma unroll
        for (int r = 0; r < RCH; ++r) {
          const int i = base + 64 * r + lane;
          if (i >= c) continue;
          NT nrm = 0;
#pragma unroll
          for (int e = 0; e < 9; ++e) {
            Ck[9 * (int64_t)i + e] = rs[r][e];
            nrm += (NT)rs[r][e] * (NT)rs[r][e];
          }
#pragma unroll
          for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y)
              S[3 * x + y] += (double)rs[r][x] * (double)rs[r][y] +
                              (double)rs[r][3 + x] * (double)rs[r][3 + y] +
                              (double)rs[r][6 + x] * (double)rs[r][6 + y];
          NT sel = a.det_pivot ? det3<NT>(rs[r]) : nrm;
          bool used = false;
#pragma unroll 1
          for (int m = 0; m < k; ++m) used |= (sh.pi[m] == i);
          if (used) { nrm = -1; sel = -1; }
          if (sel > best || (sel == best && i < bi)) { best = sel; bi = i; }
          bestf = nrm > bestf ? nrm : bestf;
        }
      }
      pending = false;   // the term k-1 is applied
      wave_sumv(S);
      if (sizeof(T) == 4) graw = wave_max(graw);
      wave_argmax(best, bi);
      bestf = wave_max(bestf);
      team_combine<TW>(tr, gx, wit, k, S, graw, bestf, best, bi, G);
      if (!a.det_pivot) bestf = best;
      // no usable row (all used or non-finite): stop without a new term
      if (!(best >= NT(0)) || bi < 0 || bi >= c) { fallback = true; break; }
      if (bestf <= NT(1e-30) * (NT)lam2) { converged = true; break; }
      // single precision: a residual at the rounding level of the raw column
      // (32 units of roundoff) carries no information; the block is converged
      if (sizeof(T) == 4 && bestf <= NT(3.6e-12) * graw) { converged = true; break; }
      team_sync<TW>();
      // pivot entry, determinant test and inverse in FP64 (every lane)
      double P[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) P[e] = (double)Ck[9 * (int64_t)bi + e];
      // stored factors keep the pivot entry P_k = a(i_k) after q_k (the
      // backward differentiates c_k = a P_k^-1 with the P_k that was used)
      if (!fuse && lead) {
        T* ps = Ck + 9 * (int64_t)(c + q);
#pragma unroll
        for (int e = 0; e < 9; ++e) ps[e] = Ck[9 * (int64_t)bi + e];
      }
      // every wave of a team holds P before the normalisation below
      // overwrites row i_k (a single wave loads it before it stores)
      if constexpr (TW > 1) __syncthreads();
      const double det = P[0] * (P[4] * P[8] - P[5] * P[7]) - P[1] * (P[3] * P[8] - P[5] * P[6]) +
                         P[2] * (P[3] * P[7] - P[4] * P[6]);
      double fro2 = 0;
#pragma unroll
      for (int e = 0; e < 9; ++e) fro2 += P[e] * P[e];
      const double sing = !a.det_pivot ? 1e-14 : sizeof(T) == 4 ? 1e-6 : 1e-8;
      if (!(fabs(det) > sing * fro2 * sqrt(fro2))) { fallback = true; break; }
      const double id = 1.0 / det;
      double Pi[9];
      Pi[0] = (P[4] * P[8] - P[5] * P[7]) * id;
      Pi[1] = (P[2] * P[7] - P[1] * P[8]) * id;
      Pi[2] = (P[1] * P[5] - P[2] * P[4]) * id;
      Pi[3] = (P[5] * P[6] - P[3] * P[8]) * id;
      Pi[4] = (P[0] * P[8] - P[2] * P[6]) * id;
      Pi[5] = (P[2] * P[3] - P[0] * P[5]) * id;
      Pi[6] = (P[3] * P[7] - P[4] * P[6]) * id;
      Pi[7] = (P[1] * P[6] - P[0] * P[7]) * id;
      Pi[8] = (P[0] * P[4] - P[1] * P[3]) * id;
      const int ik = bi;
      if (lead) sh.pi[k] = ik;
      // A_kk = Pi^T S Pi; A_mk = (Ghat_m - sum_m' A_mm' q_m'(j)) Pi (lane m)
      double Akk[9];
      {
        double SP[9], PiT[9];
        mul_mm(S, Pi, SP);
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y) PiT[3 * x + y] = Pi[3 * y + x];
        mul_mm(PiT, SP, Akk);
      }
      if (lane < k) {
#pragma unroll 1
        for (int m2 = lane; m2 < k; ++m2) {
          double Am[9], qd[9];
          load_hist(hA, lane, m2, Am);
#pragma unroll
          for (int e = 0; e < 9; ++e) qd[e] = (double)sh.qc[9 * m2 + e];
          sub_mm<double>(G, Am, qd);
        }
        double Amk[9];
        mul_mm(G, Pi, Amk);
        if (wit == 0) {
          double* d = hA + 9 * (tri(k) + lane);
#pragma unroll
          for (int e = 0; e < 9; ++e) {
            d[e] = Amk[e];
            sh.am[9 * lane + e] = Amk[e];
          }
        }
      }
      if (lead) {
        double* d = hA + 9 * (tri(k) + k);
#pragma unroll
        for (int e = 0; e < 9; ++e) d[e] = Akk[e];
      }
      // normalisation: c_k = a P^-1 in FP64, rounded to T once (P^-1 rounded
      // to single precision first would carry its rounding into c_k times the
      // condition number of P)
#pragma unroll 1
      for (int i = tid; i < c; i += stride) {
        double v[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) v[e] = (double)Ck[9 * (int64_t)i + e];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            Ck[9 * (int64_t)i + 3 * r + cc] =
                (T)(v[3 * r] * Pi[cc] + v[3 * r + 1] * Pi[3 + cc] + v[3 * r + 2] * Pi[6 + cc]);
      }
      team_sync<TW>();   // A side done with sh.qc; c_k written
#pragma unroll 1
      for (int t = tid; t < 9 * k; t += stride) {
        const int m = t / 9, e = t - 9 * m;
        sh.qc[t] = fb[sh.off[m] + 9 * (int64_t)ik + e];
      }
      const double xi0 = xt[3 * ik], xi1 = xt[3 * ik + 1], xi2 = xt[3 * ik + 2];
      if (MF) sample_mfma<TW, MF>(fr, a.kp.input_mode, xsr, q, xi0, xi1, xi2, -1.0, (float*)Qk, wit);
      team_sync<TW>();
      // ---- row pass: residual, Bhat, next column pivot, sum q_k q_k^T, t_k
      best = -1;
      bi = 0x7fffffff;
      // B_kk = sum_j q_k(j) q_k(j)^T (9), t_k (3), cross term (1):
      // sum_{m<k} tr(A_mk B_km) = sum_j < sum_{m<k} A_mk^T q_m(j), q_k(j) >_F
      double SB[13];
#pragma unroll
      for (int e = 0; e < 13; ++e) SB[e] = 0;
#pragma unroll 1
      for (int base = CH * wit; base < q; base += CH * TW) {
        T rs[RCH][9];
#pragma unroll
        for (int r = 0; r < RCH; ++r) {
          const int jj = base + 64 * r + lane;
          if (jj < q) {
            if (MF) {
#pragma unroll
              for (int e = 0; e < 9; ++e) rs[r][e] = Qk[9 * (int64_t)jj + e];
            } else {
              kernel_entry<T>(a.kp, wl, (T)(xi0 - xsr[3 * jj]), (T)(xi1 - xsr[3 * jj + 1]),
                              (T)(xi2 - xsr[3 * jj + 2]), rs[r], ik & 1, jj & 1);
            }
          } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) rs[r][e] = 0;
          }
        }
        double V[RCH][9];   // sum_{m<k} A_mk^T q_m(j)
#pragma unroll
        for (int r = 0; r < RCH; ++r)
#pragma unroll
          for (int e = 0; e < 9; ++e) V[r][e] = 0;
        // q_m(j) of the next m is loaded while m is worked on
        T qn[RCH][9];
        if (k > 0) load_rows<T>(fb + sh.off[0] + 9 * (int64_t)c, base + lane, q, qn);
#pragma unroll 1
        for (int m = 0; m < k; ++m) {
          T qq[RCH][9];
#pragma unroll
          for (int r = 0; r < RCH; ++r)
#pragma unroll
            for (int e = 0; e < 9; ++e) qq[r][e] = qn[r][e];
          if (m + 1 < k) load_rows<T>(fb + sh.off[m + 1] + 9 * (int64_t)c, base + lane, q, qn);
          T cv[9];
          double am[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) {
            cv[e] = sh.qc[9 * m + e];
            am[e] = sh.am[9 * m + e];
          }
#pragma unroll
          for (int r = 0; r < RCH; ++r) {
            const T* qv = qq[r];
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
              for (int y = 0; y < 3; ++y)
                V[r][3 * x + y] += am[x] * (double)qv[y] + am[3 + x] * (double)qv[3 + y] +
                                   am[6 + x] * (double)qv[6 + y];
            sub_mm<T>(rs[r], cv, qv);
          }
        }
#pragma unroll
        for (int r = 0; r < RCH; ++r) {
          const int jj = base + 64 * r + lane;
          if (jj >= q) continue;
          NT nrm = 0;
#pragma unroll
          for (int e = 0; e < 9; ++e) {
            Qk[9 * (int64_t)jj + e] = rs[r][e];
            nrm += (NT)rs[r][e] * (NT)rs[r][e];
          }
#pragma unroll
          for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y)
              SB[3 * x + y] += (double)rs[r][3 * x] * (double)rs[r][3 * y] +
                               (double)rs[r][3 * x + 1] * (double)rs[r][3 * y + 1] +
                               (double)rs[r][3 * x + 2] * (double)rs[r][3 * y + 2];
#pragma unroll
          for (int e = 0; e < 9; ++e) SB[12] += V[r][e] * (double)rs[r][e];
          if (fuse) {
            const T* f = a.Fs + 3 * ((int64_t)ns.x + jj);
            const double f0 = f[0], f1 = f[1], f2 = f[2];
            SB[9] += (double)rs[r][0] * f0 + (double)rs[r][1] * f1 + (double)rs[r][2] * f2;
            SB[10] += (double)rs[r][3] * f0 + (double)rs[r][4] * f1 + (double)rs[r][5] * f2;
            SB[11] += (double)rs[r][6] * f0 + (double)rs[r][7] * f1 + (double)rs[r][8] * f2;
          }
          NT sel = a.det_pivot ? det3<NT>(rs[r]) : nrm;
          bool used = false;
#pragma unroll 1
          for (int m = 0; m <= k; ++m) used |= (sh.pj[m] == jj);
          if (used) sel = -1;
          if (sel > best || (sel == best && jj < bi)) { best = sel; bi = jj; }
        }
      }
      wave_sumv(SB);
      wave_argmax(best, bi);
      {
        double d1 = 0, d2 = 0;
        team_combine<TW>(tr, gx, wit, 0, SB, d1, d2, best, bi, G);
      }
      const int jn = (bi >= 0 && bi < q) ? bi : -1;   // -1 only when every column is used
      const double cross = SB[12];
      double nu2 = 0;
      {
        const double* akk = hA + 9 * (tri(k) + k);   // A_kk, written by the lead lane
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y) nu2 += akk[3 * x + y] * SB[3 * y + x];
      }
      lam2 = lam2 + nu2 + 2.0 * cross;
      tp0 = SB[9];
      tp1 = SB[10];
      tp2 = SB[11];
      pending = true;
      rank = k + 1;
      if (nu2 <= a.eps2 * lam2) { converged = true; break; }
      if (k + 1 == min(c, q)) { converged = true; break; }
      if (jn < 0) { fallback = true; break; }
      j = jn;
    }
    if (!converged) fallback = true;
    team_sync<TW>();
    if (fuse && !fallback && pending) {
      // apply of the last term
      const T* cl = fb + sh.off[rank - 1];
#pragma unroll 1
      for (int i = tid; i < c; i += stride) {
        const T* e = cl + 9 * (int64_t)i;
        ub[3 * i] += (double)e[0] * tp0 + (double)e[1] * tp1 + (double)e[2] * tp2;
        ub[3 * i + 1] += (double)e[3] * tp0 + (double)e[4] * tp1 + (double)e[5] * tp2;
        ub[3 * i + 2] += (double)e[6] * tp0 + (double)e[7] * tp1 + (double)e[8] * tp2;
      }
    }
    if (fuse && fallback && MF) {
      // dense evaluation of the block's rows (32-row MFMA tiles)
#pragma unroll 1
      for (int t0 = 32 * wit; t0 < c; t0 += 32 * TW) {
        const int i = t0 + (lane & 31);
        const int ii = i < c ? i : t0;
        const double x0 = xt[3 * ii], x1 = xt[3 * ii + 1], x2 = xt[3 * ii + 2];
        double v0 = 0, v1 = 0, v2 = 0;
#pragma unroll 1
        for (int jj = 0; jj < q; ++jj) {
          float K[9];
          mfma_entry<MF>(fr, a.kp.input_mode, x0 - xsr[3 * jj], x1 - xsr[3 * jj + 1],
                     x2 - xsr[3 * jj + 2], K);
          const T* f = a.Fs + 3 * ((int64_t)ns.x + jj);
          v0 += (double)(K[0] * (float)f[0] + K[1] * (float)f[1] + K[2] * (float)f[2]);
          v1 += (double)(K[3] * (float)f[0] + K[4] * (float)f[1] + K[5] * (float)f[2]);
          v2 += (double)(K[6] * (float)f[0] + K[7] * (float)f[1] + K[8] * (float)f[2]);
        }
        if (i < c && lane < 32) {
          ub[3 * i] = v0;
          ub[3 * i + 1] = v1;
          ub[3 * i + 2] = v2;
        }
      }
    }
    if (fuse && fallback && !MF) {
      // dense evaluation of the block's rows replaces the partial sum
#pragma unroll 1
      for (int i = tid; i < c; i += stride) {
        const double x0 = xt[3 * i], x1 = xt[3 * i + 1], x2 = xt[3 * i + 2];
        T v0 = 0, v1 = 0, v2 = 0;
#pragma unroll 1
        for (int jj = 0; jj < q; ++jj) {
          T K[9];
          kernel_entry<T>(a.kp, wl, (T)(x0 - xsr[3 * jj]), (T)(x1 - xsr[3 * jj + 1]),
                          (T)(x2 - xsr[3 * jj + 2]), K, i & 1, jj & 1);
          const T* f = a.Fs + 3 * ((int64_t)ns.x + jj);
          v0 += K[0] * f[0] + K[1] * f[1] + K[2] * f[2];
          v1 += K[3] * f[0] + K[4] * f[1] + K[5] * f[2];
          v2 += K[6] * f[0] + K[7] * f[1] + K[8] * f[2];
        }
        ub[3 * i] = v0;
        ub[3 * i + 1] = v1;
        ub[3 * i + 2] = v2;
      }
    }
    if (lead) {
      a.rank[b] = rank;
      a.flag[b] = fallback ? 1 : 0;
    }
    if (wit == 0) {
#pragma unroll 1
      for (int t = lane; t < 2 * LMAX_CAP; t += 64) {
        const int m = t % LMAX_CAP;
        int v = -1;
        if (m < rank) v = (t < LMAX_CAP) ? sh.pi[m] : sh.pj[m];
        a.piv[b * 2 * LMAX_CAP + t] = v;
      }
    }
    team_sync<TW>();
  }
}

// Workgroups of AW waves working as one team per block. Streamed mode: the
// first tier_wg[ntier] workgroups start on the huge blocks order[b0 .. b0 +
// nhuge), tier by tier from their own (each in its own large arena). Then
// every workgroup takes the large blocks (the next nbig in the order, largest
// first).
template <class T, int KIND, int MF>
__global__ __launch_bounds__(AW_T) void k_aca_team(AcaArgs<T> a) {
  __shared__ T wl[(KIND == KIND_MLP && !MF) ? MLP_NP : 1];
  __shared__ bf16x8 frb[MF == MF_BF16 ? FR_TOTAL : 1];
  __shared__ float frf[MF == MF_F32 ? F32_FRAGS * 64 : 1];
  __shared__ TeamSh<T> sh;
  __shared__ TeamRed tr;
  const void* fr = MF == MF_F32 ? (const void*)frf : (const void*)frb;
  if (MF == MF_BF16) {
    stage_frags(frb, a.frags, AW_T);
  } else if (MF == MF_F32) {
    stage_frags_f32(frf, a.frags32, AW_T);
  } else if (KIND == KIND_MLP) {
    const T* w = (const T*)a.kp.w;
    for (int i = threadIdx.x; i < MLP_NP; i += AW_T) wl[i] = w[i];
  }
  __syncthreads();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int64_t wg = blockIdx.x;
  const bool ar = a.arena != nullptr;   // streamed mode: arenas, else the shared pool
  const int64_t r1 = a.b0 + a.nhuge, r2 = r1 + a.nbig;
  if (a.ntier > 0 && wg < a.tier_wg[a.ntier]) {
    int t0 = 0;
    while (wg >= a.tier_wg[t0 + 1]) ++t0;
    T* own = a.huge + a.tier_off[t0] + (wg - a.tier_wg[t0]) * a.tier_cap[t0];
#pragma unroll 1
    for (int tt = t0; tt < a.ntier; ++tt) {
      // a smaller size class may still need more (a thin block's rank bound
      // is larger); such a tier is left to its own workgroups
      if (a.tier_cap[tt] > a.tier_cap[t0]) continue;
      aca_worker<T, KIND, MF, AW>(a, wl, fr, sh, &tr, wv, wg * AW, a.work_huge + tt,
                                  a.b0 + a.tier_b[tt], a.b0 + a.tier_b[tt + 1], own,
                                  a.tier_cap[t0]);
      __syncthreads();   // sh.bo of the last fetch is read by every wave
    }
  }
  __syncthreads();
  aca_worker<T, KIND, MF, AW>(a, wl, fr, sh, &tr, wv, wg * AW, a.work_big, r1, r2,
                              ar ? a.arena + wg * AW * a.arena_elems : nullptr,
                              AW * a.arena_elems);
}

// Workgroups of AW waves, every wave a worker on its own small blocks
// order[b0 + nhuge + nbig .. b1) (largest first).
template <class T, int KIND, int MF>
__global__ __launch_bounds__(AW_T) void k_aca(AcaArgs<T> a) {
  __shared__ T wl[(KIND == KIND_MLP && !MF) ? MLP_NP : 1];
  __shared__ bf16x8 frb[MF == MF_BF16 ? FR_TOTAL : 1];
  __shared__ float frf[MF == MF_F32 ? F32_FRAGS * 64 : 1];
  __shared__ TeamSh<T> shw[AW];
  const void* fr = MF == MF_F32 ? (const void*)frf : (const void*)frb;
  if (MF == MF_BF16) {
    stage_frags(frb, a.frags, AW_T);
  } else if (MF == MF_F32) {
    stage_frags_f32(frf, a.frags32, AW_T);
  } else if (KIND == KIND_MLP) {
    const T* w = (const T*)a.kp.w;
    for (int i = threadIdx.x; i < MLP_NP; i += AW_T) wl[i] = w[i];
  }
  __syncthreads();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int64_t wg = blockIdx.x;
  const bool ar = a.arena != nullptr;
  const int64_t slot = a.slot0_w + wg * AW + wv;
  aca_worker<T, KIND, MF, 1>(a, wl, fr, shw[wv], nullptr, 0, slot, a.work,
                             a.b0 + a.nhuge + a.nbig, a.b1,
                             ar ? a.arena + slot * a.arena_elems : nullptr, a.arena_elems);
}

template <class T>
void launch_aca_t(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr,
                  int64_t b0, int64_t b1, T* pool, int64_t pool_elems, void* pool_top,
                  int* overflow, int* work, int* work_big, int* work_huge, int64_t nbig,
                  int64_t nhuge, const std::vector<HugeTier>* tiers, int64_t launch_rows,
                  int64_t team_rows, const void* Fs, double* ublk, const int64_t* uoff) {
  AcaArgs<T> a;
  a.G = p->G.as<int2>();
  a.nG = p->nG;
  a.order = lr->order.as<int32_t>();
  a.nodes = t->nodes.as<int4>();
  a.xs = t->xs.as<double>();
  a.kp = make_kparams(k, sizeof(T) == 8);
  a.eps2 = lr->eps * lr->eps;
  a.l_max = lr->l_max;
  a.rank = lr->rank.as<int32_t>();
  a.flag = lr->flag.as<int32_t>();
  a.piv = lr->piv.as<int32_t>();
  a.fptr = lr->fptr.as<int64_t>();
  a.pool = pool;
  a.pool_elems = pool_elems;
  a.pool_top = (unsigned long long*)pool_top;
  a.overflow = overflow;
  a.work = work;
  a.work_big = work_big;
  a.work_huge = work_huge;
  a.nbig = nbig;
  a.nhuge = nhuge;
  a.b0 = b0;
  a.b1 = b1;
  a.Fs = (const T*)Fs;
  a.ublk = ublk;
  a.uoff = uoff;
  a.frags = k->pbf.as<uint4>();
  a.frags32 = k->pf32.as<float4>();
  a.det_pivot = lr->prec != HH_FP64 || k->kind == KIND_RPY6;
  const int64_t nb = b1 - b0;
  if (nb <= 0) return;
  // persistent grid: as many workgroups as stay resident, each wave a worker
  // the kernel MLP samples on MFMA tiles: BF16 in the BF16 forms, FP32 in the
  // FP32 form; the FP64 form and the RPY kernels evaluate on the VALU
  const int mfk = k->kind != KIND_MLP ? MF_NONE
                  : is_bf16(lr->prec) ? MF_BF16
                  : lr->prec == HH_FP32 ? MF_F32 : MF_NONE;
  const void* fn = mfk == MF_BF16 ? (const void*)k_aca<float, KIND_MLP, MF_BF16>
                   : mfk == MF_F32 ? (const void*)k_aca<float, KIND_MLP, MF_F32>
                   : k->kind == KIND_MLP ? (const void*)k_aca<T, KIND_MLP, MF_NONE>
                                         : (const void*)k_aca<T, KIND_RPY, MF_NONE>;
  const void* fnt = mfk == MF_BF16 ? (const void*)k_aca_team<float, KIND_MLP, MF_BF16>
                    : mfk == MF_F32 ? (const void*)k_aca_team<float, KIND_MLP, MF_F32>
                    : k->kind == KIND_MLP ? (const void*)k_aca_team<T, KIND_MLP, MF_NONE>
                                          : (const void*)k_aca_team<T, KIND_RPY, MF_NONE>;
  int per_cu = 0, per_cu_t = 0;
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, AW_T, 0));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_t, fnt, AW_T, 0));
  HH_REQUIRE(per_cu > 0 && per_cu_t > 0, HH_ERR_HIP, "ACA kernel does not fit a compute unit");
  const int64_t nsmall = nb - nbig - nhuge;
  // persistent grids. When huge blocks hold a sizeable part of the work
  // (their long tail would leave the GPU idle behind the team kernel), the two
  // kernels run concurrently on disjoint compute units: the team kernel gets
  // units in proportion to its estimated share of the work (rows c + q, a team
  // row costing about 1.15 single-wave rows), the single waves the rest, so
  // that the two finish together. Otherwise each kernel in turn gets them all.
  int64_t huge_rows = 0;
  if (tiers)
    for (const HugeTier& h : *tiers) huge_rows += h.rows;
  const bool split = Fs != nullptr && nsmall > 0 && nbig + nhuge > 0 &&
                     (double)huge_rows >= 0.05 * (double)launch_rows;
  const int64_t ncu = ctx->n_cu;
  int64_t cu_t = ncu;
  if (split) {
    const double wt = 1.15 * (double)team_rows;
    const double ws = (double)std::max<int64_t>(launch_rows - team_rows, 0);
    cu_t = std::min<int64_t>(ncu - 1, std::max<int64_t>(1, llround((double)ncu * wt / (wt + ws))));
  }
  const int64_t grid_t = std::min<int64_t>((int64_t)per_cu_t * cu_t, std::max(nbig, nhuge));
  const int64_t cu_used = split ? (grid_t + per_cu_t - 1) / per_cu_t : 0;
  const int64_t grid_w =
      std::min<int64_t>((int64_t)per_cu * (ncu - cu_used), (nsmall + AW - 1) / AW);
  // concurrent kernels (team kernel on the side stream) give their workers
  // disjoint slots, teams [0, grid_t AW) and the single waves after them;
  // kernels in turn share the slots
  const int64_t workers = split ? (grid_t + grid_w) * AW : std::max(grid_t, grid_w) * AW;
  a.slot0_w = split ? grid_t * AW : 0;
  // per worker: Gram history A (l_max (l_max + 1) / 2 3x3 matrices), then the
  // cross-wave partials of a workgroup team [AW][64][9]
  const int64_t half = 9 * ((int64_t)lr->l_max * (lr->l_max + 1) / 2);
  const int64_t stride = half + (int64_t)AW * 64 * 9;
  if (lr->gram_workers < workers || lr->gram_stride != stride) {
    lr->gram.alloc(ctx->stream, std::max<int64_t>(1, workers * stride) * sizeof(double));
    lr->gram_workers = workers;
    lr->gram_stride = stride;
  }
  a.gram = lr->gram.as<double>();
  a.gram_stride = stride;
  a.gram_half = half;
  a.arena = nullptr;
  a.arena_elems = 0;
  a.huge = nullptr;
  a.ntier = 0;
  if (Fs) {
    // streamed mode: a factor arena per wave; huge blocks go to the first
    // workgroups of the team grid, in tiers of arenas sized per size class
    if (lr->arena_workers < workers) {
      lr->arena.alloc(ctx->stream, workers * lr->arena_elems * sizeof(T));
      lr->arena_workers = workers;
    }
    a.arena = lr->arena.as<T>();
    a.arena_elems = lr->arena_elems;
    if (nhuge > 0 && tiers && !tiers->empty()) {
      // workgroups per tier: twice the tier's share of the team's rows c + q
      // (its share of the samples), at least one, at most its blocks; scaled
      // down to the team grid and to half the budget
      const int nt = (int)tiers->size();
      HH_REQUIRE(nt <= ACA_MAX_TIERS, HH_ERR_CAPACITY, "too many size classes of huge blocks");
      std::vector<int64_t> nw(nt);
      const int64_t gt = std::max<int64_t>(grid_t, 1);
      for (int i = 0; i < nt; ++i) {
        const HugeTier& h = (*tiers)[i];
        const double share = (double)h.rows / (double)std::max<int64_t>(team_rows, 1);
        nw[i] = std::max<int64_t>(1, std::min<int64_t>(h.nblk, (int64_t)ceil(2.0 * gt * share)));
      }
      const double cap = 0.5 * (double)ctx->budget_bytes / sizeof(T);
      for (int pass = 0; pass < 64; ++pass) {
        int64_t wgs = 0;
        double mem = 0;
        for (int i = 0; i < nt; ++i) {
          wgs += nw[i];
          mem += (double)nw[i] * (double)(*tiers)[i].need;
        }
        const double f = std::min((double)gt / (double)wgs, cap / mem);
        if (f >= 1.0) break;
        bool shrunk = false;
        for (int i = 0; i < nt; ++i) {
          const int64_t v = std::max<int64_t>(1, (int64_t)floor((double)nw[i] * f));
          shrunk |= v < nw[i];
          nw[i] = v;
        }
        if (!shrunk) break;   // one workgroup per tier is the floor
      }
      int64_t off = 0, b = 0, wgs = 0;
      for (int i = 0; i < nt; ++i) {
        const HugeTier& h = (*tiers)[i];
        a.tier_wg[i] = (int)wgs;
        a.tier_b[i] = b;
        a.tier_cap[i] = h.need;
        a.tier_off[i] = off;
        wgs += nw[i];
        b += h.nblk;
        off += nw[i] * h.need;
      }
      a.tier_wg[nt] = (int)wgs;
      a.tier_b[nt] = b;
      HH_REQUIRE(wgs <= grid_t, HH_ERR_CAPACITY, "more huge tiers than team workgroups");
      HH_REQUIRE(b == nhuge, HH_ERR_CAPACITY, "huge tiers do not cover the huge blocks");
      if (lr->huge_elems < off) {
        lr->huge.alloc(ctx->stream, off * sizeof(T));
        lr->huge_elems = off;
      }
      a.huge = lr->huge.as<T>();
      a.ntier = nt;
    }
  }
  // concurrent kernels: the team kernel on the side stream, forked after the
  // work queued so far and joined before anything queued later (capturable)
  const bool both = split && grid_t > 0 && grid_w > 0;
  hipStream_t ts = both ? ctx->side : ctx->stream;
  if (both) {
    HIP_OK(hipEventRecord(ctx->fork, ctx->stream));
    HIP_OK(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
  }
#define LAUNCH(KIND_, MF_)                                                                    \
  do {                                                                                        \
    if (grid_t > 0)                                                                           \
      hipLaunchKernelGGL((k_aca_team<T, KIND_, MF_>), dim3((unsigned)grid_t), dim3(AW_T), 0,   \
                         ts, a);                                                              \
    if (grid_w > 0)                                                                           \
      hipLaunchKernelGGL((k_aca<T, KIND_, MF_>), dim3((unsigned)grid_w), dim3(AW_T), 0,        \
                         ctx->stream, a);                                                     \
  } while (0)
  if (mfk == MF_BF16) {
    if constexpr (sizeof(T) == 4) LAUNCH(KIND_MLP, MF_BF16);
  } else if (mfk == MF_F32) {
    if constexpr (sizeof(T) == 4) LAUNCH(KIND_MLP, MF_F32);
  } else if (k->kind == KIND_MLP) {
    LAUNCH(KIND_MLP, MF_NONE);
  } else {
    LAUNCH(KIND_RPY, MF_NONE);
  }
#undef LAUNCH
  HIP_OK(hipGetLastError());
  if (both) {
    HIP_OK(hipEventRecord(ctx->join, ctx->side));
    HIP_OK(hipStreamWaitEvent(ctx->stream, ctx->join, 0));
  }
}

__global__ void k_rank_stats(const int32_t* __restrict__ rank, const int32_t* __restrict__ flag,
                             const int2* __restrict__ G, const int4* __restrict__ nodes,
                             int64_t nG, int64_t* __restrict__ rk,
                             unsigned long long* __restrict__ sums) {
  int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long r = 0, fb = 0, smp = 0;
  if (b < nG) {
    int2 g = G[b];
    int cq = (nodes[g.x].y - nodes[g.x].x) + (nodes[g.y].y - nodes[g.y].x);
    int f = flag[b];
    int rr = rank[b];
    if (rk) rk[b] = f ? 0 : rr;
    r = f ? 0 : rr;
    fb = f;
    smp = (unsigned long long)rr * cq;
  }
  for (int o = 32; o > 0; o >>= 1) {
    r += __shfl_xor(r, o, 64);
    fb += __shfl_xor(fb, o, 64);
    smp += __shfl_xor(smp, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (r) atomicAdd(&sums[0], r);
    if (fb) atomicAdd(&sums[1], fb);
    if (smp) atomicAdd(&sums[2], smp);
  }
}

}  // namespace

// Rank, fallback and sample counts of a finished ACA (syncs). With toff != 0
// also fills the t offsets (exclusive prefix of the non-fallback ranks).
void lowrank_stats(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, bool toff) {
  hipStream_t st = ctx->stream;
  int64_t nG = p->nG;
  unsigned long long* sums = (unsigned long long*)ctx->scratch_flag.p;
  HIP_OK(hipMemsetAsync(sums, 0, 4 * sizeof(unsigned long long), st));
  if (toff) HIP_OK(hipMemsetAsync(lr->toff.as<int64_t>() + nG, 0, sizeof(int64_t), st));
  if (nG > 0) {
    hipLaunchKernelGGL(k_rank_stats, dim3((unsigned)((nG + 255) / 256)), dim3(256), 0, st,
                       lr->rank.as<int32_t>(), lr->flag.as<int32_t>(), p->G.as<int2>(),
                       t->nodes.as<int4>(), nG, toff ? lr->toff.as<int64_t>() : nullptr, sums);
    HIP_OK(hipGetLastError());
  }
  if (toff) scan_exclusive_i64(ctx, lr->toff.as<int64_t>(), lr->toff.as<int64_t>(), nG + 1);
  HIP_OK(hipMemcpyAsync(ctx->pinned, sums, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  ctx_sync(ctx);
  lr->rank_sum = ctx->pinned[0];
  lr->n_fallback = ctx->pinned[1];
  lr->samples = ctx->pinned[2];
  lr->stats_dirty = false;
}

// Sizes of every admissible block (host), used to plan storage.
void block_sizes(hh_ctx ctx, hh_tree t, hh_part p, std::vector<int32_t>& cs,
                 std::vector<int32_t>& qs) {
  int64_t nG = p->nG;
  std::vector<int4> nodes(t->n_nodes);
  std::vector<int2> G(nG);
  read_bytes(ctx, nodes.data(), t->nodes.p, t->n_nodes * sizeof(int4));
  read_bytes(ctx, G.data(), p->G.p, nG * sizeof(int2));
  cs.resize(nG);
  qs.resize(nG);
  for (int64_t b = 0; b < nG; ++b) {
    cs[b] = nodes[G[b].x].y - nodes[G[b].x].x;
    qs[b] = nodes[G[b].y].y - nodes[G[b].y].x;
  }
}

static inline int size_cls(int32_t c, int32_t q) {
  return 31 - __builtin_clz((unsigned)(c + q));
}

// Appends the blocks `blk` to the work order, largest first (by the power of
// two of c + q, stable).
static void append_desc(const std::vector<int32_t>& cs, const std::vector<int32_t>& qs,
                        const std::vector<int32_t>& blk, std::vector<int32_t>& ord) {
  int64_t cnt[33] = {0};
  for (int32_t b : blk) cnt[size_cls(cs[b], qs[b])]++;
  int64_t pos[33], acc = (int64_t)ord.size();
  for (int c = 32; c >= 0; --c) { pos[c] = acc; acc += cnt[c]; }
  ord.resize(acc);
  for (int32_t b : blk) ord[pos[size_cls(cs[b], qs[b])]++] = b;
}

static void upload_i32(hh_ctx ctx, DevBuf& d, const std::vector<int32_t>& v) {
  d.alloc(ctx->stream, std::max<size_t>(v.size(), 1) * sizeof(int32_t));
  if (!v.empty())
    HIP_OK(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          ctx->stream));
}

// Plans the ACA. Each launch works on a range of the work order: the large
// blocks (c + q >= 2^team_cls, whole workgroups, largest first), then the
// small ones (single waves, largest first).
// Stored mode: one launch over all blocks; the factors stay in the pool.
// Streamed mode (the factors would not fit half the context budget; Sec.
// 3.3.2: a fixed buffer is filled by a group of blocks, applied, then
// reused): a block's factors only live while its worker approximates it, so
// every wave has a fixed factor arena (sized for the worst case of the small
// blocks), a workgroup team uses the arenas of its waves, and the huge blocks
// whose worst case exceeds that go first to a few workgroups with large
// arenas. Launches are split only by the size of their output rows.
void plan_aca(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, int force_streamed) {
  hipStream_t st = ctx->stream;
  int64_t nG = p->nG;
  lr->rank.alloc(st, std::max<int64_t>(1, nG) * sizeof(int32_t));
  lr->flag.alloc(st, std::max<int64_t>(1, nG) * sizeof(int32_t));
  lr->piv.alloc(st, std::max<int64_t>(1, nG) * 2 * LMAX_CAP * sizeof(int32_t));
  lr->fptr.alloc(st, std::max<int64_t>(1, nG) * LMAX_CAP * sizeof(int64_t));
  lr->toff.alloc(st, (std::max<int64_t>(1, nG) + 1) * sizeof(int64_t));
  std::vector<int32_t> cs, qs;
  block_sizes(ctx, t, p, cs, qs);
  const size_t es = lr->prec == HH_FP64 ? 8 : 4;
  int64_t est = 0;
  std::vector<int32_t> big, small;
  int64_t arena = 0;
  for (int64_t b = 0; b < nG; ++b) {
    const int64_t cq = (int64_t)cs[b] + qs[b];
    const int64_t kc = std::min<int64_t>(std::min(cs[b], qs[b]), lr->l_max);
    est += 9 * (cq + 1) * std::min<int64_t>(kc, 20);
    if (size_cls(cs[b], qs[b]) >= ctx->team_cls) {
      big.push_back((int32_t)b);
    } else {
      small.push_back((int32_t)b);
      arena = std::max(arena, 9 * cq * kc);
    }
  }
  lr->est_elems = est;
  lr->streamed = force_streamed || (double)est * es > 0.5 * (double)ctx->budget_bytes;
  std::vector<int32_t> ord;
  ord.reserve(std::max<int64_t>(nG, 1));
  lr->bounds.assign(1, 0);
  lr->nbig.clear();
  lr->tiers.clear();
  lr->launch_rows.clear();
  lr->team_rows.clear();
  if (!lr->streamed) {
    int64_t rt = 0, ra = 0;
    for (int32_t b : big) rt += (int64_t)cs[b] + qs[b];
    for (int64_t b = 0; b < nG; ++b) ra += (int64_t)cs[b] + qs[b];
    lr->launch_rows.push_back(ra);
    lr->team_rows.push_back(rt);
    append_desc(cs, qs, big, ord);
    append_desc(cs, qs, small, ord);
    lr->bounds.push_back(nG);
    lr->nbig.push_back((int64_t)big.size());
    lr->nhuge.assign(1, 0);
    lr->arena_elems = 0;
    upload_i32(ctx, lr->order, ord);
    ctx_sync(ctx);
    return;
  }
  // streamed: small blocks in a per-wave arena, large ones in the arenas of a
  // workgroup's waves, huge ones (worst case above that) in a few large
  // arenas; launches are split only by the size of their output rows
  const int64_t wave_arena = std::max<int64_t>(arena, 1024);
  const int64_t team_arena = (int64_t)AW * wave_arena;
  std::vector<char> kind(std::max<int64_t>(nG, 1), 0);   // 0 small, 1 large, 2 huge
  for (int32_t b : big) {
    const int64_t cq = (int64_t)cs[b] + qs[b];
    const int64_t kc = std::min<int64_t>(std::min(cs[b], qs[b]), lr->l_max);
    const int64_t w = 9 * cq * kc;
    kind[b] = w > team_arena ? 2 : 1;
  }
  const int64_t rows_cap = std::max<int64_t>(1, (int64_t)(0.2 * (double)ctx->budget_bytes / 24.0));
  std::vector<int32_t> lid(std::max<int64_t>(nG, 1)), pos(std::max<int64_t>(nG, 1));
  std::vector<int64_t> uoff(1, 0);
  int64_t ub_max = 0;
  lr->nhuge.clear();
  std::vector<int32_t> hb, tb, wb;
  int64_t rows = 0;
  auto close = [&]() {
    const size_t r0 = ord.size();
    const int32_t r = (int32_t)lr->nbig.size();
    append_desc(cs, qs, hb, ord);
    lr->nhuge.push_back((int64_t)hb.size());
    // one tier per size class of the huge blocks (contiguous in the order)
    std::vector<HugeTier> tiers;
    int prev = -1;
    for (size_t i = r0; i < ord.size(); ++i) {
      const int32_t b = ord[i];
      const int cls = size_cls(cs[b], qs[b]);
      const int64_t cq = (int64_t)cs[b] + qs[b];
      const int64_t kc = std::min<int64_t>(std::min(cs[b], qs[b]), lr->l_max);
      if (cls != prev) tiers.push_back(HugeTier{0, 0, 0});
      prev = cls;
      HugeTier& h = tiers.back();
      h.nblk += 1;
      h.need = std::max(h.need, 9 * cq * kc);
      h.rows += cq;
    }
    lr->tiers.push_back(tiers);
    append_desc(cs, qs, tb, ord);
    lr->nbig.push_back((int64_t)tb.size());
    append_desc(cs, qs, wb, ord);
    lr->bounds.push_back((int64_t)ord.size());
    int64_t lrows = 0, trows = 0;
    const size_t r2 = r0 + hb.size() + tb.size();   // huge and large blocks come first
    for (size_t i = r0; i < ord.size(); ++i) {
      lrows += (int64_t)cs[ord[i]] + qs[ord[i]];
      if (i < r2) trows += (int64_t)cs[ord[i]] + qs[ord[i]];
    }
    lr->launch_rows.push_back(lrows);
    lr->team_rows.push_back(trows);
    for (size_t i = r0; i < ord.size(); ++i) {
      lid[ord[i]] = r;
      pos[ord[i]] = (int32_t)i;
      uoff.push_back(uoff.back() + cs[ord[i]]);
    }
    ub_max = std::max(ub_max, uoff.back() - uoff[r0]);
    hb.clear();
    tb.clear();
    wb.clear();
    rows = 0;
  };
  for (int64_t b = 0; b < nG; ++b) {
    if (rows > 0 && rows + cs[b] > rows_cap) close();
    (kind[b] == 2 ? hb : kind[b] == 1 ? tb : wb).push_back((int32_t)b);
    rows += cs[b];
  }
  if (rows > 0 || lr->nbig.empty()) close();
  lr->arena_elems = wave_arena;
  lr->pool_elems = 1024;   // the shared pool is not used in streamed mode
  lr->ub_elems = std::max<int64_t>(ub_max, 1);
  upload_i32(ctx, lr->order, ord);
  upload_i32(ctx, lr->lid, lid);
  upload_i32(ctx, lr->pos, pos);
  lr->uoff.alloc(st, uoff.size() * sizeof(int64_t));
  HIP_OK(hipMemcpyAsync(lr->uoff.p, uoff.data(), uoff.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, st));
  ctx_sync(ctx);
}

// Stored mode: runs the ACA over all admissible blocks once; grows the pool
// and retries when it overflows. Fills lr->{rank, flag, piv, fptr, pool, toff}.
void run_aca_stored(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr) {
  hipStream_t st = ctx->stream;
  int64_t nG = p->nG;
  size_t es = lr->prec == HH_FP64 ? 8 : 4;
  int64_t want = lr->est_elems;
  int* flags = (int*)ctx->scratch_flag.p;  // [0] overflow, [1] work counter
  int64_t* top = (int64_t*)ctx->scratch_flag.p + 4;
  for (int attempt = 0; attempt < 6; ++attempt) {
    lr->pool_elems = std::max<int64_t>(want, 1024);
    lr->pool.alloc(st, lr->pool_elems * es);
    HIP_OK(hipMemsetAsync(ctx->scratch_flag.p, 0, 8 * sizeof(int64_t), st));
    if (nG > 0) {
      PhaseTimer timer(ctx, HH_PHASE_ACA);
      if (lr->prec == HH_FP64)
        launch_aca_t<double>(ctx, t, p, k, lr, 0, nG, lr->pool.as<double>(), lr->pool_elems, top,
                             flags, flags + 1, flags + 2, flags + 3, lr->nbig[0], 0, nullptr,
                             lr->launch_rows[0], lr->team_rows[0], nullptr, nullptr, nullptr);
      else
        launch_aca_t<float>(ctx, t, p, k, lr, 0, nG, lr->pool.as<float>(), lr->pool_elems, top,
                            flags, flags + 1, flags + 2, flags + 3, lr->nbig[0], 0, nullptr,
                            lr->launch_rows[0], lr->team_rows[0], nullptr, nullptr, nullptr);
    }
    HIP_OK(hipMemcpyAsync(ctx->pinned, ctx->scratch_flag.p, 8 * sizeof(int64_t),
                          hipMemcpyDeviceToHost, st));
    ctx_sync(ctx);
    int ovf = ((int*)ctx->pinned)[0];
    int64_t used = ctx->pinned[4];
    if (!ovf) {
      lr->used_elems = used;
      break;
    }
    HH_REQUIRE(attempt < 5, HH_ERR_CAPACITY, "ACA factor pool overflow");
    want = std::max<int64_t>(2 * want, used + used / 4);
  }
  lowrank_stats(ctx, t, p, lr, true);
  lr->tbuf.alloc(st, std::max<int64_t>(1, lr->rank_sum) * 3 * sizeof(double));
}

// Streamed mode, launch i: ACA with the apply fused in; per-block rows go to
// ublk (offsets uoff[pos] - uoff[b0]). counters: ACA_COUNTERS int64 per
// launch, zeroed.
void run_aca_batch(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr, size_t i,
                   const void* Fs, int64_t* counters) {
  static_assert(2 + ACA_MAX_TIERS <= 2 * (ACA_COUNTERS - 1), "counter words");
  int64_t b0 = lr->bounds[i], b1 = lr->bounds[i + 1];
  int* work = (int*)(counters + ACA_COUNTERS * i);   // single waves, workgroups, huge tiers
  int64_t* top = counters + ACA_COUNTERS * i + ACA_COUNTERS - 1;
  int* ovf = (int*)ctx->scratch_flag.p;
  if (lr->prec == HH_FP64)
    launch_aca_t<double>(ctx, t, p, k, lr, b0, b1, lr->pool.as<double>(), lr->pool_elems, top,
                         ovf, work, work + 1, work + 2, lr->nbig[i], lr->nhuge[i], &lr->tiers[i],
                         lr->launch_rows[i], lr->team_rows[i], Fs, lr->ublk.as<double>(),
                         lr->uoff.as<int64_t>());
  else
    launch_aca_t<float>(ctx, t, p, k, lr, b0, b1, lr->pool.as<float>(), lr->pool_elems, top, ovf,
                        work, work + 1, work + 2, lr->nbig[i], lr->nhuge[i], &lr->tiers[i],
                        lr->launch_rows[i], lr->team_rows[i], Fs, lr->ublk.as<double>(),
                        lr->uoff.as<int64_t>());
}
