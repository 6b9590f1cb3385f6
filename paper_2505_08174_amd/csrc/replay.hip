// Cross approximation with given pivots: the recursion of Algorithm 2 (Eqs.
// (8)-(9)) with the pivot search and the stopping test replaced by stored
// pivots (i_k, j_k) and ranks. For every admissible block that did not fall
// back to dense evaluation, and k = 0 .. rank - 1:
//   a(i)   = K(x_i - y_{j_k}) - sum_{m<k} c_m(i) q_m(j_k)
//   P_k    = a(i_k),  c_k(i) = a(i) P_k^-1
//   q_k(j) = K(x_{i_k} - y_j) - sum_{m<k} c_m(i_k) q_m(j)
// With the pivots frozen the factors are a smooth function of the positions
// and the kernel parameters, which is what the backward pass differentiates
// and what a finite-difference check of it perturbs. The arithmetic and the
// order of every sum follow the single-wave ACA worker, so replaying a build's
// own pivots at the same positions reproduces its factors (the FP32 form's
// kernel-MLP samples come from the same FP32 MFMA tile as the build's).
// One workgroup per block; the factors go to a pool laid out as in the
// stored ACA (c_k, q_k, P_k per step).
#include <algorithm>

#include "api_guard.h"
#include "devmath.h"
#include "internal.h"
#include "mlp_mfma.h"

void lowrank_stats(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, bool toff);
void block_sizes(hh_ctx ctx, hh_tree t, hh_part p, std::vector<int32_t>& cs,
                 std::vector<int32_t>& qs);

namespace {

constexpr int TB = 256;

// K -= A B (3x3, row-major), the same expression as the ACA worker's
template <class T>
__device__ __forceinline__ void sub_mm3(T K[9], const T A[9], const T B[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      K[3 * r + cc] -= A[3 * r] * B[cc] + A[3 * r + 1] * B[3 + cc] + A[3 * r + 2] * B[6 + cc];
}

// The residual of sample K (entry of row i against the pivot column, or of the
// pivot row against column j) written to dst.
template <class T>
__device__ __forceinline__ void residual_col(T rs[9], const T* __restrict__ pool,
                                             const int64_t* __restrict__ fp, int k, int64_t i,
                                             const T* sh, T* __restrict__ dst) {
  for (int m = 0; m < k; ++m) {
    T cv[9];
    const T* cm = pool + fp[m] + 9 * i;
#pragma unroll
    for (int e = 0; e < 9; ++e) cv[e] = cm[e];
    sub_mm3<T>(rs, cv, sh + 9 * m);
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) dst[e] = rs[e];
}

template <class T>
__device__ __forceinline__ void residual_row(T rs[9], const T* __restrict__ pool,
                                             const int64_t* __restrict__ fp, int k, int64_t c,
                                             int64_t j, const T* sh, T* __restrict__ dst) {
  for (int m = 0; m < k; ++m) {
    T qv[9];
    const T* qm = pool + fp[m] + 9 * c + 9 * j;
#pragma unroll
    for (int e = 0; e < 9; ++e) qv[e] = qm[e];
    sub_mm3<T>(rs, sh + 9 * m, qv);
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) dst[e] = rs[e];
}

// F32T: kernel-MLP samples from the FP32 MFMA tile (the FP32 form's ACA
// samples), each wave taking 32 rows or columns per tile.
template <class T, int KIND, bool F32T>
__global__ __launch_bounds__(TB) void k_aca_replay(const int2* __restrict__ G, int64_t nG,
                                                   const int4* __restrict__ nodes,
                                                   const double* __restrict__ xs, KParams kp,
                                                   const float4* __restrict__ frags32,
                                                   const int32_t* __restrict__ rank,
                                                   int32_t* __restrict__ flag,
                                                   const int32_t* __restrict__ piv,
                                                   const int64_t* __restrict__ fptr,
                                                   T* __restrict__ pool, double sing) {
  __shared__ T wl[(KIND == KIND_MLP && !F32T) ? MLP_NP : 1];
  __shared__ float fr[F32T ? F32_FRAGS * 64 : 1];
  __shared__ T sh[LMAX_CAP * 9];   // q_m(j_k) in the column step, c_m(i_k) in the row step
  if (F32T) {
    stage_frags_f32(fr, frags32, TB);
  } else if (KIND == KIND_MLP) {
    const T* w = (const T*)kp.w;
    for (int i = threadIdx.x; i < MLP_NP; i += TB) wl[i] = w[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < nG; b += gridDim.x) {
    const int l = rank[b];
    if (flag[b] || l == 0) continue;
    const int2 g = G[b];
    const int4 nt = nodes[g.x], ns = nodes[g.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x;
    const double* xt = xs + 3 * (int64_t)nt.x;
    const double* xsr = xs + 3 * (int64_t)ns.x;
    const int32_t* pi = piv + b * 2 * LMAX_CAP;
    const int32_t* pj = pi + LMAX_CAP;
    const int64_t* fp = fptr + b * LMAX_CAP;
    for (int k = 0; k < l; ++k) {
      const int ik = pi[k], jk = pj[k];
      T* Ck = pool + fp[k];
      T* Qk = Ck + 9 * (int64_t)c;
      for (int t = threadIdx.x; t < 9 * k; t += TB) {
        const int m = t / 9, e = t - 9 * m;
        sh[t] = pool[fp[m] + 9 * (int64_t)c + 9 * (int64_t)jk + e];
      }
      __syncthreads();
      const double y0 = xsr[3 * jk], y1 = xsr[3 * jk + 1], y2 = xsr[3 * jk + 2];
      if constexpr (F32T) {
        for (int t0 = 32 * wv; t0 < c; t0 += 32 * (TB / 64)) {   // uniform per wave
          const int i = t0 + (lane & 31);
          const int ii = i < c ? i : t0;
          float K[9];
          entry_f32tile(fr, kp.input_mode, xt[3 * ii] - y0, xt[3 * ii + 1] - y1,
                        xt[3 * ii + 2] - y2, K);
          if (i < c && lane < 32) {
            T rs[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) rs[e] = (T)K[e];
            residual_col<T>(rs, pool, fp, k, i, sh, Ck + 9 * (int64_t)i);
          }
        }
      } else {
        for (int i = threadIdx.x; i < c; i += TB) {
          T rs[9];
          kernel_entry<T>(kp, wl, (T)(xt[3 * i] - y0), (T)(xt[3 * i + 1] - y1),
                          (T)(xt[3 * i + 2] - y2), rs, i & 1, jk & 1);
          residual_col<T>(rs, pool, fp, k, i, sh, Ck + 9 * (int64_t)i);
        }
      }
      __syncthreads();
      // pivot entry and its inverse in FP64, as in the ACA worker
      double P[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) P[e] = (double)Ck[9 * (int64_t)ik + e];
      if (threadIdx.x == 0) {
        T* ps = Ck + 9 * (int64_t)(c + q);
#pragma unroll
        for (int e = 0; e < 9; ++e) ps[e] = Ck[9 * (int64_t)ik + e];
      }
      __syncthreads();   // every thread holds P before row i_k is overwritten
      const double det = P[0] * (P[4] * P[8] - P[5] * P[7]) - P[1] * (P[3] * P[8] - P[5] * P[6]) +
                         P[2] * (P[3] * P[7] - P[4] * P[6]);
      double fro2 = 0;
#pragma unroll
      for (int e = 0; e < 9; ++e) fro2 += P[e] * P[e];
      if (!(fabs(det) > sing * fro2 * sqrt(fro2))) {
        // a pivot that has become singular at these positions: the block is
        // evaluated densely (uniform decision: every thread has the same P)
        if (threadIdx.x == 0) flag[b] = 1;
        break;
      }
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
      // c_k = a P^-1 in FP64, rounded to T once, as in the ACA worker
      for (int i = threadIdx.x; i < c; i += TB) {
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
      __syncthreads();
      for (int t = threadIdx.x; t < 9 * k; t += TB) {
        const int m = t / 9, e = t - 9 * m;
        sh[t] = pool[fp[m] + 9 * (int64_t)ik + e];
      }
      __syncthreads();
      const double x0 = xt[3 * ik], x1 = xt[3 * ik + 1], x2 = xt[3 * ik + 2];
      if constexpr (F32T) {
        for (int t0 = 32 * wv; t0 < q; t0 += 32 * (TB / 64)) {   // uniform per wave
          const int j = t0 + (lane & 31);
          const int jj = j < q ? j : t0;
          float K[9];
          entry_f32tile(fr, kp.input_mode, x0 - xsr[3 * jj], x1 - xsr[3 * jj + 1],
                        x2 - xsr[3 * jj + 2], K);
          if (j < q && lane < 32) {
            T rs[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) rs[e] = (T)K[e];
            residual_row<T>(rs, pool, fp, k, c, j, sh, Qk + 9 * (int64_t)j);
          }
        }
      } else {
        for (int j = threadIdx.x; j < q; j += TB) {
          T rs[9];
          kernel_entry<T>(kp, wl, (T)(x0 - xsr[3 * j]), (T)(x1 - xsr[3 * j + 1]),
                          (T)(x2 - xsr[3 * j + 2]), rs, ik & 1, j & 1);
          residual_row<T>(rs, pool, fp, k, c, j, sh, Qk + 9 * (int64_t)j);
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

// A stored low-rank handle whose factors are the ACA recursion replayed with
// the given pivots (host arrays in the layout of hh_lowrank_export).
hh_lowrank_s* build_lowrank_pivots(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, int prec,
                                   const int32_t* rank, const int32_t* fallback,
                                   const int32_t* piv_i, const int32_t* piv_j) {
  HH_REQUIRE(prec == HH_FP64 || prec == HH_FP32, HH_ERR_INVALID_ARG,
             "factors with given pivots are built in HH_FP64 or HH_FP32");
  const int64_t nG = p->nG;
  HH_REQUIRE(nG == 0 || (rank && fallback && piv_i && piv_j), HH_ERR_INVALID_ARG,
             "NULL pivot array");
  std::vector<int32_t> cs, qs;
  block_sizes(ctx, t, p, cs, qs);
  std::vector<int64_t> fptr(std::max<int64_t>(nG, 1) * LMAX_CAP, 0);
  std::vector<int32_t> piv(std::max<int64_t>(nG, 1) * 2 * LMAX_CAP, -1);
  std::vector<int32_t> rk(std::max<int64_t>(nG, 1), 0), fl(std::max<int64_t>(nG, 1), 0);
  int64_t off = 0;
  int32_t lmax = 1;
  for (int64_t b = 0; b < nG; ++b) {
    const int32_t c = cs[b], q = qs[b], r = rank[b], f = fallback[b];
    HH_REQUIRE(f == 0 || f == 1, HH_ERR_INVALID_ARG, "fallback flags must be 0 or 1");
    fl[b] = f;
    if (f) continue;
    HH_REQUIRE(r >= 0 && r <= std::min(std::min(c, q), (int32_t)LMAX_CAP), HH_ERR_INVALID_ARG,
               "rank out of range for block " + std::to_string(b));
    for (int m = 0; m < r; ++m) {
      const int32_t i = piv_i[b * LMAX_CAP + m], j = piv_j[b * LMAX_CAP + m];
      HH_REQUIRE(i >= 0 && i < c && j >= 0 && j < q, HH_ERR_INVALID_ARG,
                 "pivot out of range in block " + std::to_string(b));
      piv[b * 2 * LMAX_CAP + m] = i;
      piv[b * 2 * LMAX_CAP + LMAX_CAP + m] = j;
      fptr[b * LMAX_CAP + m] = off;
      off += 9 * ((int64_t)c + q + 1);
    }
    rk[b] = r;
    lmax = std::max(lmax, r);
  }
  hipStream_t st = ctx->stream;
  hh_lowrank_s* lr = new hh_lowrank_s();
  try {
    lr->ctx = ctx;
    lr->part = p;
    lr->prec = prec;
    lr->nG = nG;
    lr->l_max = lmax;
    lr->eps = 0.0;
    lr->kern = k;
    lr->streamed = false;
    const size_t es = elem_size(prec);
    const int64_t nb = std::max<int64_t>(nG, 1);
    lr->rank.alloc(st, nb * sizeof(int32_t));
    lr->flag.alloc(st, nb * sizeof(int32_t));
    lr->piv.alloc(st, nb * 2 * LMAX_CAP * sizeof(int32_t));
    lr->fptr.alloc(st, nb * LMAX_CAP * sizeof(int64_t));
    lr->toff.alloc(st, (nb + 1) * sizeof(int64_t));
    lr->pool_elems = std::max<int64_t>(off, 1024);
    lr->pool.alloc(st, lr->pool_elems * es);
    lr->used_elems = off;
    HIP_OK(hipMemcpyAsync(lr->rank.p, rk.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(lr->flag.p, fl.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(lr->piv.p, piv.data(), piv.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(lr->fptr.p, fptr.data(), fptr.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, st));
    if (nG > 0) {
      PhaseTimer timer(ctx, HH_PHASE_ACA);
      const KParams kp = make_kparams(k, prec == HH_FP64);
      // the singularity guard of the pivot rule and working type the build used
      const double sing = prec != HH_FP64 ? 1e-6 : k->kind == KIND_RPY6 ? 1e-8 : 1e-14;
      const unsigned grid = (unsigned)std::min<int64_t>(nG, 4096);
#define REPLAY(T_, KIND_, F32T_)                                                             \
  hipLaunchKernelGGL((k_aca_replay<T_, KIND_, F32T_>), dim3(grid), dim3(TB), 0, st,           \
                     p->G.as<int2>(), nG, t->nodes.as<int4>(), t->xs.as<double>(), kp,         \
                     k->pf32.as<float4>(), lr->rank.as<int32_t>(), lr->flag.as<int32_t>(),    \
                     lr->piv.as<int32_t>(), lr->fptr.as<int64_t>(), lr->pool.as<T_>(), sing)
      if (prec == HH_FP64) {
        if (k->kind == KIND_MLP) REPLAY(double, KIND_MLP, false);
        else REPLAY(double, KIND_RPY, false);
      } else {
        if (k->kind == KIND_MLP) REPLAY(float, KIND_MLP, true);
        else REPLAY(float, KIND_RPY, false);
      }
#undef REPLAY
      HIP_OK(hipGetLastError());
    }
    lowrank_stats(ctx, t, p, lr, true);
    lr->tbuf.alloc(st, std::max<int64_t>(1, lr->rank_sum) * 3 * sizeof(double));
    // the plan of a stored build: one range over all blocks
    lr->bounds.assign({0, nG});
  } catch (...) {
    delete lr;
    throw;
  }
  return lr;
}

extern "C" hh_status hh_aca_build_pivots(hh_ctx ctx, hh_tree tree, hh_part part, hh_kernel kern,
                                         hh_precision prec, const int32_t* rank,
                                         const int32_t* fallback, const int32_t* piv_i,
                                         const int32_t* piv_j, hh_lowrank* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && tree && part && kern, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(part->tree == tree, HH_ERR_INVALID_ARG, "partition was built on another tree");
  check_kernel_tree(tree, kern);
  HH_REQUIRE(kern->kind != KIND_RPY6 || prec == HH_FP64 || prec == HH_FP32, HH_ERR_INVALID_ARG,
             "the 6N kernel runs in HH_FP64 and HH_FP32");
  *out = build_lowrank_pivots(ctx, tree, part, kern, prec, rank, fallback, piv_i, piv_j);
  HH_API_END(ctx)
}
