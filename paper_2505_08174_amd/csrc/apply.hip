// Far-field low-rank apply, self term, combine and unpermute; the matvec and
// ACA entry points.
//
// The low-rank product of an admissible block is applied right to left as in
// Sec. 3: t_k = sum_j q_k(j) F_j for every term (one workgroup per block),
// then u_i += sum_k c_k(i) t_k. The second half runs per target particle: a
// thread walks from the particle's leaf up to the root and adds the terms of
// every admissible block whose target cluster contains it, in a fixed order,
// so the sum is deterministic without atomics. The same walk adds blocks that
// fell back to dense evaluation, the near-field partial sum and the self term
// alpha_1 F_i (Eq. (2)), and writes U in the caller's particle order.
#include "api_guard.h"
#include "devmath.h"
#include "internal.h"

void plan_aca(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, int force_streamed);
void run_aca_stored(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr);
void run_aca_batch(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr, size_t i,
                   const void* Fs, int64_t* counters);
void lowrank_stats(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, bool toff);
hh_lowrank_s* build_lowrank_pivots(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, int prec,
                                   const int32_t* rank, const int32_t* fallback,
                                   const int32_t* piv_i, const int32_t* piv_j);

namespace {

constexpr int T256 = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + T256 - 1) / T256); }

template <class TI, class TO>
__global__ __launch_bounds__(T256) void k_gather_rows(const TI* __restrict__ F,
                                                      const int32_t* __restrict__ perm, int64_t n,
                                                      TO* __restrict__ Fs) {
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n) return;
  int64_t o = perm[s];
  Fs[3 * s] = (TO)F[3 * o];
  Fs[3 * s + 1] = (TO)F[3 * o + 1];
  Fs[3 * s + 2] = (TO)F[3 * o + 2];
}

// t[toff[b] + k] = sum_j q_k(j) F_sigma(j) for every non-fallback block.
template <class T>
__global__ __launch_bounds__(T256) void k_far_t(const int2* __restrict__ G, int64_t nG,
                                                const int4* __restrict__ nodes,
                                                const int32_t* __restrict__ rank,
                                                const int32_t* __restrict__ flag,
                                                const int64_t* __restrict__ fptr,
                                                const int64_t* __restrict__ toff,
                                                const T* __restrict__ pool,
                                                const T* __restrict__ Fs,
                                                double* __restrict__ tbuf) {
  __shared__ double red[T256 / 64][3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < nG; b += gridDim.x) {
    if (flag[b]) continue;
    const int2 g = G[b];
    const int4 nt = nodes[g.x], ns = nodes[g.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x;
    const int l = rank[b];
    for (int k = 0; k < l; ++k) {
      const T* Qk = pool + fptr[b * LMAX_CAP + k] + 9 * (int64_t)c;
      double s0 = 0, s1 = 0, s2 = 0;
      for (int j = threadIdx.x; j < q; j += T256) {
        const T* e = Qk + 9 * (int64_t)j;
        double f0 = Fs[3 * (int64_t)(ns.x + j)], f1 = Fs[3 * (int64_t)(ns.x + j) + 1],
               f2 = Fs[3 * (int64_t)(ns.x + j) + 2];
        s0 += (double)e[0] * f0 + (double)e[1] * f1 + (double)e[2] * f2;
        s1 += (double)e[3] * f0 + (double)e[4] * f1 + (double)e[5] * f2;
        s2 += (double)e[6] * f0 + (double)e[7] * f1 + (double)e[8] * f2;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      __syncthreads();
      if (lane == 0) { red[w][0] = s0; red[w][1] = s1; red[w][2] = s2; }
      __syncthreads();
      if (threadIdx.x < 3) {
        double v = 0;
        for (int ww = 0; ww < T256 / 64; ++ww) v += red[ww][threadIdx.x];
        tbuf[3 * (toff[b] + k) + threadIdx.x] = v;
      }
    }
  }
}

template <class T, class TU, class TO, int KIND>
__global__ __launch_bounds__(T256) void k_combine(
    int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ leaf_of,
    const int32_t* __restrict__ parent, const int4* __restrict__ nodes,
    const int32_t* __restrict__ far_ptr, const int2* __restrict__ G,
    const int32_t* __restrict__ rank, const int32_t* __restrict__ flag,
    const int64_t* __restrict__ fptr, const int64_t* __restrict__ toff,
    const T* __restrict__ pool, const double* __restrict__ tbuf, const double* __restrict__ xs,
    const T* __restrict__ Fs, const TU* __restrict__ Un, KParams kp, TO* __restrict__ U) {
  __shared__ T wl[KIND == KIND_MLP ? MLP_NP : 1];
  if (KIND == KIND_MLP) {
    const T* w = (const T*)kp.w;
    for (int i = threadIdx.x; i < MLP_NP; i += T256) wl[i] = w[i];
    __syncthreads();
  }
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n) return;
  double u0 = (double)Un[3 * s], u1 = (double)Un[3 * s + 1], u2 = (double)Un[3 * s + 2];
  const double x0 = xs[3 * s], x1 = xs[3 * s + 1], x2 = xs[3 * s + 2];
  for (int tau = leaf_of[s]; tau >= 0; tau = parent[tau]) {
    const int il = (int)(s - nodes[tau].x);
    const int p1 = far_ptr[tau + 1];
    for (int p = far_ptr[tau]; p < p1; ++p) {
      if (flag[p]) {
        // dense fallback: evaluate the block row directly
        const int4 ns = nodes[G[p].y];
        T v0 = 0, v1 = 0, v2 = 0;
        for (int j = ns.x; j < ns.y; ++j) {
          T K[9];
          kernel_entry<T>(kp, wl, (T)(x0 - xs[3 * (int64_t)j]), (T)(x1 - xs[3 * (int64_t)j + 1]),
                          (T)(x2 - xs[3 * (int64_t)j + 2]), K, (int)(s & 1), j & 1);
          T f0 = Fs[3 * (int64_t)j], f1 = Fs[3 * (int64_t)j + 1], f2 = Fs[3 * (int64_t)j + 2];
          v0 += K[0] * f0 + K[1] * f1 + K[2] * f2;
          v1 += K[3] * f0 + K[4] * f1 + K[5] * f2;
          v2 += K[6] * f0 + K[7] * f1 + K[8] * f2;
        }
        u0 += v0; u1 += v1; u2 += v2;
        continue;
      }
      const int l = rank[p];
      const double* tb = tbuf + 3 * toff[p];
      for (int k = 0; k < l; ++k) {
        const T* e = pool + fptr[(int64_t)p * LMAX_CAP + k] + 9 * (int64_t)il;
        const double t0 = tb[3 * k], t1 = tb[3 * k + 1], t2 = tb[3 * k + 2];
        u0 += (double)e[0] * t0 + (double)e[1] * t1 + (double)e[2] * t2;
        u1 += (double)e[3] * t0 + (double)e[4] * t1 + (double)e[5] * t2;
        u2 += (double)e[6] * t0 + (double)e[7] * t1 + (double)e[8] * t2;
      }
    }
  }
  const double a1 = (s & 1) ? kp.alpha2 : kp.alpha1;
  u0 += a1 * (double)Fs[3 * s];
  u1 += a1 * (double)Fs[3 * s + 1];
  u2 += a1 * (double)Fs[3 * s + 2];
  const int64_t o = perm[s];
  U[3 * o] = (TO)u0;
  U[3 * o + 1] = (TO)u1;
  U[3 * o + 2] = (TO)u2;
}

// Streamed mode: add the rows of the admissible blocks of launch r that
// contain particle s, walking from its leaf to the root (fixed order, no
// atomics). Block b's rows sit at uoff[pos[b]] - uoff[start of launch r].
__global__ __launch_bounds__(T256) void k_far_gather(
    int64_t n, const int32_t* __restrict__ leaf_of, const int32_t* __restrict__ parent,
    const int4* __restrict__ nodes, const int32_t* __restrict__ far_ptr, int32_t r,
    int64_t r0, const int32_t* __restrict__ lid, const int32_t* __restrict__ pos,
    const int64_t* __restrict__ uoff, const double* __restrict__ ublk, double* __restrict__ Uf) {
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n) return;
  double u0 = 0, u1 = 0, u2 = 0;
  const int64_t base = uoff[r0];
  for (int tau = leaf_of[s]; tau >= 0; tau = parent[tau]) {
    const int p0 = far_ptr[tau], p1 = far_ptr[tau + 1];
    if (p0 >= p1) continue;
    const int64_t il = s - nodes[tau].x;
    for (int p = p0; p < p1; ++p) {
      if (lid[p] != r) continue;
      const double* u = ublk + 3 * (uoff[pos[p]] - base + il);
      u0 += u[0]; u1 += u[1]; u2 += u[2];
    }
  }
  Uf[3 * s] += u0;
  Uf[3 * s + 1] += u1;
  Uf[3 * s + 2] += u2;
}

template <class T, class TU, class TO>
__global__ __launch_bounds__(T256) void k_final(int64_t n, const int32_t* __restrict__ perm,
                                                const T* __restrict__ Fs, const TU* __restrict__ Un,
                                                const double* __restrict__ Uf, double alpha1,
                                                double alpha2, TO* __restrict__ U) {
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n) return;
  const int64_t o = perm[s];
  const double a1 = (s & 1) ? alpha2 : alpha1;   // odd rows: rotational rows of a 6N kernel
#pragma unroll
  for (int d = 0; d < 3; ++d)
    U[3 * o + d] = (TO)(((double)Un[3 * s + d] + Uf[3 * s + d]) + a1 * (double)Fs[3 * s + d]);
}

// Stored mode. Fs_ws and Un_ws hold the sorted forces (3 n T) and the
// near-field rows (3 n TU); timed = false records no phase events.
template <class T, class TI, class TO, class TU>
void matvec_t(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k, const void* F,
              void* U, void* Fs_ws, void* Un_ws, bool timed) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  T* Fs = (T*)Fs_ws;
  TU* Un = (TU*)Un_ws;
  hipLaunchKernelGGL((k_gather_rows<TI, T>), dim3(nblk(n)), dim3(T256), 0, st, (const TI*)F,
                     t->perm.as<int32_t>(), n, Fs);
  {
    PhaseTimer timer(ctx, HH_PHASE_NEAR, timed);
    launch_near(ctx, t, p, k, lr->prec, Fs, Un);
  }
  int64_t nG = p->nG;
  if (nG > 0) {
    PhaseTimer timer(ctx, HH_PHASE_FAR, timed);
    int grid = (int)std::min<int64_t>(nG, 8192);
    hipLaunchKernelGGL((k_far_t<T>), dim3(grid), dim3(T256), 0, st, p->G.as<int2>(), nG,
                       t->nodes.as<int4>(), lr->rank.as<int32_t>(), lr->flag.as<int32_t>(),
                       lr->fptr.as<int64_t>(), lr->toff.as<int64_t>(), lr->pool.as<T>(), Fs,
                       lr->tbuf.as<double>());
  }
  KParams kp = make_kparams(k, sizeof(T) == 8);
#define COMBINE(KIND_)                                                                       \
  hipLaunchKernelGGL((k_combine<T, TU, TO, KIND_>), dim3(nblk(n)), dim3(T256), 0, st, n,      \
                     t->perm.as<int32_t>(), t->leaf_of.as<int32_t>(), t->parent.as<int32_t>(), \
                     t->nodes.as<int4>(), p->far_ptr.as<int32_t>(), p->G.as<int2>(),           \
                     lr->rank.as<int32_t>(), lr->flag.as<int32_t>(), lr->fptr.as<int64_t>(),   \
                     lr->toff.as<int64_t>(), lr->pool.as<T>(), lr->tbuf.as<double>(),          \
                     t->xs.as<double>(), Fs, Un, kp, (TO*)U)
  {
    PhaseTimer timer(ctx, HH_PHASE_COMBINE, timed);
    if (k->kind == KIND_MLP) COMBINE(KIND_MLP); else COMBINE(KIND_RPY);
  }
#undef COMBINE
  HIP_OK(hipGetLastError());
}

// Stored mode with the workspaces of the low-rank handle (sized on the first
// product, reused after).
template <class T, class TI, class TO, class TU>
void matvec_ws_t(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k, const void* F,
                 void* U) {
  const int64_t n = t->n;
  lr->ws_f.ensure(ctx->stream, 3 * n * sizeof(T));
  lr->ws_near.ensure(ctx->stream, 3 * n * sizeof(TU));
  matvec_t<T, TI, TO, TU>(ctx, t, p, lr, k, F, U, lr->ws_f.p, lr->ws_near.p, true);
}

// The allocation-free product: the same launches with the workspaces in the
// device's static scratch (base, HH_NOALLOC_SCRATCH_BYTES).
template <class T, class TI, class TO, class TU>
void matvec_noalloc_t(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k,
                      const void* F, void* U, char* base) {
  const int64_t n = t->n;
  const int64_t bf = (3 * n * (int64_t)sizeof(T) + 255) / 256 * 256;
  const int64_t bu = 3 * n * (int64_t)sizeof(TU);
  HH_REQUIRE(bf + bu <= (int64_t)HH_NOALLOC_SCRATCH_BYTES, HH_ERR_CAPACITY,
             "hh_matvec_noalloc: " + std::to_string(n) + " particles need " +
                 std::to_string(bf + bu) + " bytes of scratch, more than the " +
                 std::to_string((int64_t)HH_NOALLOC_SCRATCH_BYTES) + " available");
  matvec_t<T, TI, TO, TU>(ctx, t, p, lr, k, F, U, base, base + bf, false);
}

template <class T, class TI, class TO, class TU>
void matvec_streamed_t(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k,
                       const void* F, void* U) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  DevBuf& Fs = lr->ws_f;
  DevBuf& Un = lr->ws_near;
  DevBuf& Uf = lr->ws_far;
  DevBuf& counters = lr->ws_cnt;
  Fs.ensure(st, 3 * n * sizeof(T));
  Un.ensure(st, 3 * n * sizeof(TU));
  Uf.ensure(st, 3 * n * sizeof(double));
  hipLaunchKernelGGL((k_gather_rows<TI, T>), dim3(nblk(n)), dim3(T256), 0, st, (const TI*)F,
                     t->perm.as<int32_t>(), n, Fs.as<T>());
  {
    PhaseTimer timer(ctx, HH_PHASE_NEAR);
    launch_near(ctx, t, p, k, lr->prec, Fs.p, Un.p);
  }
  zero_words(ctx, Uf.p, 3 * n);
  const size_t nb = lr->bounds.size() - 1;
  counters.ensure(st, ACA_COUNTERS * nb * sizeof(int64_t));
  zero_words(ctx, counters.p, ACA_COUNTERS * (int64_t)nb);
  if (!lr->pool.p) lr->pool.alloc(st, lr->pool_elems * (lr->prec == HH_FP64 ? 8 : 4));
  if (!lr->ublk.p) lr->ublk.alloc(st, lr->ub_elems * 3 * sizeof(double));
  for (size_t i = 0; i < nb; ++i) {
    {
      PhaseTimer timer(ctx, HH_PHASE_ACA);
      run_aca_batch(ctx, t, p, k, lr, i, Fs.p, counters.as<int64_t>());
    }
    PhaseTimer timer(ctx, HH_PHASE_FAR);
    hipLaunchKernelGGL(k_far_gather, dim3(nblk(n)), dim3(T256), 0, st, n,
                       t->leaf_of.as<int32_t>(), t->parent.as<int32_t>(), t->nodes.as<int4>(),
                       p->far_ptr.as<int32_t>(), (int32_t)i, lr->bounds[i], lr->lid.as<int32_t>(),
                       lr->pos.as<int32_t>(), lr->uoff.as<int64_t>(), lr->ublk.as<double>(),
                       Uf.as<double>());
    HIP_OK(hipGetLastError());
  }
  {
    PhaseTimer timer(ctx, HH_PHASE_COMBINE);
    hipLaunchKernelGGL((k_final<T, TU, TO>), dim3(nblk(n)), dim3(T256), 0, st, n,
                       t->perm.as<int32_t>(), Fs.as<T>(), Un.as<TU>(), Uf.as<double>(),
                       k->alpha1, k->alpha2, (TO*)U);
  }
  HIP_OK(hipGetLastError());
  lr->stats_dirty = true;
}

}  // namespace

extern "C" {

hh_status hh_aca_build(hh_ctx ctx, hh_tree tree, hh_part part, hh_kernel kern,
                       hh_precision prec, double eps, int32_t l_max,
                       hh_lowrank freeze_pivots_from, hh_lowrank* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && tree && part && kern, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(part->tree == tree, HH_ERR_INVALID_ARG, "partition was built on another tree");
  check_kernel_tree(tree, kern);
  HH_REQUIRE(kern->kind != KIND_RPY6 || prec == HH_FP64 || prec == HH_FP32, HH_ERR_INVALID_ARG,
             "the 6N kernel runs in HH_FP64 and HH_FP32");
  if (freeze_pivots_from) {
    // the recursion replayed with the pivots, ranks and fallbacks of an
    // earlier build on the same partition (eps and l_max unused)
    hh_lowrank src = freeze_pivots_from;
    HH_REQUIRE(src->part == part, HH_ERR_INVALID_ARG,
               "freeze_pivots_from was built on another partition");
    HH_REQUIRE(!src->streamed, HH_ERR_INVALID_ARG,
               "freeze_pivots_from must hold stored factors (streamed mode keeps none)");
    const int64_t nG = part->nG;
    std::vector<int32_t> rk(std::max<int64_t>(nG, 1)), fb(std::max<int64_t>(nG, 1));
    std::vector<int32_t> pv(std::max<int64_t>(nG, 1) * 2 * LMAX_CAP);
    std::vector<int32_t> pi(std::max<int64_t>(nG, 1) * LMAX_CAP),
        pj(std::max<int64_t>(nG, 1) * LMAX_CAP);
    if (nG > 0) {
      read_bytes(ctx, rk.data(), src->rank.p, nG * sizeof(int32_t));
      read_bytes(ctx, fb.data(), src->flag.p, nG * sizeof(int32_t));
      read_bytes(ctx, pv.data(), src->piv.p, nG * 2 * LMAX_CAP * sizeof(int32_t));
    }
    for (int64_t b = 0; b < nG; ++b)
      for (int m = 0; m < LMAX_CAP; ++m) {
        pi[b * LMAX_CAP + m] = pv[b * 2 * LMAX_CAP + m];
        pj[b * LMAX_CAP + m] = pv[b * 2 * LMAX_CAP + LMAX_CAP + m];
      }
    *out = build_lowrank_pivots(ctx, tree, part, kern, prec, rk.data(), fb.data(), pi.data(),
                                pj.data());
  } else {
    HH_REQUIRE(prec == HH_FP64 || prec == HH_FP32 || is_bf16(prec), HH_ERR_INVALID_ARG,
               "unknown precision");
    HH_REQUIRE(eps >= 0.0 && eps < INFINITY, HH_ERR_INVALID_ARG, "eps must be >= 0");
    HH_REQUIRE(l_max >= 1 && l_max <= LMAX_CAP, HH_ERR_INVALID_ARG, "l_max must be in [1, 64]");
    hh_lowrank_s* lr = new hh_lowrank_s();
    try {
      lr->ctx = ctx;
      lr->part = part;
      lr->prec = prec;
      lr->nG = part->nG;
      lr->l_max = l_max;
      lr->eps = eps;
      lr->kern = kern;
      plan_aca(ctx, tree, part, lr, 0);
      if (!lr->streamed) run_aca_stored(ctx, tree, part, kern, lr);
    } catch (...) {
      delete lr;
      throw;
    }
    *out = lr;
  }
  HH_API_END(ctx)
}

hh_status hh_matvec(hh_ctx ctx, hh_tree tree, hh_part part, hh_lowrank lr, hh_kernel kern,
                    hh_precision prec, const void* F, void* U) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(tree && part && lr && kern && F && U, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(part->tree == tree && lr->part == part, HH_ERR_INVALID_ARG,
             "handles do not belong together");
  HH_REQUIRE(lr->prec == prec, HH_ERR_INVALID_ARG, "precision differs from the ACA build");
  HH_REQUIRE(lr->kern == kern, HH_ERR_INVALID_ARG, "kernel differs from the ACA build");
  // <storage/kernel type, F type, U type, near-field row type>
  const bool mfma = is_bf16(prec) && kern->kind == KIND_MLP;
  if (lr->streamed) {
    if (prec == HH_FP64)
      matvec_streamed_t<double, double, double, double>(ctx, tree, part, lr, kern, F, U);
    else if (prec == HH_FP32)
      matvec_streamed_t<float, float, float, float>(ctx, tree, part, lr, kern, F, U);
    else if (mfma)
      matvec_streamed_t<float, float, double, double>(ctx, tree, part, lr, kern, F, U);
    else
      matvec_streamed_t<float, float, double, float>(ctx, tree, part, lr, kern, F, U);
  } else if (prec == HH_FP64) {
    matvec_ws_t<double, double, double, double>(ctx, tree, part, lr, kern, F, U);
  } else if (prec == HH_FP32) {
    matvec_ws_t<float, float, float, float>(ctx, tree, part, lr, kern, F, U);
  } else if (mfma) {
    matvec_ws_t<float, float, double, double>(ctx, tree, part, lr, kern, F, U);
  } else {
    matvec_ws_t<float, float, double, float>(ctx, tree, part, lr, kern, F, U);
  }
  HH_API_END(ctx)
}

hh_status hh_matvec_noalloc(hh_ctx ctx, hh_tree tree, hh_part part, hh_lowrank lr,
                            hh_kernel kern, hh_precision prec, const void* F, void* U) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(tree && part && lr && kern && F && U, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(part->tree == tree && lr->part == part, HH_ERR_INVALID_ARG,
             "handles do not belong together");
  HH_REQUIRE(lr->prec == prec, HH_ERR_INVALID_ARG, "precision differs from the ACA build");
  HH_REQUIRE(lr->kern == kern, HH_ERR_INVALID_ARG, "kernel differs from the ACA build");
  HH_REQUIRE(ctx->noalloc_scratch, HH_ERR_HIP, "no scratch address on this device");
  char* base = (char*)ctx->noalloc_scratch;
  const bool mfma = is_bf16(prec) && kern->kind == KIND_MLP;
  // the size limit first: it depends only on n and the precision
  const int64_t n = tree->n;
  const int64_t need = (3 * n * (prec == HH_FP64 ? 8 : 4) + 255) / 256 * 256 +
                       3 * n * ((prec == HH_FP64 || mfma) ? 8 : 4);
  HH_REQUIRE(need <= (int64_t)HH_NOALLOC_SCRATCH_BYTES, HH_ERR_CAPACITY,
             "hh_matvec_noalloc: " + std::to_string(n) + " particles need " +
                 std::to_string(need) + " bytes of scratch, more than the " +
                 std::to_string((int64_t)HH_NOALLOC_SCRATCH_BYTES) + " available");
  HH_REQUIRE(!lr->streamed, HH_ERR_INVALID_ARG,
             "hh_matvec_noalloc needs stored factors (streamed mode runs the ACA in the product)");
  HH_REQUIRE(tree->n_units > 0, HH_ERR_INVALID_ARG, "tree has no near-field work units");
  if (prec == HH_FP64)
    matvec_noalloc_t<double, double, double, double>(ctx, tree, part, lr, kern, F, U, base);
  else if (prec == HH_FP32)
    matvec_noalloc_t<float, float, float, float>(ctx, tree, part, lr, kern, F, U, base);
  else if (mfma)
    matvec_noalloc_t<float, float, double, double>(ctx, tree, part, lr, kern, F, U, base);
  else
    matvec_noalloc_t<float, float, double, float>(ctx, tree, part, lr, kern, F, U, base);
  HH_API_END(ctx)
}

void hh_lowrank_free(hh_lowrank l) { delete l; }

hh_status hh_lowrank_info(hh_lowrank l, int64_t* n_blocks, int64_t* rank_sum,
                          int64_t* n_fallback, int64_t* samples, int64_t* bytes) {
  if (!l) return HH_ERR_INVALID_ARG;
  if (l->stats_dirty && (!l->streamed || l->pool.p)) {
    try {
      (void)hipSetDevice(l->ctx->device);
      lowrank_stats(l->ctx, l->part->tree, l->part, l, false);
    } catch (const hh_error& e) {
      l->ctx->last_error = e.msg;
      return e.st;
    }
  }
  if (n_blocks) *n_blocks = l->nG;
  if (rank_sum) *rank_sum = l->rank_sum;
  if (n_fallback) *n_fallback = l->n_fallback;
  if (samples) *samples = l->samples;
  if (bytes) *bytes = l->used_elems * (int64_t)(l->prec == HH_FP64 ? 8 : 4);
  return HH_OK;
}

hh_status hh_lowrank_export(hh_lowrank l, int32_t* rank, int32_t* fallback, int32_t* piv_i,
                            int32_t* piv_j) {
  if (!l) return HH_ERR_INVALID_ARG;
  hh_ctx ctx = l->ctx;
  HH_API_BEGIN(ctx)
  int64_t nG = l->nG;
  if (rank) read_bytes(ctx, rank, l->rank.p, nG * sizeof(int32_t));
  if (fallback) read_bytes(ctx, fallback, l->flag.p, nG * sizeof(int32_t));
  if (piv_i || piv_j) {
    std::vector<int32_t> pv(nG * 2 * LMAX_CAP);
    read_bytes(ctx, pv.data(), l->piv.p, pv.size() * sizeof(int32_t));
    for (int64_t b = 0; b < nG; ++b)
      for (int m = 0; m < LMAX_CAP; ++m) {
        if (piv_i) piv_i[b * LMAX_CAP + m] = pv[b * 2 * LMAX_CAP + m];
        if (piv_j) piv_j[b * LMAX_CAP + m] = pv[b * 2 * LMAX_CAP + LMAX_CAP + m];
      }
  }
  HH_API_END(ctx)
}

hh_status hh_lowrank_factor(hh_lowrank l, int64_t b, int32_t k, double* ck, double* qk) {
  if (!l) return HH_ERR_INVALID_ARG;
  hh_ctx ctx = l->ctx;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(!l->streamed, HH_ERR_INVALID_ARG,
             "factors are not kept in streamed mode (they live only inside a batch)");
  HH_REQUIRE(b >= 0 && b < l->nG, HH_ERR_INVALID_ARG, "block index out of range");
  int32_t r;
  read_bytes(ctx, &r, l->rank.as<int32_t>() + b, sizeof(int32_t));
  HH_REQUIRE(k >= 0 && k < r, HH_ERR_INVALID_ARG, "term index out of range");
  hh_tree t = l->part->tree;
  int2 g;
  read_bytes(ctx, &g, l->part->G.as<int2>() + b, sizeof(int2));
  int4 nt, ns;
  read_bytes(ctx, &nt, t->nodes.as<int4>() + g.x, sizeof(int4));
  read_bytes(ctx, &ns, t->nodes.as<int4>() + g.y, sizeof(int4));
  int64_t off;
  read_bytes(ctx, &off, l->fptr.as<int64_t>() + b * LMAX_CAP + k, sizeof(int64_t));
  int64_t c = nt.y - nt.x, q = ns.y - ns.x;
  int64_t cnt = 9 * (c + q);
  std::vector<double> v(cnt);
  if (l->prec == HH_FP64) {
    read_bytes(ctx, v.data(), l->pool.as<double>() + off, cnt * sizeof(double));
  } else {
    std::vector<float> f(cnt);
    read_bytes(ctx, f.data(), l->pool.as<float>() + off, cnt * sizeof(float));
    for (int64_t i = 0; i < cnt; ++i) v[i] = f[i];
  }
  if (ck) for (int64_t i = 0; i < 9 * c; ++i) ck[i] = v[i];
  if (qk) for (int64_t i = 0; i < 9 * q; ++i) qk[i] = v[9 * c + i];
  HH_API_END(ctx)
}

}  // extern "C"
