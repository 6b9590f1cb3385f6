// Near field: U_i += sum over inadmissible leaf blocks (tau, sigma) in P^H of
// sum_{j in sigma, j != i} K(x_i - x_j) F_j (Sec. 3.3.1), kernel evaluated on
// the fly and never stored.
//
// One workgroup per target leaf tau (owner computes: each target row is
// written once, no atomics). The sources of each near leaf sigma are staged
// through LDS in tiles of NEAR_T particles (positions FP64, forces in the
// working type), so every thread reads them with LDS broadcasts. Inputs are
// in Morton order, so the staging loads are contiguous.
#include "devmath.h"
#include "internal.h"

namespace {

constexpr int NEAR_T = 128;

template <class T>
struct NearArgs {
  const int4* nodes;
  const int32_t* leaves;
  const int32_t* near_ptr;
  const int2* H;
  const double* xs;
  const T* Fs;
  T* Un;
  KParams kp;
  int64_t n_leaves;
  double sgn;   // +1: K(x_i - x_j); -1: K(x_j - x_i) (transposed product)
};

template <class T, int KIND>
__global__ __launch_bounds__(NEAR_T) void k_near_valu(NearArgs<T> a) {
  __shared__ T wl[KIND == KIND_MLP ? MLP_NP : 1];
  __shared__ double sx[NEAR_T * 3];
  __shared__ T sf[NEAR_T * 3];
  if (KIND == KIND_MLP) {
    const T* w = (const T*)a.kp.w;
    for (int i = threadIdx.x; i < MLP_NP; i += NEAR_T) wl[i] = w[i];
  }
  const int leaf = blockIdx.x;
  const int4 nt = a.nodes[a.leaves[leaf]];
  const int p0 = a.near_ptr[leaf], p1 = a.near_ptr[leaf + 1];
  for (int ib = nt.x; ib < nt.y; ib += NEAR_T) {
    const int i = ib + threadIdx.x;
    const bool act = i < nt.y;
    double xi0 = 0, xi1 = 0, xi2 = 0;
    if (act) { xi0 = a.xs[3 * (int64_t)i]; xi1 = a.xs[3 * (int64_t)i + 1]; xi2 = a.xs[3 * (int64_t)i + 2]; }
    T u0 = 0, u1 = 0, u2 = 0;
    for (int p = p0; p < p1; ++p) {
      const int4 ns = a.nodes[a.H[p].y];
      for (int jb = ns.x; jb < ns.y; jb += NEAR_T) {
        const int cnt = min(NEAR_T, ns.y - jb);
        __syncthreads();
        for (int t = threadIdx.x; t < 3 * cnt; t += NEAR_T) {
          sx[t] = a.xs[3 * (int64_t)jb + t];
          sf[t] = a.Fs[3 * (int64_t)jb + t];
        }
        __syncthreads();
        if (act) {
          for (int jj = 0; jj < cnt; ++jj) {
            if (same_particle(a.kp.kind, jb + jj, i)) continue;
            T rx = (T)(a.sgn * (xi0 - sx[3 * jj])), ry = (T)(a.sgn * (xi1 - sx[3 * jj + 1])),
              rz = (T)(a.sgn * (xi2 - sx[3 * jj + 2]));
            T K[9];
            kernel_entry<T>(a.kp, wl, rx, ry, rz, K, i & 1, (jb + jj) & 1);
            T f0 = sf[3 * jj], f1 = sf[3 * jj + 1], f2 = sf[3 * jj + 2];
            u0 += K[0] * f0 + K[1] * f1 + K[2] * f2;
            u1 += K[3] * f0 + K[4] * f1 + K[5] * f2;
            u2 += K[6] * f0 + K[7] * f1 + K[8] * f2;
          }
        }
      }
    }
    if (act) {
      a.Un[3 * (int64_t)i] = u0;
      a.Un[3 * (int64_t)i + 1] = u1;
      a.Un[3 * (int64_t)i + 2] = u2;
    }
  }
}

template <class T>
void launch_near_t(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const void* Fs, void* Un,
                   double sgn = 1.0) {
  NearArgs<T> a;
  a.sgn = sgn;
  a.nodes = t->nodes.as<int4>();
  a.leaves = t->leaves.as<int32_t>();
  a.near_ptr = p->near_ptr.as<int32_t>();
  a.H = p->H.as<int2>();
  a.xs = t->xs.as<double>();
  a.Fs = (const T*)Fs;
  a.Un = (T*)Un;
  a.kp.kind = k->kind;
  a.kp.input_mode = k->input_mode;
  a.kp.a = k->a;
  a.kp.c8 = 1.0 / (8.0 * HH_PI * k->mu);
  a.kp.c6 = 1.0 / (6.0 * HH_PI * k->mu * k->a);
  a.kp.alpha1 = k->alpha1;
  a.kp.alpha2 = k->alpha2;
  a.kp.w = sizeof(T) == 8 ? k->p64.p : k->p32.p;
  a.n_leaves = t->n_leaves;
  if (k->kind == KIND_MLP)
    hipLaunchKernelGGL((k_near_valu<T, KIND_MLP>), dim3(t->n_leaves), dim3(NEAR_T), 0,
                       ctx->stream, a);
  else
    hipLaunchKernelGGL((k_near_valu<T, KIND_RPY>), dim3(t->n_leaves), dim3(NEAR_T), 0,
                       ctx->stream, a);
  HIP_OK(hipGetLastError());
}

}  // namespace

// Near field with the displacement reversed: sum_j K(x_j - x_i) v_j, which is
// the transposed near product (K entries are symmetric 3x3 matrices).
void launch_near_neg(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, int prec, const void* Vs,
                     void* out) {
  if (prec == HH_FP64)
    launch_near_t<double>(ctx, t, p, k, Vs, out, -1.0);
  else if (k->kind == KIND_MLP)
    launch_near_f32(ctx, t, p, k, Vs, out, -1.0f);
  else
    launch_near_t<float>(ctx, t, p, k, Vs, out, -1.0);
}

void launch_near(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, int prec, const void* Fs,
                 void* Un) {
  if (prec == HH_FP64)
    launch_near_t<double>(ctx, t, p, k, Fs, Un);
  else if (prec == HH_FP32 && k->kind == KIND_MLP)
    launch_near_f32(ctx, t, p, k, Fs, Un);
  else if (prec == HH_FP32 || k->kind != KIND_MLP)
    launch_near_t<float>(ctx, t, p, k, Fs, Un);
  else
    launch_near_bf16(ctx, t, p, k, Fs, Un, prec == HH_BF16_SPLIT);   // writes FP64 rows
}
