// Forces and the explicit Euler update of a time step (Sec. 4.3).
//
// Every particle carries a uniform external force (gravity, (0, 0, -1) in
// Sec. 4.3.1). Filaments are chains of n_beads consecutive particles (chain c
// holds [c n_beads, (c + 1) n_beads)) with the two internal forces of Sec.
// 4.3.2: tension k_t (|r| - l_0) r / |r| on each bond r = x_{i+1} - x_i
// (+ on bead i, - on bead i+1), and COS bending on each interior bead i:
// t_1, t_2 the unit bond vectors into and out of i, T = -k_b (t_1 x t_2)
// |t_1 x t_2|, forces T x t_1 on i-1, -T x t_2 on i+1 and minus their sum
// on i. One thread per particle gathers every term that touches it (its two
// bonds and the three bends it takes part in), so no atomics are needed and
// the result is deterministic. The Euler step is X += dt U.
#include <algorithm>

#include "api_guard.h"
#include "internal.h"

namespace {

constexpr int TB = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + TB - 1) / TB); }

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 ld(const double* X, int64_t i) {
  return V3{X[3 * i], X[3 * i + 1], X[3 * i + 2]};
}
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 add(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 mul(V3 a, double s) { return V3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double norm(V3 a) { return sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// tension force of bond (i, i+1) as added to bead i
__device__ __forceinline__ V3 tension(const double* X, int64_t i, double kt, double l0) {
  const V3 r = sub(ld(X, i + 1), ld(X, i));
  const double d = norm(r);
  return mul(r, kt * (d - l0) / d);
}

// bending forces of the triple centred at bead i: on i-1 (prev), i+1 (next)
__device__ __forceinline__ void bend(const double* X, int64_t i, double kb, V3& prev, V3& next) {
  const V3 a = sub(ld(X, i), ld(X, i - 1)), b = sub(ld(X, i + 1), ld(X, i));
  const V3 t1 = mul(a, 1.0 / norm(a)), t2 = mul(b, 1.0 / norm(b));
  const V3 c = cross(t1, t2);
  const V3 T = mul(c, -kb * norm(c));
  prev = cross(T, t1);
  next = mul(cross(T, t2), -1.0);
}

template <class TF>
__global__ __launch_bounds__(TB) void k_forces(const double* __restrict__ X, int64_t n,
                                               int64_t n_fil, int n_beads, double kt, double l0,
                                               double kb, double g0, double g1, double g2,
                                               TF* __restrict__ F) {
  const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  V3 f{g0, g1, g2};
  if (s < n_fil * (int64_t)n_beads) {
    const int b = (int)(s % n_beads);
    if (b + 1 < n_beads) f = add(f, tension(X, s, kt, l0));
    if (b > 0) f = sub(f, tension(X, s - 1, kt, l0));
    V3 p, q;
    if (b >= 2) {   // bend centred at s-1: s is its next bead
      bend(X, s - 1, kb, p, q);
      f = add(f, q);
    }
    if (b >= 1 && b + 1 < n_beads) {   // bend centred at s
      bend(X, s, kb, p, q);
      f = sub(f, add(p, q));
    }
    if (b + 2 < n_beads) {   // bend centred at s+1: s is its previous bead
      bend(X, s + 1, kb, p, q);
      f = add(f, p);
    }
  }
  F[3 * s] = (TF)f.x;
  F[3 * s + 1] = (TF)f.y;
  F[3 * s + 2] = (TF)f.z;
}

template <class TU>
__global__ __launch_bounds__(TB) void k_euler(double* __restrict__ X, const TU* __restrict__ U,
                                              int64_t n, double dt) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= 3 * n) return;
  X[i] += dt * (double)U[i];
}

}  // namespace

extern "C" {

hh_status hh_filament_forces(hh_ctx ctx, const double* X, int64_t n, int64_t n_fil,
                             int32_t n_beads, double k_t, double l0, double k_b,
                             const double* gravity, hh_precision prec, void* F) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(X && F && gravity, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(n >= 1 && n_fil >= 0 && (n_fil == 0 || n_beads >= 2), HH_ERR_INVALID_ARG,
             "n >= 1, n_fil >= 0 and n_beads >= 2 for filaments");
  HH_REQUIRE(n_fil * (int64_t)std::max(n_beads, 0) <= n, HH_ERR_INVALID_ARG,
             "the filaments hold more beads than there are particles");
  HH_REQUIRE(l0 >= 0, HH_ERR_INVALID_ARG, "l0 must be >= 0");
  if (prec == HH_FP64)
    hipLaunchKernelGGL(k_forces<double>, dim3(nblk(n)), dim3(TB), 0, ctx->stream, X, n, n_fil,
                       n_beads, k_t, l0, k_b, gravity[0], gravity[1], gravity[2], (double*)F);
  else
    hipLaunchKernelGGL(k_forces<float>, dim3(nblk(n)), dim3(TB), 0, ctx->stream, X, n, n_fil,
                       n_beads, k_t, l0, k_b, gravity[0], gravity[1], gravity[2], (float*)F);
  HIP_OK(hipGetLastError());
  HH_API_END(ctx)
}

hh_status hh_euler_step(hh_ctx ctx, double* X, const void* U, int64_t n, double dt,
                        hh_precision prec) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(X && U && n >= 1, HH_ERR_INVALID_ARG, "NULL argument or n < 1");
  if (prec == HH_FP32)
    hipLaunchKernelGGL(k_euler<float>, dim3(nblk(3 * n)), dim3(TB), 0, ctx->stream, X,
                       (const float*)U, n, dt);
  else
    hipLaunchKernelGGL(k_euler<double>, dim3(nblk(3 * n)), dim3(TB), 0, ctx->stream, X,
                       (const double*)U, n, dt);
  HIP_OK(hipGetLastError());
  HH_API_END(ctx)
}

}  // extern "C"
