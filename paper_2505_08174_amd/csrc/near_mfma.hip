// Near field with the seeded MLP kernel on BF16 MFMA (the BF16 form).
//
// Work unit = 32 consecutive targets of one leaf tau (one wave). The wave
// walks every source j of every near leaf sigma of tau (uniform across the
// wave, so x_j and F_j come through scalar loads) and evaluates the 32 pairs
// (i, j) as one MFMA tile; each lane accumulates K(x_i - x_j) F_j for its own
// target in FP64 (owner computes, no reduction, no atomics). Four units per
// workgroup share the weight fragments staged in LDS.
#include "internal.h"
#include "mlp_mfma.h"

#define T256_UNITS 256

namespace {

constexpr int NB_T = 256;

__global__ __launch_bounds__(T256_UNITS) void k_units_count(const int32_t* __restrict__ leaves,
                                                            int64_t nl,
                                                            const int4* __restrict__ nodes,
                                                            int64_t* __restrict__ cnt) {
  int64_t l = (int64_t)blockIdx.x * T256_UNITS + threadIdx.x;
  if (l > nl) return;
  if (l == nl) { cnt[nl] = 0; return; }
  int4 nd = nodes[leaves[l]];
  cnt[l] = (nd.y - nd.x + 31) / 32;
}

__global__ __launch_bounds__(T256_UNITS) void k_units_fill(const int64_t* __restrict__ cnt,
                                                           const int64_t* __restrict__ pos,
                                                           int64_t nl, int2* __restrict__ units) {
  int64_t l = (int64_t)blockIdx.x * T256_UNITS + threadIdx.x;
  if (l >= nl) return;
  for (int64_t c = 0; c < cnt[l]; ++c) units[pos[l] + c] = make_int2((int)l, (int)c);
}

struct NearB {
  const uint4* frags;
  const int4* nodes;
  const int32_t* leaves;
  const int32_t* near_ptr;
  const int2* H;
  const int2* units;
  int64_t n_units;
  const double* xs;
  const float* Fs;
  double* Un;
  int input_mode;
};

// Adds K(x_i - x_j) F_j for the sources j0, j0 + 1, .., j0 + NT - 1 (one MFMA
// tile each, evaluated together), in that order.
template <bool ACC, int NT>
__device__ __forceinline__ void near_terms(const NearB& a, const bf16x8* fr, bool dir, bool act,
                                           int ii, double xi0, double xi1, double xi2, int j0,
                                           double& u0, double& u1, double& u2) {
  const float c16 = (float)(1.0 / (16.0 * HH_PI));
  float v[NT][3], rs[NT], o[NT][9];
  bool skip[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + t;
    float rx = (float)(xi0 - a.xs[3 * (int64_t)j]);
    float ry = (float)(xi1 - a.xs[3 * (int64_t)j + 1]);
    float rz = (float)(xi2 - a.xs[3 * (int64_t)j + 2]);
    skip[t] = (j == ii) || !act;
    if (j == ii) { rx = 1.0f; ry = 0.0f; rz = 0.0f; }
    rs[t] = hh_rsqrt(rx * rx + ry * ry + rz * rz);
    const float sc = dir ? rs[t] : 1.0f;
    v[t][0] = rx * sc;
    v[t][1] = ry * sc;
    v[t][2] = rz * sc;
  }
  mlp_tiles_bf16<ACC, NT>(fr, v, o);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + t;
    const float sc = skip[t] ? 0.0f : rs[t] * c16;
    const float f0 = a.Fs[3 * (int64_t)j], f1 = a.Fs[3 * (int64_t)j + 1],
                f2 = a.Fs[3 * (int64_t)j + 2];
    const float* q = o[t];
    u0 += (double)(sc * (2.0f * q[0] * f0 + (q[1] + q[3]) * f1 + (q[2] + q[6]) * f2));
    u1 += (double)(sc * ((q[3] + q[1]) * f0 + 2.0f * q[4] * f1 + (q[5] + q[7]) * f2));
    u2 += (double)(sc * ((q[6] + q[2]) * f0 + (q[7] + q[5]) * f1 + 2.0f * q[8] * f2));
  }
}

template <bool ACC>
__global__ __launch_bounds__(NB_T) void k_near_bf16(NearB a) {
  __shared__ bf16x8 fr[FR_TOTAL];
  stage_frags(fr, a.frags, NB_T);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t unit = (int64_t)blockIdx.x * (NB_T / 64) + w;
  if (unit >= a.n_units) return;
  const int2 un = a.units[unit];
  const int4 nt = a.nodes[a.leaves[un.x]];
  const int i = nt.x + 32 * un.y + (lane & 31);
  const bool act = i < nt.y;
  const int ii = act ? i : nt.x;
  const double xi0 = a.xs[3 * (int64_t)ii], xi1 = a.xs[3 * (int64_t)ii + 1],
               xi2 = a.xs[3 * (int64_t)ii + 2];
  const bool dir = a.input_mode == HH_MLP_INPUT_DIRECTION;
  double u0 = 0, u1 = 0, u2 = 0;
  const int p0 = a.near_ptr[un.x], p1 = a.near_ptr[un.x + 1];
  for (int p = p0; p < p1; ++p) {
    const int4 ns = a.nodes[a.H[p].y];
    int j = ns.x;
    // two sources at a time: two independent MFMA chains per wave
    for (; j + 1 < ns.y; j += 2)
      near_terms<ACC, 2>(a, fr, dir, act, ii, xi0, xi1, xi2, j, u0, u1, u2);
    if (j < ns.y) near_terms<ACC, 1>(a, fr, dir, act, ii, xi0, xi1, xi2, j, u0, u1, u2);
  }
  if (act && lane < 32) {
    a.Un[3 * (int64_t)i] = u0;
    a.Un[3 * (int64_t)i + 1] = u1;
    a.Un[3 * (int64_t)i + 2] = u2;
  }
}

// The plain FP32 form on FP32 MFMA: the same work units and walk, one FP32
// tile per source. F and U are FP32; each lane sums its target's terms in
// FP64 and rounds once.
struct NearF {
  const float4* frags;
  const int4* nodes;
  const int32_t* leaves;
  const int32_t* near_ptr;
  const int2* H;
  const int2* units;
  int64_t n_units;
  const double* xs;
  const float* Fs;
  float* Un;
  int input_mode;
  float sgn;   // +1: K(x_i - x_j); -1: K(x_j - x_i) (the transposed product)
};

__global__ __launch_bounds__(NB_T) void k_near_f32(NearF a) {
  __shared__ float fr[F32_FRAGS * 64];
  stage_frags_f32(fr, a.frags, NB_T);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t unit = (int64_t)blockIdx.x * (NB_T / 64) + w;
  if (unit >= a.n_units) return;
  const int2 un = a.units[unit];
  const int4 nt = a.nodes[a.leaves[un.x]];
  const int i = nt.x + 32 * un.y + (lane & 31);
  const bool act = i < nt.y;
  const int ii = act ? i : nt.x;
  const double xi0 = a.xs[3 * (int64_t)ii], xi1 = a.xs[3 * (int64_t)ii + 1],
               xi2 = a.xs[3 * (int64_t)ii + 2];
  const bool dir = a.input_mode == HH_MLP_INPUT_DIRECTION;
  const float c16 = (float)(1.0 / (16.0 * HH_PI));
  double u0 = 0, u1 = 0, u2 = 0;
  const int p0 = a.near_ptr[un.x], p1 = a.near_ptr[un.x + 1];
  for (int p = p0; p < p1; ++p) {
    const int4 ns = a.nodes[a.H[p].y];
    for (int j = ns.x; j < ns.y; ++j) {
      float rx = a.sgn * (float)(xi0 - a.xs[3 * (int64_t)j]);
      float ry = a.sgn * (float)(xi1 - a.xs[3 * (int64_t)j + 1]);
      float rz = a.sgn * (float)(xi2 - a.xs[3 * (int64_t)j + 2]);
      const bool skip = (j == ii) || !act;
      if (j == ii) { rx = 1.0f; ry = 0.0f; rz = 0.0f; }
      const float rs = hh_rsqrt(rx * rx + ry * ry + rz * rz);
      const float sv = dir ? rs : 1.0f;
      float q[9];
      mlp_tile_f32(fr, rx * sv, ry * sv, rz * sv, q);
      const float sc = skip ? 0.0f : rs * c16;
      const float f0 = a.Fs[3 * (int64_t)j], f1 = a.Fs[3 * (int64_t)j + 1],
                  f2 = a.Fs[3 * (int64_t)j + 2];
      u0 += (double)(sc * (2.0f * q[0] * f0 + (q[1] + q[3]) * f1 + (q[2] + q[6]) * f2));
      u1 += (double)(sc * ((q[3] + q[1]) * f0 + 2.0f * q[4] * f1 + (q[5] + q[7]) * f2));
      u2 += (double)(sc * ((q[6] + q[2]) * f0 + (q[7] + q[5]) * f1 + 2.0f * q[8] * f2));
    }
  }
  if (act && lane < 32) {
    a.Un[3 * (int64_t)i] = (float)u0;
    a.Un[3 * (int64_t)i + 1] = (float)u1;
    a.Un[3 * (int64_t)i + 2] = (float)u2;
  }
}

}  // namespace

// Work units (leaf rank, chunk of 32 targets), built once per tree.
void ensure_units(hh_ctx ctx, hh_tree t) {
  if (t->n_units > 0) return;
  hipStream_t st = ctx->stream;
  int64_t nl = t->n_leaves;
  DevBuf cnt, pos;
  cnt.alloc(st, (nl + 1) * sizeof(int64_t));
  pos.alloc(st, (nl + 1) * sizeof(int64_t));
  unsigned g = (unsigned)((nl + 1 + T256_UNITS - 1) / T256_UNITS);
  hipLaunchKernelGGL(k_units_count, dim3(g), dim3(T256_UNITS), 0, st, t->leaves.as<int32_t>(), nl,
                     t->nodes.as<int4>(), cnt.as<int64_t>());
  scan_exclusive_i64(ctx, cnt.as<int64_t>(), pos.as<int64_t>(), nl + 1);
  int64_t nu = read_i64(ctx, pos.as<int64_t>() + nl);
  t->units.alloc(st, std::max<int64_t>(1, nu) * sizeof(int2));
  hipLaunchKernelGGL(k_units_fill, dim3(g), dim3(T256_UNITS), 0, st, cnt.as<int64_t>(),
                     pos.as<int64_t>(), nl, t->units.as<int2>());
  HIP_OK(hipGetLastError());
  t->n_units = nu;
}

void launch_near_bf16(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const void* Fs, void* Un,
                      bool split) {
  HH_REQUIRE(k->kind == KIND_MLP, HH_ERR_INVALID_ARG, "the BF16 form needs the MLP kernel");
  ensure_units(ctx, t);
  NearB a;
  a.frags = k->pbf.as<uint4>();
  a.nodes = t->nodes.as<int4>();
  a.leaves = t->leaves.as<int32_t>();
  a.near_ptr = p->near_ptr.as<int32_t>();
  a.H = p->H.as<int2>();
  a.units = t->units.as<int2>();
  a.n_units = t->n_units;
  a.xs = t->xs.as<double>();
  a.Fs = (const float*)Fs;
  a.Un = (double*)Un;
  a.input_mode = k->input_mode;
  unsigned grid = (unsigned)((t->n_units + 3) / 4);
  if (split)
    hipLaunchKernelGGL(k_near_bf16<true>, dim3(grid), dim3(NB_T), 0, ctx->stream, a);
  else
    hipLaunchKernelGGL(k_near_bf16<false>, dim3(grid), dim3(NB_T), 0, ctx->stream, a);
  HIP_OK(hipGetLastError());
}

void launch_near_f32(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, const void* Fs, void* Un,
                     float sgn) {
  HH_REQUIRE(k->kind == KIND_MLP, HH_ERR_INVALID_ARG, "the FP32 MFMA tile needs the MLP kernel");
  ensure_units(ctx, t);
  NearF a;
  a.frags = k->pf32.as<float4>();
  a.nodes = t->nodes.as<int4>();
  a.leaves = t->leaves.as<int32_t>();
  a.near_ptr = p->near_ptr.as<int32_t>();
  a.H = p->H.as<int2>();
  a.units = t->units.as<int2>();
  a.n_units = t->n_units;
  a.xs = t->xs.as<double>();
  a.Fs = (const float*)Fs;
  a.Un = (float*)Un;
  a.input_mode = k->input_mode;
  a.sgn = sgn;
  unsigned grid = (unsigned)((t->n_units + 3) / 4);
  hipLaunchKernelGGL(k_near_f32, dim3(grid), dim3(NB_T), 0, ctx->stream, a);
  HIP_OK(hipGetLastError());
}
