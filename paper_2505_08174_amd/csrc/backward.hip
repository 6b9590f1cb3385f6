// Gradients of L = sum_i dU_i . U_i for the H-matrix product, with the tree,
// the partition and the ACA pivots frozen (the product is then a smooth
// function of X, F and the MLP parameters, and these are its exact
// derivatives).
//
//  dF = alpha_1 w + (near field with the displacement reversed) + Q^T (C^T w)
//  dX, dtheta: every near pair (i, j) re-evaluates the MLP and back-propagates
//  the cotangent w_i F_j^T (no pair activations are stored); every admissible
//  block runs the reverse of the ACA recursion (the column, pivot and row steps of Algorithm 2, with
//  the pivots frozen; the pivot entry P_k equals q_k(j_k)), which yields a
//  cotangent for every kernel sample it took, and those sampled pairs are
//  back-propagated the same way.
// Accumulation: dX of a target row in registers, of a source row with FP64
// atomics; dtheta per workgroup in LDS (FP64 in every form), then summed over
// workgroups in a fixed order in FP64. The FP32 form back-propagates the near
// pairs and the ACA samples on FP32 MFMA tiles instead (backward_mfma.hip).
#include "api_guard.h"
#include "devmath.h"
#include "internal.h"

void block_sizes(hh_ctx ctx, hh_tree t, hh_part p, std::vector<int32_t>& cs,
                 std::vector<int32_t>& qs);

namespace {

constexpr int TB = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + TB - 1) / TB); }
// cotangent-pool elements per chunk of blocks (8 GiB in FP32): few chunks, so
// that the back-propagation of the samples runs in few launches
constexpr int64_t GPOOL_CHUNK = 2048ll << 20;

// dtheta: every wave sums its 64 lanes' contributions to a parameter with DPP
// (all lanes active, a fixed order), and one lane per wave adds the total to
// the workgroup's FP64 accumulator in LDS, up to 64 parameters per atomic
// instruction (one per lane, distinct addresses).

// v + (v of the source lane given by a DPP control); 0 from lanes outside the
// row or in rows masked off
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int x = __float_as_int(v);
  const int s = ROW_MASK == 0xf ? __builtin_amdgcn_update_dpp(x, x, CTRL, 0xf, 0xf, true)
                                : __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, false);
  return v + __int_as_float(s);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int slo, shi;
  if (ROW_MASK == 0xf) {
    slo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, true);
    shi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, true);
  } else {
    slo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
    shi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
  }
  return v + __hiloint2double(shi, slo);
}

// Sum over the 64 lanes (every lane active), returned in every lane: scans
// by row shifts 1, 2, 4, 8 in each 16-lane row, then the lane-15 and lane-31
// row broadcasts carry the row sums into lane 63.
template <class T>
__device__ __forceinline__ T wave_total(T v) {
  v = dpp_add<0x111, 0xf>(v);
  v = dpp_add<0x112, 0xf>(v);
  v = dpp_add<0x114, 0xf>(v);
  v = dpp_add<0x118, 0xf>(v);
  v = dpp_add<0x142, 0xa>(v);
  v = dpp_add<0x143, 0xc>(v);
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  } else {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
  }
}

// Wave totals of up to 64 parameters, total k kept in lane k, then added to
// dth[base + stride * lane] (one LDS atomic instruction).
template <class T>
struct RowSum {
  T r = 0;
  __device__ __forceinline__ void put(int k, T v) {
    const T t = wave_total(v);
    r = (int)(threadIdx.x & 63) == k ? t : r;
  }
  __device__ __forceinline__ void flush(double* base, int count, int stride = 1) {
    const int lane = threadIdx.x & 63;
    if (lane < count) atomicAdd(base + stride * lane, (double)r);
    r = 0;
  }
};

// Cotangent of one kernel entry K(r) (3x3, symmetric) for the MLP kernel:
// adds d/dtheta of sum_ab gb_ab K_ab(r) over the wave's 64 lanes into dth
// (LDS, packed layout) and returns this lane's d/dr. Every lane of the wave
// must call it (a lane with nothing to add passes gb = 0 and any r != 0).
template <class T>
__device__ void mlp_vjp(const T* __restrict__ P, int mode, T rx, T ry, T rz,
                        const T gb[9], double* __restrict__ dth, T dr[3]) {
  const T d2 = rx * rx + ry * ry + rz * rz;
  const T id = hh_rsqrt(d2);
  T v0 = rx, v1 = ry, v2 = rz;
  const bool dir = mode == HH_MLP_INPUT_DIRECTION;
  if (dir) { v0 *= id; v1 *= id; v2 *= id; }
  T h1[MLP_H], h2[MLP_H], h3[MLP_H], dl[MLP_H], o[9];
#pragma unroll 8
  for (int k = 0; k < MLP_H; ++k)
    h1[k] = hh_tanh(P[OFF_B1 + k] + P[OFF_W1 + 3 * k] * v0 + P[OFF_W1 + 3 * k + 1] * v1 +
                    P[OFF_W1 + 3 * k + 2] * v2);
  for (int a = 0; a < MLP_H; ++a) {
    T z = P[OFF_B2 + a];
    for (int k = 0; k < MLP_H; ++k) z += P[OFF_W2 + MLP_H * a + k] * h1[k];
    h2[a] = hh_tanh(z);
  }
  for (int a = 0; a < MLP_H; ++a) {
    T z = P[OFF_B3 + a];
    for (int k = 0; k < MLP_H; ++k) z += P[OFF_W3 + MLP_H * a + k] * h2[k];
    h3[a] = hh_tanh(z);
  }
  for (int m = 0; m < 9; ++m) {
    T z = P[OFF_B4 + m];
    for (int k = 0; k < MLP_H; ++k) z += P[OFF_W4 + MLP_H * m + k] * h3[k];
    o[m] = z;
  }
  // g = symmetric part of the cotangent, flattened row-major; s = 1/(8 pi |r|)
  T g[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) g[3 * a + b] = T(0.5) * (gb[3 * a + b] + gb[3 * b + a]);
  const T s = id * T(1.0 / (8.0 * HH_PI));
  T og = 0, d4[9];
  RowSum<T> rb;
  for (int m = 0; m < 9; ++m) {
    og += o[m] * g[m];
    d4[m] = s * g[m];
    rb.put(m, d4[m]);
  }
  rb.flush(&dth[OFF_B4], 9);
  for (int k = 0; k < MLP_H; ++k) {
    T acc = 0;
    for (int m = 0; m < 9; ++m) acc += P[OFF_W4 + MLP_H * m + k] * d4[m];
    dl[k] = acc * (T(1) - h3[k] * h3[k]);   // delta_3
  }
  for (int m = 0; m < 9; ++m) {
    RowSum<T> rw;
    for (int k = 0; k < MLP_H; ++k) rw.put(k, d4[m] * h3[k]);
    rw.flush(&dth[OFF_W4 + MLP_H * m], MLP_H);
  }
  // layer 3: delta_3 -> dW3, db3, delta_2 (into h3, no longer needed)
  for (int k = 0; k < MLP_H; ++k) h3[k] = 0;
  for (int a = 0; a < MLP_H; ++a) {
    const T da = dl[a];
    rb.put(a, da);
    RowSum<T> rw;
    for (int k = 0; k < MLP_H; ++k) {
      rw.put(k, da * h2[k]);
      h3[k] += P[OFF_W3 + MLP_H * a + k] * da;
    }
    rw.flush(&dth[OFF_W3 + MLP_H * a], MLP_H);
  }
  rb.flush(&dth[OFF_B3], MLP_H);
  for (int k = 0; k < MLP_H; ++k) dl[k] = h3[k] * (T(1) - h2[k] * h2[k]);   // delta_2
  for (int k = 0; k < MLP_H; ++k) h3[k] = 0;
  for (int a = 0; a < MLP_H; ++a) {
    const T da = dl[a];
    rb.put(a, da);
    RowSum<T> rw;
    for (int k = 0; k < MLP_H; ++k) {
      rw.put(k, da * h1[k]);
      h3[k] += P[OFF_W2 + MLP_H * a + k] * da;
    }
    rw.flush(&dth[OFF_W2 + MLP_H * a], MLP_H);
  }
  rb.flush(&dth[OFF_B2], MLP_H);
  T gv0 = 0, gv1 = 0, gv2 = 0;
  RowSum<T> r0, r1, r2;
  for (int k = 0; k < MLP_H; ++k) {
    const T d1 = h3[k] * (T(1) - h1[k] * h1[k]);   // delta_1
    rb.put(k, d1);
    r0.put(k, d1 * v0);
    r1.put(k, d1 * v1);
    r2.put(k, d1 * v2);
    gv0 += P[OFF_W1 + 3 * k] * d1;
    gv1 += P[OFF_W1 + 3 * k + 1] * d1;
    gv2 += P[OFF_W1 + 3 * k + 2] * d1;
  }
  rb.flush(&dth[OFF_B1], MLP_H);
  r0.flush(&dth[OFF_W1], MLP_H, 3);
  r1.flush(&dth[OFF_W1 + 1], MLP_H, 3);
  r2.flush(&dth[OFF_W1 + 2], MLP_H, 3);
  if (dir) {
    const T vg = v0 * gv0 + v1 * gv1 + v2 * gv2;
    gv0 = (gv0 - v0 * vg) * id;
    gv1 = (gv1 - v1 * vg) * id;
    gv2 = (gv2 - v2 * vg) * id;
  }
  const T c3 = og * id * id * id * T(1.0 / (8.0 * HH_PI));
  dr[0] = gv0 - rx * c3;
  dr[1] = gv1 - ry * c3;
  dr[2] = gv2 - rz * c3;
}

__device__ __forceinline__ void atomic_add3(double* p, double a, double b, double c) {
  atomicAdd(p, a);
  atomicAdd(p + 1, b);
  atomicAdd(p + 2, c);
}

template <class T>
__device__ __forceinline__ void stage_params(T* wl, double* dth, const T* w) {
  for (int i = threadIdx.x; i < MLP_NP; i += TB) {
    wl[i] = w[i];
    dth[i] = 0;
  }
}

// adds (launches in turn may share a slot; slots start at zero)
__device__ __forceinline__ void flush_params(const double* dth, double* part) {
  for (int i = threadIdx.x; i < MLP_NP; i += TB) part[(int64_t)blockIdx.x * MLP_NP + i] += dth[i];
}

// Near pairs: one workgroup per target leaf, thread per target i (as the
// forward near field); cotangent of K(x_i - x_j) is w_i F_j^T.
template <class T>
__global__ __launch_bounds__(TB) void k_near_vjp(const int4* __restrict__ nodes,
                                                 const int32_t* __restrict__ leaves,
                                                 const int32_t* __restrict__ near_ptr,
                                                 const int2* __restrict__ H,
                                                 const double* __restrict__ xs,
                                                 const T* __restrict__ Fs, const T* __restrict__ ws,
                                                 const T* __restrict__ wgt, int mode,
                                                 double* __restrict__ dXs, double* __restrict__ part) {
  __shared__ T wl[MLP_NP];
  __shared__ double dth[MLP_NP];
  stage_params(wl, dth, wgt);
  __syncthreads();
  const int leaf = blockIdx.x;
  const int4 nt = nodes[leaves[leaf]];
  const int w64 = threadIdx.x & ~63;   // first thread of this wave
  for (int ib = nt.x; ib < nt.y; ib += TB) {
    if (ib + w64 >= nt.y) continue;   // the whole wave past the leaf (uniform)
    // every lane of the wave runs every pair (mlp_vjp reduces across the
    // wave); a lane past the leaf or on its own particle adds nothing
    const int i = ib + threadIdx.x;
    const bool vi = i < nt.y;
    const int ii = vi ? i : nt.x;
    const double x0 = xs[3 * (int64_t)ii], x1 = xs[3 * (int64_t)ii + 1], x2 = xs[3 * (int64_t)ii + 2];
    const T w0 = ws[3 * (int64_t)ii], w1 = ws[3 * (int64_t)ii + 1], w2 = ws[3 * (int64_t)ii + 2];
    double a0 = 0, a1 = 0, a2 = 0;
    for (int p = near_ptr[leaf]; p < near_ptr[leaf + 1]; ++p) {
      const int4 ns = nodes[H[p].y];
      for (int j = ns.x; j < ns.y; ++j) {
        const bool ok = vi && j != i;
        const T f0 = Fs[3 * (int64_t)j], f1 = Fs[3 * (int64_t)j + 1], f2 = Fs[3 * (int64_t)j + 2];
        const T u0 = ok ? w0 : T(0), u1 = ok ? w1 : T(0), u2 = ok ? w2 : T(0);
        T gb[9] = {u0 * f0, u0 * f1, u0 * f2, u1 * f0, u1 * f1, u1 * f2, u2 * f0, u2 * f1, u2 * f2};
        T dr[3];
        const T rx = ok ? (T)(x0 - xs[3 * (int64_t)j]) : T(1);
        const T ry = ok ? (T)(x1 - xs[3 * (int64_t)j + 1]) : T(0);
        const T rz = ok ? (T)(x2 - xs[3 * (int64_t)j + 2]) : T(0);
        mlp_vjp<T>(wl, mode, rx, ry, rz, gb, dth, dr);
        if (ok) {
          a0 += dr[0]; a1 += dr[1]; a2 += dr[2];
          atomic_add3(dXs + 3 * (int64_t)j, -(double)dr[0], -(double)dr[1], -(double)dr[2]);
        }
      }
    }
    if (vi) atomic_add3(dXs + 3 * (int64_t)i, a0, a1, a2);
  }
  __syncthreads();
  flush_params(dth, part);
}

// Reverse of the ACA recursion of one admissible block per workgroup, for
// the blocks [b0, b1). Writes the cotangents of the sampled columns and rows
// of block b into the cotangent pool at goff[b] (term k: 9 (c + q) values,
// column then row), and adds Q^T (C^T w) to dFs.
template <class T>
__global__ __launch_bounds__(TB) void k_aca_adjoint(
    const int2* __restrict__ G, int64_t b0, int64_t b1, const int4* __restrict__ nodes,
    const int32_t* __restrict__ rank, const int32_t* __restrict__ flag,
    const int32_t* __restrict__ piv, const int64_t* __restrict__ fptr,
    const int64_t* __restrict__ goff, const T* __restrict__ pool, T* __restrict__ gpool,
    const T* __restrict__ Fs, const T* __restrict__ ws, double* __restrict__ dFs) {
  __shared__ double s_t[LMAX_CAP][3], s_tb[LMAX_CAP][3];
  __shared__ double red[TB / 64][9];
  __shared__ double s_M[9];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // block-wide sum of 9 doubles, result in s_M (all threads may read after)
  auto reduce9 = [&](double (&v)[9]) {
    for (int e = 0; e < 9; ++e) v[e] = wave_sum(v[e]);
    __syncthreads();
    if (lane == 0)
      for (int e = 0; e < 9; ++e) red[wv][e] = v[e];
    __syncthreads();
    if (threadIdx.x < 9) {
      double a = 0;
      for (int w = 0; w < TB / 64; ++w) a += red[w][threadIdx.x];
      s_M[threadIdx.x] = a;
    }
    __syncthreads();
  };
  for (int64_t b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    if (flag[b] || rank[b] == 0) continue;
    const int2 g = G[b];
    const int4 nt = nodes[g.x], ns = nodes[g.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x, l = rank[b];
    const int32_t* pi = piv + b * 2 * LMAX_CAP;
    const int32_t* pj = pi + LMAX_CAP;
    auto Cp = [&](int k) { return pool + fptr[b * LMAX_CAP + k]; };
    auto Qp = [&](int k) { return pool + fptr[b * LMAX_CAP + k] + 9 * (int64_t)c; };
    auto Cb = [&](int k) { return gpool + goff[b] + 9 * (int64_t)k * (c + q); };
    auto Qb = [&](int k) { return gpool + goff[b] + 9 * (int64_t)k * (c + q) + 9 * (int64_t)c; };
    // t_k = sum_j q_k(j) F_j, tb_k = sum_i c_k(i)^T w_i
    for (int k = 0; k < l; ++k) {
      double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int j = threadIdx.x; j < q; j += TB) {
        const T* e = Qp(k) + 9 * (int64_t)j;
        const T* f = Fs + 3 * ((int64_t)ns.x + j);
        for (int a = 0; a < 3; ++a)
          v[a] += (double)e[3 * a] * f[0] + (double)e[3 * a + 1] * f[1] + (double)e[3 * a + 2] * f[2];
      }
      for (int i = threadIdx.x; i < c; i += TB) {
        const T* e = Cp(k) + 9 * (int64_t)i;
        const T* w = ws + 3 * ((int64_t)nt.x + i);
        for (int a = 0; a < 3; ++a)
          v[3 + a] += (double)e[a] * w[0] + (double)e[3 + a] * w[1] + (double)e[6 + a] * w[2];
      }
      reduce9(v);
      if (threadIdx.x < 3) {
        s_t[k][threadIdx.x] = s_M[threadIdx.x];
        s_tb[k][threadIdx.x] = s_M[3 + threadIdx.x];
      }
    }
    __syncthreads();
    // initial cotangents and dF_sigma += sum_k q_k(j)^T tb_k
    for (int i = threadIdx.x; i < c; i += TB) {
      const T* w = ws + 3 * ((int64_t)nt.x + i);
      for (int k = 0; k < l; ++k)
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) Cb(k)[9 * (int64_t)i + 3 * a + bb] = (T)(w[a] * s_t[k][bb]);
    }
    for (int j = threadIdx.x; j < q; j += TB) {
      const T* f = Fs + 3 * ((int64_t)ns.x + j);
      double d0 = 0, d1 = 0, d2 = 0;
      for (int k = 0; k < l; ++k) {
        const T* e = Qp(k) + 9 * (int64_t)j;
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) Qb(k)[9 * (int64_t)j + 3 * a + bb] = (T)(s_tb[k][a] * f[bb]);
        d0 += (double)e[0] * s_tb[k][0] + (double)e[3] * s_tb[k][1] + (double)e[6] * s_tb[k][2];
        d1 += (double)e[1] * s_tb[k][0] + (double)e[4] * s_tb[k][1] + (double)e[7] * s_tb[k][2];
        d2 += (double)e[2] * s_tb[k][0] + (double)e[5] * s_tb[k][1] + (double)e[8] * s_tb[k][2];
      }
      atomic_add3(dFs + 3 * ((int64_t)ns.x + j), d0, d1, d2);
    }
    __syncthreads();
    for (int k = l - 1; k >= 0; --k) {
      const int ik = pi[k], jk = pj[k];
      // q_k = G(i_k, :) - sum_{m<k} c_m(i_k) q_m: the row cotangent stays in
      // place; c_m(i_k) -= sum_j qb_k(j) q_m(j)^T, qb_m(j) -= c_m(i_k)^T qb_k(j)
      for (int m = 0; m < k; ++m) {
        double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = threadIdx.x; j < q; j += TB) {
          const T* x = Qb(k) + 9 * (int64_t)j;
          const T* y = Qp(m) + 9 * (int64_t)j;
          for (int a = 0; a < 3; ++a)
            for (int cc = 0; cc < 3; ++cc)
              v[3 * a + cc] += (double)x[3 * a] * y[3 * cc] + (double)x[3 * a + 1] * y[3 * cc + 1] +
                               (double)x[3 * a + 2] * y[3 * cc + 2];
        }
        reduce9(v);
        if (threadIdx.x < 9) Cb(m)[9 * (int64_t)ik + threadIdx.x] -= (T)s_M[threadIdx.x];
        const T* cm = Cp(m) + 9 * (int64_t)ik;
        for (int j = threadIdx.x; j < q; j += TB) {
          const T* x = Qb(k) + 9 * (int64_t)j;
          T* y = Qb(m) + 9 * (int64_t)j;
          for (int a = 0; a < 3; ++a)
            for (int cc = 0; cc < 3; ++cc)
              y[3 * a + cc] -= cm[a] * x[cc] + cm[3 + a] * x[3 + cc] + cm[6 + a] * x[6 + cc];
        }
        __syncthreads();
      }
      // c_k = a_k P^-1, P = q_k(j_k), a_k(i) = c_k(i) P:
      //   ab(i) = cb_k(i) P^-T, ab(i_k) -= P^-T S P^-T, S = sum_i a_k(i)^T cb_k(i)
      double Pm[9], Pi[9];
      {
        const T* P = Cp(k) + 9 * (int64_t)(c + q);   // the pivot entry the forward used
        for (int e = 0; e < 9; ++e) Pm[e] = P[e];
        double det = Pm[0] * (Pm[4] * Pm[8] - Pm[5] * Pm[7]) - Pm[1] * (Pm[3] * Pm[8] - Pm[5] * Pm[6]) +
                     Pm[2] * (Pm[3] * Pm[7] - Pm[4] * Pm[6]);
        double idt = 1.0 / det;
        Pi[0] = (Pm[4] * Pm[8] - Pm[5] * Pm[7]) * idt;
        Pi[1] = (Pm[2] * Pm[7] - Pm[1] * Pm[8]) * idt;
        Pi[2] = (Pm[1] * Pm[5] - Pm[2] * Pm[4]) * idt;
        Pi[3] = (Pm[5] * Pm[6] - Pm[3] * Pm[8]) * idt;
        Pi[4] = (Pm[0] * Pm[8] - Pm[2] * Pm[6]) * idt;
        Pi[5] = (Pm[2] * Pm[3] - Pm[0] * Pm[5]) * idt;
        Pi[6] = (Pm[3] * Pm[7] - Pm[4] * Pm[6]) * idt;
        Pi[7] = (Pm[1] * Pm[6] - Pm[0] * Pm[7]) * idt;
        Pi[8] = (Pm[0] * Pm[4] - Pm[1] * Pm[3]) * idt;
      }
      {
        double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = threadIdx.x; i < c; i += TB) {
          const T* cc_ = Cp(k) + 9 * (int64_t)i;
          const T* cb = Cb(k) + 9 * (int64_t)i;
          double A[9];   // a_k(i) = c_k(i) P
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb)
              A[3 * a + bb] = (double)cc_[3 * a] * Pm[bb] + (double)cc_[3 * a + 1] * Pm[3 + bb] +
                              (double)cc_[3 * a + 2] * Pm[6 + bb];
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb)
              v[3 * a + bb] += A[a] * cb[bb] + A[3 + a] * cb[3 + bb] + A[6 + a] * cb[6 + bb];
        }
        reduce9(v);
      }
      double Sm[9];
      for (int e = 0; e < 9; ++e) Sm[e] = s_M[e];
      __syncthreads();
      // corr = P^-T S P^-T
      double T1[9], corr[9];
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb)
          T1[3 * a + bb] = Pi[a] * Sm[bb] + Pi[3 + a] * Sm[3 + bb] + Pi[6 + a] * Sm[6 + bb];
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb)
          corr[3 * a + bb] = T1[3 * a] * Pi[3 * bb] + T1[3 * a + 1] * Pi[3 * bb + 1] + T1[3 * a + 2] * Pi[3 * bb + 2];
      for (int i = threadIdx.x; i < c; i += TB) {
        T* cb = Cb(k) + 9 * (int64_t)i;
        double o[9];
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb)   // cb P^-T
            o[3 * a + bb] = (double)cb[3 * a] * Pi[3 * bb] + (double)cb[3 * a + 1] * Pi[3 * bb + 1] +
                            (double)cb[3 * a + 2] * Pi[3 * bb + 2];
        if (i == ik)
          for (int e = 0; e < 9; ++e) o[e] -= corr[e];
        for (int e = 0; e < 9; ++e) cb[e] = (T)o[e];   // column cotangent of step k
      }
      __syncthreads();
      // a_k = G(:, j_k) - sum_{m<k} c_m q_m(j_k):
      //   cb_m(i) -= ab(i) q_m(j_k)^T,  qb_m(j_k) -= sum_i c_m(i)^T ab(i)
      for (int m = 0; m < k; ++m) {
        const T* qm = Qp(m) + 9 * (int64_t)jk;
        double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = threadIdx.x; i < c; i += TB) {
          const T* ab = Cb(k) + 9 * (int64_t)i;
          const T* cm = Cp(m) + 9 * (int64_t)i;
          T* cbm = Cb(m) + 9 * (int64_t)i;
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) {
              cbm[3 * a + bb] -= ab[3 * a] * qm[3 * bb] + ab[3 * a + 1] * qm[3 * bb + 1] +
                                 ab[3 * a + 2] * qm[3 * bb + 2];
              v[3 * a + bb] += (double)cm[a] * ab[bb] + (double)cm[3 + a] * ab[3 + bb] +
                               (double)cm[6 + a] * ab[6 + bb];
            }
        }
        reduce9(v);
        if (threadIdx.x < 9) Qb(m)[9 * (int64_t)jk + threadIdx.x] -= (T)s_M[threadIdx.x];
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// Back-propagation of the sampled far pairs: workgroup per (block, term k).
template <class T>
__global__ __launch_bounds__(TB) void k_far_vjp(const int2* __restrict__ G, int64_t b0,
                                                int64_t b1, const int4* __restrict__ nodes,
                                                const int32_t* __restrict__ rank,
                                                const int32_t* __restrict__ flag,
                                                const int32_t* __restrict__ piv,
                                                const int64_t* __restrict__ goff,
                                                const T* __restrict__ gpool,
                                                const double* __restrict__ xs,
                                                const T* __restrict__ wgt, int mode,
                                                double* __restrict__ dXs,
                                                double* __restrict__ part) {
  __shared__ T wl[MLP_NP];
  __shared__ double dth[MLP_NP];
  stage_params(wl, dth, wgt);
  __syncthreads();
  for (int64_t b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    if (flag[b] || rank[b] == 0) continue;
    const int2 g = G[b];
    const int4 nt = nodes[g.x], ns = nodes[g.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x, l = rank[b];
    for (int k = 0; k < l; ++k) {
      const int ik = piv[b * 2 * LMAX_CAP + k], jk = piv[b * 2 * LMAX_CAP + LMAX_CAP + k];
      const T* gc = gpool + goff[b] + 9 * (int64_t)k * (c + q);
      const T* gr = gc + 9 * (int64_t)c;
      const int w64 = threadIdx.x & ~63;
      for (int t0 = 0; t0 < c + q; t0 += TB) {
        if (t0 + w64 >= c + q) continue;   // the whole wave past the samples (uniform)
        const int t = t0 + threadIdx.x;
        const bool ok = t < c + q;         // lanes past the samples add nothing
        const int tt = ok ? t : 0;
        const bool colp = tt < c;
        const int i = colp ? nt.x + tt : nt.x + ik;
        const int j = colp ? ns.x + jk : ns.x + (tt - c);
        const T* gsrc = colp ? gc + 9 * (int64_t)tt : gr + 9 * (int64_t)(tt - c);
        T gb[9];
        for (int e = 0; e < 9; ++e) gb[e] = ok ? gsrc[e] : T(0);
        T dr[3];
        mlp_vjp<T>(wl, mode, (T)(xs[3 * (int64_t)i] - xs[3 * (int64_t)j]),
                   (T)(xs[3 * (int64_t)i + 1] - xs[3 * (int64_t)j + 1]),
                   (T)(xs[3 * (int64_t)i + 2] - xs[3 * (int64_t)j + 2]), gb, dth, dr);
        if (ok) {
          atomic_add3(dXs + 3 * (int64_t)i, dr[0], dr[1], dr[2]);
          atomic_add3(dXs + 3 * (int64_t)j, -(double)dr[0], -(double)dr[1], -(double)dr[2]);
        }
      }
    }
  }
  __syncthreads();
  flush_params(dth, part);
}

// Admissible blocks that fell back to dense evaluation: their transposed
// product (into farT) and their pair cotangents w_i F_j^T. Thread per row.
template <class T, int KIND>
__global__ __launch_bounds__(TB) void k_fallback_bwd(const int2* __restrict__ G, int64_t nG,
                                                     const int4* __restrict__ nodes,
                                                     const int32_t* __restrict__ flag,
                                                     const double* __restrict__ xs,
                                                     const T* __restrict__ Fs,
                                                     const T* __restrict__ ws, KParams kp,
                                                     int want_grad, double* __restrict__ farT,
                                                     double* __restrict__ dXs,
                                                     double* __restrict__ part) {
  __shared__ T wl[KIND == KIND_MLP ? MLP_NP : 1];
  __shared__ double dth[KIND == KIND_MLP ? MLP_NP : 1];
  if (KIND == KIND_MLP) stage_params(wl, dth, (const T*)kp.w);
  __syncthreads();
  for (int64_t b = blockIdx.x; b < nG; b += gridDim.x) {
    if (!flag[b]) continue;
    const int4 nt = nodes[G[b].x], ns = nodes[G[b].y];
    const int w64 = threadIdx.x & ~63;
    for (int ib = nt.x; ib < nt.y; ib += TB) {
      if (ib + w64 >= nt.y) continue;   // the whole wave past the block (uniform)
      const int i = ib + threadIdx.x;
      const bool vi = i < nt.y;          // lanes past the block add nothing
      const int ii = vi ? i : nt.x;
      const double x0 = xs[3 * (int64_t)ii], x1 = xs[3 * (int64_t)ii + 1], x2 = xs[3 * (int64_t)ii + 2];
      const T w0 = vi ? ws[3 * (int64_t)ii] : T(0), w1 = vi ? ws[3 * (int64_t)ii + 1] : T(0),
              w2 = vi ? ws[3 * (int64_t)ii + 2] : T(0);
      double a0 = 0, a1 = 0, a2 = 0;
      for (int j = ns.x; j < ns.y; ++j) {
        const T rx = (T)(x0 - xs[3 * (int64_t)j]), ry = (T)(x1 - xs[3 * (int64_t)j + 1]),
                rz = (T)(x2 - xs[3 * (int64_t)j + 2]);
        T K[9];
        kernel_entry<T>(kp, wl, rx, ry, rz, K);
        if (vi)
          atomic_add3(farT + 3 * (int64_t)j, (double)(K[0] * w0 + K[3] * w1 + K[6] * w2),
                      (double)(K[1] * w0 + K[4] * w1 + K[7] * w2),
                      (double)(K[2] * w0 + K[5] * w1 + K[8] * w2));
        if (KIND == KIND_MLP && want_grad) {
          const T f0 = Fs[3 * (int64_t)j], f1 = Fs[3 * (int64_t)j + 1], f2 = Fs[3 * (int64_t)j + 2];
          T gb[9] = {w0 * f0, w0 * f1, w0 * f2, w1 * f0, w1 * f1, w1 * f2, w2 * f0, w2 * f1, w2 * f2};
          T dr[3];
          mlp_vjp<T>(wl, kp.input_mode, rx, ry, rz, gb, dth, dr);
          if (vi) {
            a0 += dr[0]; a1 += dr[1]; a2 += dr[2];
            atomic_add3(dXs + 3 * (int64_t)j, -(double)dr[0], -(double)dr[1], -(double)dr[2]);
          }
        }
      }
      if (KIND == KIND_MLP && want_grad && vi) atomic_add3(dXs + 3 * (int64_t)i, a0, a1, a2);
    }
  }
  if (KIND == KIND_MLP) {
    __syncthreads();
    flush_params(dth, part);
  }
}

// dparams[i] += sum over workgroup partials, fixed order.
__global__ __launch_bounds__(TB) void k_param_reduce(const double* __restrict__ part, int nparts,
                                                     double* __restrict__ out) {
  int i = blockIdx.x * TB + threadIdx.x;
  if (i >= MLP_NP) return;
  double s = 0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * MLP_NP + i];
  out[i] += s;
}

template <class T>
__global__ __launch_bounds__(TB) void k_gather3(const T* __restrict__ v,
                                                const int32_t* __restrict__ perm, int64_t n,
                                                T* __restrict__ vs) {
  int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  int64_t o = perm[s];
  vs[3 * s] = v[3 * o];
  vs[3 * s + 1] = v[3 * o + 1];
  vs[3 * s + 2] = v[3 * o + 2];
}

// out[perm[s]] = (a1 * ws[s] + near_T[s] + far_T[s]) or dX scatter
template <class T>
__global__ __launch_bounds__(TB) void k_scatter_dF(const T* __restrict__ ws,
                                                   const T* __restrict__ nearT,
                                                   const double* __restrict__ farT,
                                                   const int32_t* __restrict__ perm, int64_t n,
                                                   double a1, T* __restrict__ dF) {
  int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  int64_t o = perm[s];
  for (int d = 0; d < 3; ++d)
    dF[3 * o + d] = (T)((a1 * (double)ws[3 * s + d] + (double)nearT[3 * s + d]) + farT[3 * s + d]);
}

__global__ __launch_bounds__(TB) void k_scatter_dX(const double* __restrict__ dXs,
                                                   const int32_t* __restrict__ perm, int64_t n,
                                                   double* __restrict__ dX) {
  int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (s >= n) return;
  int64_t o = perm[s];
  for (int d = 0; d < 3; ++d) dX[3 * o + d] = dXs[3 * s + d];
}

template <class T>
void backward_t(hh_ctx ctx, hh_tree t, hh_part p, hh_lowrank lr, hh_kernel k, const void* F,
                const void* dU, void* dF, double* dX, double* dparams) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  DevBuf Fs, ws, nearT, farT, dXs, gpool, part;
  Fs.alloc(st, 3 * n * sizeof(T));
  ws.alloc(st, 3 * n * sizeof(T));
  hipLaunchKernelGGL((k_gather3<T>), dim3(nblk(n)), dim3(TB), 0, st, (const T*)F,
                     t->perm.as<int32_t>(), n, Fs.as<T>());
  hipLaunchKernelGGL((k_gather3<T>), dim3(nblk(n)), dim3(TB), 0, st, (const T*)dU,
                     t->perm.as<int32_t>(), n, ws.as<T>());
  farT.alloc(st, 3 * n * sizeof(double));
  HIP_OK(hipMemsetAsync(farT.p, 0, 3 * n * sizeof(double), st));
  const bool mlp = k->kind == KIND_MLP && (dX || dparams);
  const int64_t nG = p->nG;
  // cotangent pool: the blocks in chunks of consecutive blocks whose
  // cotangents (rank 9 (c + q) values each) fit GPOOL_CHUNK elements (a block
  // larger than that is a chunk of its own); each chunk's adjoint is
  // followed by the back-propagation of its sampled pairs
  std::vector<int64_t> bounds(1, 0);
  int64_t chunk_max = 1;
  DevBuf goff;
  if (nG > 0 && (dF || mlp)) {
    std::vector<int32_t> cs, qs, rk(nG), fl(nG);
    block_sizes(ctx, t, p, cs, qs);
    read_bytes(ctx, rk.data(), lr->rank.p, nG * sizeof(int32_t));
    read_bytes(ctx, fl.data(), lr->flag.p, nG * sizeof(int32_t));
    std::vector<int64_t> off(nG);
    int64_t cur = 0;
    for (int64_t b = 0; b < nG; ++b) {
      const int64_t need = fl[b] ? 0 : 9 * (int64_t)rk[b] * ((int64_t)cs[b] + qs[b]);
      if (cur > 0 && cur + need > GPOOL_CHUNK) {
        bounds.push_back(b);
        chunk_max = std::max(chunk_max, cur);
        cur = 0;
      }
      off[b] = cur;
      cur += need;
    }
    chunk_max = std::max(chunk_max, cur);
    bounds.push_back(nG);
    goff.alloc(st, nG * sizeof(int64_t));
    HIP_OK(hipMemcpyAsync(goff.p, off.data(), nG * sizeof(int64_t), hipMemcpyHostToDevice, st));
    gpool.alloc(st, chunk_max * sizeof(T));
  }
  const int gfb = (int)std::min<int64_t>(std::max<int64_t>(nG, 1), 256);
  if (mlp) {
    dXs.alloc(st, 3 * n * sizeof(double));
    HIP_OK(hipMemsetAsync(dXs.p, 0, 3 * n * sizeof(double), st));
  }
  // FP32: near and sampled pairs on the FP32 MFMA tile (persistent waves, one
  // dtheta slot per wave); FP64: the VALU kernels (one slot per workgroup)
  constexpr bool mf = sizeof(T) == 4;
  const int gnear = mf ? (int)vjp_f32_waves(ctx) : (int)t->n_leaves;
  const int gfar = mf ? (int)vjp_f32_waves(ctx)
                      : (int)std::min<int64_t>(std::max<int64_t>(nG, 1), 2048);
  const int nparts = gnear + gfar + gfb;   // dtheta partial slots: near, far, fallback
  if (mlp) {
    part.alloc(st, (int64_t)nparts * MLP_NP * sizeof(double));
    HIP_OK(hipMemsetAsync(part.p, 0, (int64_t)nparts * MLP_NP * sizeof(double), st));
  }
  const T* wgt = (const T*)(sizeof(T) == 8 ? k->p64.p : k->p32.p);
  for (size_t c = 0; c + 1 < bounds.size(); ++c) {
    const int64_t b0 = bounds[c], b1 = bounds[c + 1];
    if (b1 <= b0) continue;
    const unsigned grid = (unsigned)std::min<int64_t>(b1 - b0, 4096);
    hipLaunchKernelGGL((k_aca_adjoint<T>), dim3(grid), dim3(TB), 0, st, p->G.as<int2>(), b0, b1,
                       t->nodes.as<int4>(), lr->rank.as<int32_t>(), lr->flag.as<int32_t>(),
                       lr->piv.as<int32_t>(), lr->fptr.as<int64_t>(), goff.as<int64_t>(),
                       lr->pool.as<T>(), gpool.as<T>(), Fs.as<T>(), ws.as<T>(),
                       farT.as<double>());
    if (mlp && mf)
      launch_far_vjp_f32(ctx, t, p, lr, k, b0, b1, goff.as<int64_t>(), gpool.as<float>(),
                         dXs.as<double>(), part.as<double>() + (int64_t)gnear * MLP_NP);
    else if (mlp)
      hipLaunchKernelGGL((k_far_vjp<T>), dim3(gfar), dim3(TB), 0, st, p->G.as<int2>(), b0, b1,
                         t->nodes.as<int4>(), lr->rank.as<int32_t>(), lr->flag.as<int32_t>(),
                         lr->piv.as<int32_t>(), goff.as<int64_t>(), gpool.as<T>(),
                         t->xs.as<double>(), wgt, k->input_mode, dXs.as<double>(),
                         part.as<double>() + (int64_t)gnear * MLP_NP);
    HIP_OK(hipGetLastError());
  }
  if (lr->n_fallback > 0 && (dF || mlp)) {
    const KParams kp = make_kparams(k, sizeof(T) == 8);
    double* fbpart = mlp ? part.as<double>() + (int64_t)(gnear + gfar) * MLP_NP : nullptr;
    if (k->kind == KIND_MLP)
      hipLaunchKernelGGL((k_fallback_bwd<T, KIND_MLP>), dim3(gfb), dim3(TB), 0, st,
                         p->G.as<int2>(), nG, t->nodes.as<int4>(), lr->flag.as<int32_t>(),
                         t->xs.as<double>(), Fs.as<T>(), ws.as<T>(), kp, mlp ? 1 : 0,
                         farT.as<double>(), mlp ? dXs.as<double>() : nullptr, fbpart);
    else
      hipLaunchKernelGGL((k_fallback_bwd<T, KIND_RPY>), dim3(gfb), dim3(TB), 0, st,
                         p->G.as<int2>(), nG, t->nodes.as<int4>(), lr->flag.as<int32_t>(),
                         t->xs.as<double>(), Fs.as<T>(), ws.as<T>(), kp, 0, farT.as<double>(),
                         nullptr, nullptr);
    HIP_OK(hipGetLastError());
  }
  if (dF) {
    nearT.alloc(st, 3 * n * sizeof(T));
    launch_near_neg(ctx, t, p, k, sizeof(T) == 8 ? HH_FP64 : HH_FP32, ws.p, nearT.p);
    hipLaunchKernelGGL((k_scatter_dF<T>), dim3(nblk(n)), dim3(TB), 0, st, ws.as<T>(),
                       nearT.as<T>(), farT.as<double>(), t->perm.as<int32_t>(), n, k->alpha1,
                       (T*)dF);
  }
  if (mlp) {
    if constexpr (mf)
      launch_near_vjp_f32(ctx, t, p, k, Fs.as<float>(), ws.as<float>(), dXs.as<double>(),
                          part.as<double>());
    else
      hipLaunchKernelGGL((k_near_vjp<T>), dim3(gnear), dim3(TB), 0, st, t->nodes.as<int4>(),
                         t->leaves.as<int32_t>(), p->near_ptr.as<int32_t>(), p->H.as<int2>(),
                         t->xs.as<double>(), Fs.as<T>(), ws.as<T>(), wgt, k->input_mode,
                         dXs.as<double>(), part.as<double>());
    HIP_OK(hipGetLastError());
    if (dX)
      hipLaunchKernelGGL(k_scatter_dX, dim3(nblk(n)), dim3(TB), 0, st, dXs.as<double>(),
                         t->perm.as<int32_t>(), n, dX);
    if (dparams)
      hipLaunchKernelGGL(k_param_reduce, dim3((MLP_NP + TB - 1) / TB), dim3(TB), 0, st,
                         part.as<double>(), nparts, dparams);
    HIP_OK(hipGetLastError());
  }
}

}  // namespace

extern "C" hh_status hh_matvec_backward(hh_ctx ctx, hh_tree tree, hh_part part, hh_lowrank lr,
                                        hh_kernel kern, hh_precision prec, const void* F,
                                        const void* dU, void* dF, double* dX, double* dparams) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(tree && part && lr && kern && F && dU, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(part->tree == tree && lr->part == part && lr->kern == kern, HH_ERR_INVALID_ARG,
             "handles do not belong together");
  HH_REQUIRE(lr->prec == prec, HH_ERR_INVALID_ARG, "precision differs from the ACA build");
  HH_REQUIRE(prec == HH_FP64 || prec == HH_FP32, HH_ERR_INVALID_ARG,
             "the backward is available in FP64 and FP32");
  HH_REQUIRE(!lr->streamed, HH_ERR_INVALID_ARG,
             "the backward needs stored factors (raise the budget with hh_ctx_set_budget)");
  HH_REQUIRE(!(dX || dparams) || kern->kind == KIND_MLP, HH_ERR_INVALID_ARG,
             "dX and dparams need the MLP kernel");
  HH_REQUIRE(kern->kind != KIND_RPY6, HH_ERR_INVALID_ARG,
             "the backward takes the 3N kernels (the 6N matrix is symmetric: dF = M dU)");
  PhaseTimer timer(ctx, HH_PHASE_BACKWARD);
  if (prec == HH_FP64)
    backward_t<double>(ctx, tree, part, lr, kern, F, dU, dF, dX, dparams);
  else
    backward_t<float>(ctx, tree, part, lr, kern, F, dU, dF, dX, dparams);
  HH_API_END(ctx)
}
