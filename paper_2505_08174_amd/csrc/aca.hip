// Adaptive cross approximation with 3x3 entries (Algorithm 2, Eqs. (8)-(10)).
//
// One workgroup (256 threads) per admissible block, fetched from a global
// work counter (dynamic load balance; the results do not depend on the
// order). The rank loop runs inside the workgroup:
//   column j_k: a(i) = K(x_i - y_j) - sum_{m<k} c_m(i) q_m(j)
//   i_k = argmax over unused rows of ||a(i)||_F^2, lowest index on ties
//   c_k(i) = a(i) P^-1, P = a(i_k)
//   row i_k:  q_k(j) = K(x_ik - y_j) - sum_{m<k} c_m(i_k) q_m(j)
//   j_{k+1} = argmax over unused columns of ||q_k(j)||_F^2
//   nu^2 = tr(A_kk B_kk), lambda^2 += nu^2 + 2 sum_{m<k} tr(A_mk B_km)
//   with A_mk = sum_i c_m(i)^T c_k(i), B_km = sum_j q_k(j) q_m(j)^T
//   stop when nu^2 <= eps^2 lambda^2 or after min(c, q) terms.
// Pivot magnitude: squared Frobenius norm in the FP64 form (Algorithm 2);
// |det| of the 3x3 entry in the FP32 and BF16 forms (the magnitude the text
// around Eq. (9) names), which avoids nearly singular pivots whose inverse
// would amplify single-precision rounding in c_k = a P^-1.
// Guards: a residual column with ||a||^2 <= 1e-30 lambda^2 ends as converged
// without a new term; |det P| <= 1e-14 ||P||_F^3 ends with a dense fallback;
// l_max terms without convergence end with a dense fallback.
// Factors c_k (c entries) and q_k (q entries), 9 values each, are stored
// contiguously per step in a pool; each step bump-allocates 9 (c + q) values.
// Row and column samples are evaluated with the VALU kernel, in the working
// type T; norms, pivots and Gram sums in NT.
#include "devmath.h"
#include "internal.h"
#include "mlp_mfma.h"

namespace {

constexpr int ACA_T = 256;
constexpr int NW = ACA_T / 64;
constexpr int GCH = 8;   // Gram matrices reduced per LDS round

template <class T>
struct AcaArgs {
  const int2* G;
  int64_t nG;
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
  unsigned long long* pool_top;
  int* overflow;
  int* work;         // dynamic block counter
  int64_t b0, b1;    // block range of this launch
  // fused apply (streamed mode): Fs != nullptr
  const T* Fs;       // sorted forces
  double* ublk;      // per-block output rows [c][3], at uoff[b] - uoff[b0]
  const int64_t* uoff;
  const uint4* frags;   // BF16 MFMA weight fragments (MF kernels)
  int det_pivot;        // pivot magnitude |det| (else squared Frobenius norm)
};

template <class NT, class T>
__device__ __forceinline__ NT det3(const T* K) {
  return fabs((NT)K[0] * ((NT)K[4] * (NT)K[8] - (NT)K[5] * (NT)K[7]) -
              (NT)K[1] * ((NT)K[3] * (NT)K[8] - (NT)K[5] * (NT)K[6]) +
              (NT)K[2] * ((NT)K[3] * (NT)K[7] - (NT)K[4] * (NT)K[6]));
}

// K(x_i - y_j) from the MFMA MLP tile: symmetrised 3x3 entry of a pair.
__device__ __forceinline__ void mfma_entry(const bf16x8* fr, int mode, double dx, double dy,
                                           double dz, float K[9]) {
  float rx = (float)dx, ry = (float)dy, rz = (float)dz;
  const float rs = hh_rsqrt(rx * rx + ry * ry + rz * rz);
  float o[9];
  if (mode == HH_MLP_INPUT_DIRECTION)
    mlp_tile_bf16<true>(fr, rx * rs, ry * rs, rz * rs, o);
  else
    mlp_tile_bf16<true>(fr, rx, ry, rz, o);
  const float s = rs * (float)(1.0 / (16.0 * HH_PI));
  K[0] = 2.0f * o[0] * s; K[1] = (o[1] + o[3]) * s; K[2] = (o[2] + o[6]) * s;
  K[3] = K[1];            K[4] = 2.0f * o[4] * s;   K[5] = (o[5] + o[7]) * s;
  K[6] = K[2];            K[7] = K[5];              K[8] = 2.0f * o[8] * s;
}

// block-wide argmax (ties to the lowest index), result broadcast to all threads
template <class NT>
__device__ __forceinline__ void block_argmax(NT& v, int& i, NT* sv, int* si) {
  wave_argmax(v, i);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { sv[w] = v; si[w] = i; }
  __syncthreads();
  v = sv[0];
  i = si[0];
  for (int k = 1; k < NW; ++k)
    if (sv[k] > v || (sv[k] == v && si[k] < i)) { v = sv[k]; i = si[k]; }
}

template <class T, class NT, int KIND, bool MF>
__global__ __launch_bounds__(ACA_T) void k_aca(AcaArgs<T> a) {
  // MF: kernel samples from the BF16 MFMA MLP (weights as LDS fragments)
  __shared__ T wl[(KIND == KIND_MLP && !MF) ? MLP_NP : 1];
  __shared__ bf16x8 fr[MF ? FR_TOTAL : 1];
  __shared__ T s_qj[LMAX_CAP * 9];   // q_m(j_k), m < k
  __shared__ T s_ci[LMAX_CAP * 9];   // c_m(i_k), m < k
  __shared__ T s_pinv[9];
  __shared__ int64_t s_off[LMAX_CAP];
  __shared__ int s_pi[LMAX_CAP], s_pj[LMAX_CAP + 1];
  __shared__ NT s_red[NW][GCH][18];
  __shared__ NT s_av[NW];
  __shared__ int s_ai[NW];
  __shared__ NT s_lam2;
  __shared__ double s_t[NW][3];
  __shared__ int s_b, s_stop, s_fb;
  if (MF) {
    stage_frags(fr, a.frags, ACA_T);
  } else if (KIND == KIND_MLP) {
    const T* w = (const T*)a.kp.w;
    for (int i = threadIdx.x; i < MLP_NP; i += ACA_T) wl[i] = w[i];
  }
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_b = atomicAdd(a.work, 1);
    __syncthreads();
    const int64_t b = a.b0 + s_b;
    if (b >= a.b1) break;
    const int2 g = a.G[b];
    const int4 nt = a.nodes[g.x], ns = a.nodes[g.y];
    const int c = nt.y - nt.x, q = ns.y - ns.x;
    const double* xt = a.xs + 3 * (int64_t)nt.x;
    const double* xsr = a.xs + 3 * (int64_t)ns.x;
    const int kmax = min(min(c, q), a.l_max);
    int j = q / 2;
    int rank = 0;
    bool converged = false, fallback = false;
    if (tid == 0) { s_lam2 = 0; s_stop = 0; s_fb = 0; }
    const bool fuse = a.Fs != nullptr;
    double* ub = fuse ? a.ublk + 3 * (a.uoff[b] - a.uoff[a.b0]) : nullptr;
    if (fuse)
      for (int i = tid; i < 3 * c; i += ACA_T) ub[i] = 0.0;
    for (int k = 0; k < kmax; ++k) {
      __syncthreads();
      if (tid == 0) {
        s_pj[k] = j;
        unsigned long long need = 9ull * (unsigned long long)(c + q);
        unsigned long long off = atomicAdd(a.pool_top, need);
        if ((int64_t)(off + need) > a.pool_elems) {
          atomicOr(a.overflow, 1);
          s_fb = 1;
        }
        s_off[k] = (int64_t)off;
        a.fptr[b * LMAX_CAP + k] = (int64_t)off;
      }
      __syncthreads();
      if (s_fb) { fallback = true; break; }
      for (int t = tid; t < 9 * k; t += ACA_T) {
        int m = t / 9, e = t % 9;
        s_qj[t] = a.pool[s_off[m] + 9 * (int64_t)c + 9 * (int64_t)j + e];
      }
      __syncthreads();
      T* Ck = a.pool + s_off[k];
      T* Qk = Ck + 9 * (int64_t)c;
      // residual column j and its largest unused entry
      NT best = -1, bestf = -1;   // selection magnitude, largest squared norm
      int bi = 0x7fffffff;
      NT graw = 0;   // largest raw entry of the column (precision floor)
      const double yj0 = xsr[3 * j], yj1 = xsr[3 * j + 1], yj2 = xsr[3 * j + 2];
      if (MF) {
        // raw column samples in 32-row MFMA tiles, parked in the c_k slot
        for (int t0 = 32 * wv; t0 < c; t0 += 32 * NW) {
          const int i = t0 + (lane & 31);
          const int ii = i < c ? i : t0;
          float K[9];
          mfma_entry(fr, a.kp.input_mode, xt[3 * ii] - yj0, xt[3 * ii + 1] - yj1,
                     xt[3 * ii + 2] - yj2, K);
          if (i < c && lane < 32)
#pragma unroll
            for (int e = 0; e < 9; ++e) Ck[9 * (int64_t)i + e] = (T)K[e];
        }
        __syncthreads();
      }
      for (int i = tid; i < c; i += ACA_T) {
        T K[9];
        if (MF) {
#pragma unroll
          for (int e = 0; e < 9; ++e) K[e] = Ck[9 * (int64_t)i + e];
        } else {
          kernel_entry<T>(a.kp, wl, (T)(xt[3 * i] - yj0), (T)(xt[3 * i + 1] - yj1),
                          (T)(xt[3 * i + 2] - yj2), K);
        }
        if (sizeof(T) == 4) {
          NT g2 = 0;
#pragma unroll
          for (int e = 0; e < 9; ++e) g2 += (NT)K[e] * (NT)K[e];
          graw = g2 > graw ? g2 : graw;
        }
        for (int m = 0; m < k; ++m) {
          const T* cm = a.pool + s_off[m] + 9 * (int64_t)i;
          T cv[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) cv[e] = cm[e];
          const T* qm = s_qj + 9 * m;
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              K[3 * r + cc] -= cv[3 * r] * qm[cc] + cv[3 * r + 1] * qm[3 + cc] + cv[3 * r + 2] * qm[6 + cc];
        }
        NT nrm = 0;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          Ck[9 * (int64_t)i + e] = K[e];
          nrm += (NT)K[e] * (NT)K[e];
        }
        NT sel = a.det_pivot ? det3<NT>(K) : nrm;
        bool used = false;
        for (int m = 0; m < k; ++m) used |= (s_pi[m] == i);
        if (used) { nrm = -1; sel = -1; }
        if (sel > best || (sel == best && i < bi)) { best = sel; bi = i; }
        bestf = nrm > bestf ? nrm : bestf;
      }
      if (sizeof(T) == 4) {
        int dummy = 0;
        block_argmax(graw, dummy, s_av, s_ai);
      }
      block_argmax(best, bi, s_av, s_ai);
      if (a.det_pivot) {
        int dummy = 0;
        block_argmax(bestf, dummy, s_av, s_ai);
      } else {
        bestf = best;
      }
      // no usable row (all used or non-finite): stop without a new term
      if (!(best >= NT(0)) || bi < 0 || bi >= c) { fallback = true; break; }
      if (bestf <= NT(1e-30) * s_lam2) { converged = true; break; }
      // single precision: a residual at the rounding level of the raw column
      // (32 units of roundoff) carries no information; the block is converged
      if (sizeof(T) == 4 && bestf <= NT(3.6e-12) * graw) { converged = true; break; }
      if (tid == 0) {
        const T* P = Ck + 9 * (int64_t)bi;
        double p[9];   // pivot determinant and inverse in FP64 in every form
        for (int e = 0; e < 9; ++e) p[e] = (double)P[e];
        double det = p[0] * (p[4] * p[8] - p[5] * p[7]) - p[1] * (p[3] * p[8] - p[5] * p[6]) +
                     p[2] * (p[3] * p[7] - p[4] * p[6]);
        double fro2 = 0;
        for (int e = 0; e < 9; ++e) fro2 += p[e] * p[e];
        double fro = sqrt(fro2);
        if (!(fabs(det) > 1e-14 * fro2 * fro)) {
          s_stop = 1;
        } else {
          double id = 1.0 / det;
          s_pinv[0] = (T)((p[4] * p[8] - p[5] * p[7]) * id);
          s_pinv[1] = (T)((p[2] * p[7] - p[1] * p[8]) * id);
          s_pinv[2] = (T)((p[1] * p[5] - p[2] * p[4]) * id);
          s_pinv[3] = (T)((p[5] * p[6] - p[3] * p[8]) * id);
          s_pinv[4] = (T)((p[0] * p[8] - p[2] * p[6]) * id);
          s_pinv[5] = (T)((p[2] * p[3] - p[0] * p[5]) * id);
          s_pinv[6] = (T)((p[3] * p[7] - p[4] * p[6]) * id);
          s_pinv[7] = (T)((p[1] * p[6] - p[0] * p[7]) * id);
          s_pinv[8] = (T)((p[0] * p[4] - p[1] * p[3]) * id);
        }
        s_pi[k] = bi;
      }
      __syncthreads();
      if (s_stop) { fallback = true; break; }
      // normalisation: c_k = a P^-1
      for (int i = tid; i < c; i += ACA_T) {
        T v[9], o[9];
        for (int e = 0; e < 9; ++e) v[e] = Ck[9 * (int64_t)i + e];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            o[3 * r + cc] = v[3 * r] * s_pinv[cc] + v[3 * r + 1] * s_pinv[3 + cc] + v[3 * r + 2] * s_pinv[6 + cc];
        for (int e = 0; e < 9; ++e) Ck[9 * (int64_t)i + e] = o[e];
      }
      __syncthreads();
      const int ik = s_pi[k];
      for (int t = tid; t < 9 * k; t += ACA_T) {
        int m = t / 9, e = t % 9;
        s_ci[t] = a.pool[s_off[m] + 9 * (int64_t)ik + e];
      }
      __syncthreads();
      // residual row i_k and the next column pivot
      const double xi0 = xt[3 * ik], xi1 = xt[3 * ik + 1], xi2 = xt[3 * ik + 2];
      best = -1;
      bi = 0x7fffffff;
      double tp0 = 0, tp1 = 0, tp2 = 0;   // t_k = sum_j q_k(j) F_j (fused apply)
      if (MF) {
        for (int t0 = 32 * wv; t0 < q; t0 += 32 * NW) {
          const int jj = t0 + (lane & 31);
          const int jc = jj < q ? jj : t0;
          float K[9];
          mfma_entry(fr, a.kp.input_mode, xi0 - xsr[3 * jc], xi1 - xsr[3 * jc + 1],
                     xi2 - xsr[3 * jc + 2], K);
          if (jj < q && lane < 32)
#pragma unroll
            for (int e = 0; e < 9; ++e) Qk[9 * (int64_t)jj + e] = (T)K[e];
        }
        __syncthreads();
      }
      for (int jj = tid; jj < q; jj += ACA_T) {
        T K[9];
        if (MF) {
#pragma unroll
          for (int e = 0; e < 9; ++e) K[e] = Qk[9 * (int64_t)jj + e];
        } else {
          kernel_entry<T>(a.kp, wl, (T)(xi0 - xsr[3 * jj]), (T)(xi1 - xsr[3 * jj + 1]),
                          (T)(xi2 - xsr[3 * jj + 2]), K);
        }
        for (int m = 0; m < k; ++m) {
          const T* qm = a.pool + s_off[m] + 9 * (int64_t)c + 9 * (int64_t)jj;
          T qv[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) qv[e] = qm[e];
          const T* cm = s_ci + 9 * m;
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              K[3 * r + cc] -= cm[3 * r] * qv[cc] + cm[3 * r + 1] * qv[3 + cc] + cm[3 * r + 2] * qv[6 + cc];
        }
        NT nrm = 0;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          Qk[9 * (int64_t)jj + e] = K[e];
          nrm += (NT)K[e] * (NT)K[e];
        }
        if (fuse) {
          const T* f = a.Fs + 3 * ((int64_t)ns.x + jj);
          const double f0 = f[0], f1 = f[1], f2 = f[2];
          tp0 += (double)K[0] * f0 + (double)K[1] * f1 + (double)K[2] * f2;
          tp1 += (double)K[3] * f0 + (double)K[4] * f1 + (double)K[5] * f2;
          tp2 += (double)K[6] * f0 + (double)K[7] * f1 + (double)K[8] * f2;
        }
        NT sel = a.det_pivot ? det3<NT>(K) : nrm;
        bool used = false;
        for (int m = 0; m <= k; ++m) used |= (s_pj[m] == jj);
        if (used) sel = -1;
        if (sel > best || (sel == best && jj < bi)) { best = sel; bi = jj; }
      }
      block_argmax(best, bi, s_av, s_ai);
      const int jn = (bi >= 0 && bi < q) ? bi : -1;   // -1 only when every column is used
      if (fuse) {
        // u_i += c_k(i) t_k for the rows of this block (owner thread per row)
        tp0 = wave_sum(tp0);
        tp1 = wave_sum(tp1);
        tp2 = wave_sum(tp2);
        if (lane == 0) { s_t[wv][0] = tp0; s_t[wv][1] = tp1; s_t[wv][2] = tp2; }
        __syncthreads();
        double t0 = 0, t1 = 0, t2 = 0;
        for (int w = 0; w < NW; ++w) { t0 += s_t[w][0]; t1 += s_t[w][1]; t2 += s_t[w][2]; }
        for (int i = tid; i < c; i += ACA_T) {
          const T* e = Ck + 9 * (int64_t)i;
          ub[3 * i] += (double)e[0] * t0 + (double)e[1] * t1 + (double)e[2] * t2;
          ub[3 * i + 1] += (double)e[3] * t0 + (double)e[4] * t1 + (double)e[5] * t2;
          ub[3 * i + 2] += (double)e[6] * t0 + (double)e[7] * t1 + (double)e[8] * t2;
        }
      }
      // Gram matrices, nu^2 and the lambda^2 update
      __syncthreads();   // all of c_k and q_k are written
      NT nu2 = 0, cross = 0;
      for (int m0 = 0; m0 <= k; m0 += GCH) {
        const int mc = min(GCH, k + 1 - m0);
        for (int mm = 0; mm < mc; ++mm) {
          const int m = m0 + mm;
          NT A[9] = {0}, B[9] = {0};
          const T* Cm = a.pool + s_off[m];
          const T* Qm = Cm + 9 * (int64_t)c;
          for (int i = tid; i < c; i += ACA_T) {
            T x[9], y[9];
            for (int e = 0; e < 9; ++e) { x[e] = Cm[9 * (int64_t)i + e]; y[e] = Ck[9 * (int64_t)i + e]; }
            for (int r = 0; r < 3; ++r)
              for (int cc = 0; cc < 3; ++cc)
                A[3 * r + cc] += (NT)x[r] * (NT)y[cc] + (NT)x[3 + r] * (NT)y[3 + cc] + (NT)x[6 + r] * (NT)y[6 + cc];
          }
          for (int jj = tid; jj < q; jj += ACA_T) {
            T x[9], y[9];
            for (int e = 0; e < 9; ++e) { x[e] = Qk[9 * (int64_t)jj + e]; y[e] = Qm[9 * (int64_t)jj + e]; }
            for (int r = 0; r < 3; ++r)
              for (int cc = 0; cc < 3; ++cc)
                B[3 * r + cc] += (NT)x[3 * r] * (NT)y[3 * cc] + (NT)x[3 * r + 1] * (NT)y[3 * cc + 1] + (NT)x[3 * r + 2] * (NT)y[3 * cc + 2];
          }
          for (int e = 0; e < 9; ++e) {
            NT sa = wave_sum(A[e]), sb = wave_sum(B[e]);
            if (lane == 0) { s_red[wv][mm][e] = sa; s_red[wv][mm][9 + e] = sb; }
          }
        }
        __syncthreads();
        if (tid == 0) {
          for (int mm = 0; mm < mc; ++mm) {
            NT A[9], B[9];
            for (int e = 0; e < 9; ++e) {
              NT sa = 0, sb = 0;
              for (int w = 0; w < NW; ++w) { sa += s_red[w][mm][e]; sb += s_red[w][mm][9 + e]; }
              A[e] = sa;
              B[e] = sb;
            }
            NT tr = 0;
            for (int r = 0; r < 3; ++r)
              for (int cc = 0; cc < 3; ++cc) tr += A[3 * r + cc] * B[3 * cc + r];
            if (m0 + mm == k) nu2 = tr; else cross += tr;
          }
        }
        __syncthreads();
      }
      if (tid == 0) {
        s_lam2 = s_lam2 + nu2 + NT(2) * cross;
        s_stop = (nu2 <= NT(a.eps2) * s_lam2) ? 1 : 0;
      }
      __syncthreads();
      rank = k + 1;
      if (s_stop) { converged = true; break; }
      if (k + 1 == min(c, q)) { converged = true; break; }
      if (jn < 0) { fallback = true; break; }
      j = jn;
    }
    if (!converged) fallback = true;
    __syncthreads();
    if (fuse && fallback && MF) {
      // dense evaluation of the block's rows (32-row MFMA tiles)
      for (int t0 = 32 * wv; t0 < c; t0 += 32 * NW) {
        const int i = t0 + (lane & 31);
        const int ii = i < c ? i : t0;
        const double x0 = xt[3 * ii], x1 = xt[3 * ii + 1], x2 = xt[3 * ii + 2];
        double v0 = 0, v1 = 0, v2 = 0;
        for (int jj = 0; jj < q; ++jj) {
          float K[9];
          mfma_entry(fr, a.kp.input_mode, x0 - xsr[3 * jj], x1 - xsr[3 * jj + 1],
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
      for (int i = tid; i < c; i += ACA_T) {
        const double x0 = xt[3 * i], x1 = xt[3 * i + 1], x2 = xt[3 * i + 2];
        T v0 = 0, v1 = 0, v2 = 0;
        for (int jj = 0; jj < q; ++jj) {
          T K[9];
          kernel_entry<T>(a.kp, wl, (T)(x0 - xsr[3 * jj]), (T)(x1 - xsr[3 * jj + 1]),
                          (T)(x2 - xsr[3 * jj + 2]), K);
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
    if (tid == 0) {
      a.rank[b] = rank;
      a.flag[b] = fallback ? 1 : 0;
    }
    for (int t = tid; t < 2 * LMAX_CAP; t += ACA_T) {
      int m = t % LMAX_CAP;
      int v = -1;
      if (m < rank) v = (t < LMAX_CAP) ? s_pi[m] : s_pj[m];
      a.piv[b * 2 * LMAX_CAP + t] = v;
    }
  }
}

template <class T>
void launch_aca_t(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr,
                  int64_t b0, int64_t b1, T* pool, int64_t pool_elems, void* pool_top,
                  int* overflow, int* work, const void* Fs, double* ublk, const int64_t* uoff) {
  AcaArgs<T> a;
  a.G = p->G.as<int2>();
  a.nG = p->nG;
  a.nodes = t->nodes.as<int4>();
  a.xs = t->xs.as<double>();
  a.kp.kind = k->kind;
  a.kp.input_mode = k->input_mode;
  a.kp.a = k->a;
  a.kp.c8 = 1.0 / (8.0 * HH_PI * k->mu);
  a.kp.c6 = 1.0 / (6.0 * HH_PI * k->mu * k->a);
  a.kp.alpha1 = k->alpha1;
  a.kp.w = sizeof(T) == 8 ? k->p64.p : k->p32.p;
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
  a.b0 = b0;
  a.b1 = b1;
  a.Fs = (const T*)Fs;
  a.ublk = ublk;
  a.uoff = uoff;
  a.frags = k->pbf.as<uint4>();
  a.det_pivot = lr->prec != HH_FP64;
  int grid = (int)std::min<int64_t>(b1 - b0, 4096);
  if (grid <= 0) return;
  const bool fp64norm = lr->prec != HH_FP32;
#define LAUNCH(NT_, KIND_, MF_)                                                             \
  hipLaunchKernelGGL((k_aca<T, NT_, KIND_, MF_>), dim3(grid), dim3(ACA_T), 0, ctx->stream, a)
  if (k->kind == KIND_MLP && lr->prec == HH_BF16) {
    if constexpr (sizeof(T) == 4) LAUNCH(double, KIND_MLP, true);
  } else if (k->kind == KIND_MLP) {
    if (fp64norm) LAUNCH(double, KIND_MLP, false); else LAUNCH(T, KIND_MLP, false);
  } else {
    if (fp64norm) LAUNCH(double, KIND_RPY, false); else LAUNCH(T, KIND_RPY, false);
  }
#undef LAUNCH
  HIP_OK(hipGetLastError());
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
static void block_sizes(hh_ctx ctx, hh_tree t, hh_part p, std::vector<int32_t>& cs,
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

// Plans the ACA: stored factors when they fit the context budget, otherwise
// streamed batches whose worst-case factor storage fits it (Sec. 3.3.2: a
// fixed buffer is filled by a group of blocks, applied, then reused).
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
  int64_t est = 0, worst = 0;
  for (int64_t b = 0; b < nG; ++b) {
    int64_t cq = (int64_t)cs[b] + qs[b];
    int64_t kc = std::min<int64_t>(std::min(cs[b], qs[b]), lr->l_max);
    est += 9 * cq * std::min<int64_t>(kc, 20);
    worst += 9 * cq * kc;
  }
  lr->est_elems = est;
  lr->streamed = force_streamed || (double)est * es > 0.5 * (double)ctx->budget_bytes;
  if (!lr->streamed) return;
  // batches: worst-case factor elements + 3 c output doubles per block
  const double cap = 0.5 * (double)ctx->budget_bytes;
  lr->bounds.clear();
  lr->bounds.push_back(0);
  std::vector<int64_t> uoff(nG + 1, 0);
  double acc = 0;
  int64_t pool_max = 0, ub_max = 0, pe = 0, ue = 0;
  for (int64_t b = 0; b < nG; ++b) {
    int64_t cq = (int64_t)cs[b] + qs[b];
    int64_t kc = std::min<int64_t>(std::min(cs[b], qs[b]), lr->l_max);
    double bytes = (double)(9 * cq * kc) * es + 24.0 * cs[b];
    if (acc > 0 && acc + bytes > cap) {
      lr->bounds.push_back(b);
      pool_max = std::max(pool_max, pe);
      ub_max = std::max(ub_max, ue);
      acc = 0;
      pe = ue = 0;
    }
    acc += bytes;
    pe += 9 * cq * kc;
    ue += cs[b];
    uoff[b + 1] = uoff[b] + cs[b];
  }
  lr->bounds.push_back(nG);
  pool_max = std::max(pool_max, pe);
  ub_max = std::max(ub_max, ue);
  lr->pool_elems = std::max<int64_t>(pool_max, 1024);
  lr->ub_elems = std::max<int64_t>(ub_max, 1);
  lr->uoff.alloc(st, (nG + 1) * sizeof(int64_t));
  HIP_OK(hipMemcpyAsync(lr->uoff.p, uoff.data(), (nG + 1) * sizeof(int64_t),
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
                             flags, flags + 1, nullptr, nullptr, nullptr);
      else
        launch_aca_t<float>(ctx, t, p, k, lr, 0, nG, lr->pool.as<float>(), lr->pool_elems, top,
                            flags, flags + 1, nullptr, nullptr, nullptr);
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

// Streamed mode, batch i: ACA with the apply fused in; per-block rows go to
// ublk (offsets uoff - uoff[b0]). counters: 2 int64 per batch, zeroed.
void run_aca_batch(hh_ctx ctx, hh_tree t, hh_part p, hh_kernel k, hh_lowrank lr, size_t i,
                   const void* Fs, int64_t* counters) {
  int64_t b0 = lr->bounds[i], b1 = lr->bounds[i + 1];
  int* work = (int*)(counters + 2 * i);
  int64_t* top = counters + 2 * i + 1;
  int* ovf = (int*)ctx->scratch_flag.p;
  if (lr->prec == HH_FP64)
    launch_aca_t<double>(ctx, t, p, k, lr, b0, b1, lr->pool.as<double>(), lr->pool_elems, top,
                         ovf, work, Fs, lr->ublk.as<double>(), lr->uoff.as<int64_t>());
  else
    launch_aca_t<float>(ctx, t, p, k, lr, b0, b1, lr->pool.as<float>(), lr->pool_elems, top, ovf,
                        work, Fs, lr->ublk.as<double>(), lr->uoff.as<int64_t>());
}
