// Cluster tree (Definition 1, bisection along x, y, z as in Fig. 2) on gfx950.
//
// Steps: exact min/max of the centres -> power-of-two root cube -> 21-bit
// quantised coordinates -> 63-bit Morton keys -> stable radix sort of (key,
// index) -> binary radix tree over the sorted keys (each internal node splits
// its Morton range at the highest differing bit; equal keys are split by
// position, which is the index order) -> truncation: a node is kept when its
// parent holds >= c_leaf particles with differing keys -> pre-order numbering
// by sorting kept nodes on (begin, -end) -> leaf tables and tight node boxes.
// Cutting a binary radix tree this way yields exactly the tree of recursive
// midpoint bisection of the cube with empty halves skipped.
#include <math.h>

#include "api_guard.h"
#include "internal.h"

#pragma clang fp contract(off)

namespace {

constexpr int T256 = 256;

__global__ __launch_bounds__(T256) void k_minmax_partial(const double* __restrict__ X, int64_t n,
                                                         double* __restrict__ part,
                                                         int* __restrict__ bad) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool nonfinite = false;
  for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * T256) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = X[3 * i + d];
      if (!isfinite(v)) nonfinite = true;
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  }
  if (nonfinite) atomicOr(bad, 1);
  __shared__ double red[6][T256 / 64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int o = 32; o > 0; o >>= 1) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
    }
    if (lane == 0) { red[d][w] = lo[d]; red[3 + d][w] = hi[d]; }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = red[threadIdx.x][0];
    for (int i = 1; i < T256 / 64; ++i)
      v = threadIdx.x < 3 ? fmin(v, red[threadIdx.x][i]) : fmax(v, red[threadIdx.x][i]);
    part[6 * blockIdx.x + threadIdx.x] = v;
  }
}

// Final reduction and the quantisation constants: lo[3], scale (2^(21-e)).
__global__ void k_minmax_final(const double* __restrict__ part, int nb, double* __restrict__ q) {
  if (threadIdx.x != 0) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = 0; b < nb; ++b)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], part[6 * b + d]);
      hi[d] = fmax(hi[d], part[6 * b + 3 + d]);
    }
  double E = fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
  int e = 0;
  if (E > 0.0) (void)frexp(E, &e);  // E = m 2^e, m in [0.5, 1): smallest e with 2^e > E
  q[0] = lo[0]; q[1] = lo[1]; q[2] = lo[2];
  q[3] = ldexp(1.0, 21 - e);
}

__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  // place bit k of a 21-bit value at bit 3k
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ __launch_bounds__(T256) void k_morton(const double* __restrict__ X, int64_t n,
                                                 const double* __restrict__ q,
                                                 uint64_t* __restrict__ keys,
                                                 uint32_t* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= n) return;
  const double lo0 = q[0], lo1 = q[1], lo2 = q[2], sc = q[3];
  const double cap = 2097151.0;
  double fx = fmin(floor((X[3 * i] - lo0) * sc), cap);
  double fy = fmin(floor((X[3 * i + 1] - lo1) * sc), cap);
  double fz = fmin(floor((X[3 * i + 2] - lo2) * sc), cap);
  uint64_t k = (spread3((uint64_t)fx) << 2) | (spread3((uint64_t)fy) << 1) | spread3((uint64_t)fz);
  keys[i] = k;
  idx[i] = (uint32_t)i;
}

__global__ __launch_bounds__(T256) void k_gather_check(const double* __restrict__ X, int64_t n,
                                                       const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ idx,
                                                       double* __restrict__ xs,
                                                       int32_t* __restrict__ perm,
                                                       int* __restrict__ dup) {
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n) return;
  uint32_t o = idx[s];
  double x0 = X[3 * (int64_t)o], x1 = X[3 * (int64_t)o + 1], x2 = X[3 * (int64_t)o + 2];
  xs[3 * s] = x0; xs[3 * s + 1] = x1; xs[3 * s + 2] = x2;
  perm[s] = (int32_t)o;
  // identical positions have identical keys: compare within the run of equal keys
  uint64_t k = keys[s];
  for (int64_t t = s + 1; t < n && keys[t] == k; ++t) {
    if (t - s > 4096) { atomicOr(dup, 2); break; }
    uint32_t u = idx[t];
    if (X[3 * (int64_t)u] == x0 && X[3 * (int64_t)u + 1] == x1 && X[3 * (int64_t)u + 2] == x2) {
      atomicOr(dup, 1);
      break;
    }
  }
}

// Common-prefix length of sorted keys at positions i, j (index tie-break).
__device__ __forceinline__ int delta(const uint64_t* __restrict__ k, int64_t n, int64_t i,
                                     int64_t j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = k[i], b = k[j];
  if (a != b) return __clzll((long long)(a ^ b));
  return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// Binary radix tree (one thread per internal node i in [0, n-2]).
// rng[i] = (first, last) inclusive; kid[i] = (left, right) in the combined id
// space: internal node u -> u, sorted position s -> (n-1) + s.
__global__ __launch_bounds__(T256) void k_radix_tree(const uint64_t* __restrict__ k, int64_t n,
                                                     int2* __restrict__ rng, int2* __restrict__ kid,
                                                     int32_t* __restrict__ par) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= n - 1) return;
  int d = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) >= 0 ? 1 : -1;
  int dmin = delta(k, n, i, i - d);
  int64_t lmax = 2;
  while (delta(k, n, i, i + lmax * d) > dmin) lmax *= 2;
  int64_t l = 0;
  for (int64_t t = lmax / 2; t >= 1; t /= 2)
    if (delta(k, n, i, i + (l + t) * d) > dmin) l += t;
  int64_t j = i + l * d;
  int dnode = delta(k, n, i, j);
  int64_t s = 0;
  int64_t t = l;
  do {
    t = (t + 1) / 2;
    if (delta(k, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int64_t g = i + s * d + (d < 0 ? -1 : 0);
  int64_t first = i < j ? i : j, last = i < j ? j : i;
  int left = (first == g) ? (int)(n - 1 + g) : (int)g;
  int right = (last == g + 1) ? (int)(n - 1 + g + 1) : (int)(g + 1);
  rng[i] = make_int2((int)first, (int)last);
  kid[i] = make_int2(left, right);
  par[left] = (int)i;
  par[right] = (int)i;
}

__device__ __forceinline__ int2 node_range(const int2* __restrict__ rng, int64_t n, int u) {
  return u < n - 1 ? rng[u] : make_int2(u - (int)(n - 1), u - (int)(n - 1));
}

__device__ __forceinline__ bool splittable(const int2* __restrict__ rng,
                                           const uint64_t* __restrict__ k, int64_t n, int u,
                                           int c_leaf) {
  if (u >= n - 1) return false;
  int2 r = rng[u];
  return (r.y - r.x + 1) >= c_leaf && k[r.x] != k[r.y];
}

__global__ __launch_bounds__(T256) void k_keep(const int2* __restrict__ rng,
                                               const int32_t* __restrict__ par,
                                               const uint64_t* __restrict__ k, int64_t n,
                                               int c_leaf, int64_t* __restrict__ flag) {
  int64_t u = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (u >= 2 * n - 1) return;
  int root = n > 1 ? 0 : 0;
  bool kept = (u == root) || (par[u] >= 0 && splittable(rng, k, n, par[u], c_leaf));
  if (n == 1) kept = (u == 0);
  flag[u] = kept ? 1 : 0;
}

__global__ __launch_bounds__(T256) void k_keep_emit(const int2* __restrict__ rng,
                                                    const int64_t* __restrict__ flag,
                                                    const int64_t* __restrict__ pos, int64_t n,
                                                    uint64_t* __restrict__ skey,
                                                    uint32_t* __restrict__ sval) {
  int64_t u = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (u >= 2 * n - 1 || !flag[u]) return;
  int2 r = node_range(rng, n, (int)u);
  uint64_t b = (uint64_t)r.x, e = (uint64_t)r.y + 1;
  skey[pos[u]] = (b << 32) | (0xffffffffull - e);
  sval[pos[u]] = (uint32_t)u;
}

__global__ __launch_bounds__(T256) void k_map(const uint32_t* __restrict__ sval, int64_t m,
                                              int32_t* __restrict__ map) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p < m) map[sval[p]] = (int32_t)p;
}

__global__ __launch_bounds__(T256) void k_nodes(const uint32_t* __restrict__ sval, int64_t m,
                                                const int2* __restrict__ rng,
                                                const int2* __restrict__ kid,
                                                const uint64_t* __restrict__ k, int64_t n,
                                                int c_leaf, const int32_t* __restrict__ map,
                                                int4* __restrict__ nodes,
                                                int32_t* __restrict__ parent,
                                                int64_t* __restrict__ isleaf) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p >= m) return;
  int u = (int)sval[p];
  int2 r = node_range(rng, n, u);
  int4 nd = make_int4(r.x, r.y + 1, -1, -1);
  if (splittable(rng, k, n, u, c_leaf)) {
    int2 c = kid[u];
    nd.z = map[c.x];
    nd.w = map[c.y];
    parent[nd.z] = (int)p;
    parent[nd.w] = (int)p;
  }
  if (p == 0) parent[0] = -1;
  nodes[p] = nd;
  isleaf[p] = nd.z < 0 ? 1 : 0;
}

__global__ __launch_bounds__(T256) void k_leaves(const int64_t* __restrict__ isleaf,
                                                 const int64_t* __restrict__ lpos, int64_t m,
                                                 int32_t* __restrict__ leaf_id,
                                                 int32_t* __restrict__ leaves) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p >= m) return;
  if (isleaf[p]) {
    leaf_id[p] = (int32_t)lpos[p];
    leaves[lpos[p]] = (int32_t)p;
  } else {
    leaf_id[p] = -1;
  }
}

// One wave per leaf: leaf_of and the tight box of the members.
__global__ __launch_bounds__(T256) void k_leaf_box(const int32_t* __restrict__ leaves,
                                                   int64_t nl, const int4* __restrict__ nodes,
                                                   const double* __restrict__ xs,
                                                   int32_t* __restrict__ leaf_of,
                                                   double* __restrict__ bbox) {
  int64_t lw = ((int64_t)blockIdx.x * T256 + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (lw >= nl) return;
  int p = leaves[lw];
  int4 nd = nodes[p];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int s = nd.x + lane; s < nd.y; s += 64) {
    leaf_of[s] = p;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = xs[3 * (int64_t)s + d];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int o = 32; o > 0; o >>= 1) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
    }
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      bbox[6 * (int64_t)p + d] = lo[d];
      bbox[6 * (int64_t)p + 3 + d] = hi[d];
    }
}

// One wave per internal node: reduce the boxes of the leaves it contains.
__global__ __launch_bounds__(T256) void k_inner_box(const int4* __restrict__ nodes, int64_t m,
                                                    const int32_t* __restrict__ leaves,
                                                    int64_t nl, double* __restrict__ bbox) {
  int64_t p = ((int64_t)blockIdx.x * T256 + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (p >= m) return;
  int4 nd = nodes[p];
  if (nd.z < 0) return;
  // leaves are in begin order: find the first with begin >= nd.x and >= nd.y
  auto lower = [&](int key) {
    int64_t a = 0, b = nl;
    while (a < b) {
      int64_t mid = (a + b) / 2;
      if (nodes[leaves[mid]].x < key) a = mid + 1; else b = mid;
    }
    return a;
  };
  int64_t l0 = lower(nd.x), l1 = lower(nd.y);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t l = l0 + lane; l < l1; l += 64) {
    int q = leaves[l];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], bbox[6 * (int64_t)q + d]);
      hi[d] = fmax(hi[d], bbox[6 * (int64_t)q + 3 + d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int o = 32; o > 0; o >>= 1) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
    }
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      bbox[6 * p + d] = lo[d];
      bbox[6 * p + 3 + d] = hi[d];
    }
}

inline unsigned nblk(int64_t n, int t = T256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

extern "C" {

hh_status hh_build_tree(hh_ctx ctx, const double* X, int64_t n, int32_t c_leaf, hh_tree* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && X, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(n >= 1 && n < (1ll << 31) - 1, HH_ERR_INVALID_ARG, "n must be in [1, 2^31-2]");
  HH_REQUIRE(c_leaf >= 2, HH_ERR_INVALID_ARG, "c_leaf must be >= 2");
  hipStream_t st = ctx->stream;
  PhaseTimer timer(ctx, HH_PHASE_TREE);
  hh_tree_s* t = new hh_tree_s();
  try {
    t->ctx = ctx;
    t->n = n;
    t->c_leaf = c_leaf;
    // a1: box, quantisation constants, Morton keys
    int nbmm = (int)std::min<int64_t>(1024, nblk(n));
    DevBuf part, qc, keys_tmp;
    part.alloc(st, 6 * nbmm * sizeof(double));
    qc.alloc(st, 4 * sizeof(double));
    int* flags = (int*)ctx->scratch_flag.p;   // [0] non-finite, [1] duplicates
    HIP_OK(hipMemsetAsync(flags, 0, 4 * sizeof(int), st));
    hipLaunchKernelGGL(k_minmax_partial, dim3(nbmm), dim3(T256), 0, st, X, n,
                       part.as<double>(), flags);
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(64), 0, st, part.as<double>(), nbmm,
                       qc.as<double>());
    t->keys.alloc(st, n * sizeof(uint64_t));
    DevBuf idx;
    idx.alloc(st, n * sizeof(uint32_t));
    hipLaunchKernelGGL(k_morton, dim3(nblk(n)), dim3(T256), 0, st, X, n, qc.as<double>(),
                       t->keys.as<uint64_t>(), idx.as<uint32_t>());
    HIP_OK(hipGetLastError());
    // a2: stable sort by key (ties keep input order), gather, duplicate check
    radix_sort_u64(ctx, t->keys.as<uint64_t>(), idx.as<uint32_t>(), n, 63);
    t->xs.alloc(st, 3 * n * sizeof(double));
    t->perm.alloc(st, n * sizeof(int32_t));
    hipLaunchKernelGGL(k_gather_check, dim3(nblk(n)), dim3(T256), 0, st, X, n,
                       t->keys.as<uint64_t>(), idx.as<uint32_t>(), t->xs.as<double>(),
                       t->perm.as<int32_t>(), flags + 1);
    HIP_OK(hipGetLastError());
    // a3: radix tree, truncation, pre-order
    int64_t nt = 2 * n - 1;
    DevBuf rng, kid, par, keep, kpos;
    rng.alloc(st, std::max<int64_t>(1, n - 1) * sizeof(int2));
    kid.alloc(st, std::max<int64_t>(1, n - 1) * sizeof(int2));
    par.alloc(st, nt * sizeof(int32_t));
    HIP_OK(hipMemsetAsync(par.p, 0xff, nt * sizeof(int32_t), st));
    if (n > 1)
      hipLaunchKernelGGL(k_radix_tree, dim3(nblk(n - 1)), dim3(T256), 0, st,
                         t->keys.as<uint64_t>(), n, rng.as<int2>(), kid.as<int2>(),
                         par.as<int32_t>());
    keep.alloc(st, (nt + 1) * sizeof(int64_t));
    kpos.alloc(st, (nt + 1) * sizeof(int64_t));
    HIP_OK(hipMemsetAsync(keep.as<int64_t>() + nt, 0, sizeof(int64_t), st));
    hipLaunchKernelGGL(k_keep, dim3(nblk(nt)), dim3(T256), 0, st, rng.as<int2>(),
                       par.as<int32_t>(), t->keys.as<uint64_t>(), n, c_leaf, keep.as<int64_t>());
    scan_exclusive_i64(ctx, keep.as<int64_t>(), kpos.as<int64_t>(), nt + 1);
    HIP_OK(hipMemcpyAsync(ctx->pinned, kpos.as<int64_t>() + nt, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(ctx->pinned + 1, flags, 8, hipMemcpyDeviceToHost, st));
    ctx_sync(ctx);
    int64_t m = ctx->pinned[0];
    int fl_nonfinite = ((int*)(ctx->pinned + 1))[0], fl_dup = ((int*)(ctx->pinned + 1))[1];
    HH_REQUIRE(!fl_nonfinite, HH_ERR_INVALID_ARG, "X holds a non-finite coordinate");
    HH_REQUIRE(!fl_dup, HH_ERR_DUPLICATE_POINTS, "two particles have identical positions");
    t->n_nodes = m;
    DevBuf skey, sval, map;
    skey.alloc(st, m * sizeof(uint64_t));
    sval.alloc(st, m * sizeof(uint32_t));
    hipLaunchKernelGGL(k_keep_emit, dim3(nblk(nt)), dim3(T256), 0, st, rng.as<int2>(),
                       keep.as<int64_t>(), kpos.as<int64_t>(), n, skey.as<uint64_t>(),
                       sval.as<uint32_t>());
    int bits = 32;
    while ((1ll << (bits - 32)) <= n) ++bits;
    radix_sort_u64(ctx, skey.as<uint64_t>(), sval.as<uint32_t>(), m, bits);
    map.alloc(st, nt * sizeof(int32_t));
    hipLaunchKernelGGL(k_map, dim3(nblk(m)), dim3(T256), 0, st, sval.as<uint32_t>(), m,
                       map.as<int32_t>());
    t->nodes.alloc(st, m * sizeof(int4));
    t->parent.alloc(st, m * sizeof(int32_t));
    DevBuf isleaf, lpos;
    isleaf.alloc(st, (m + 1) * sizeof(int64_t));
    lpos.alloc(st, (m + 1) * sizeof(int64_t));
    HIP_OK(hipMemsetAsync(isleaf.as<int64_t>() + m, 0, sizeof(int64_t), st));
    hipLaunchKernelGGL(k_nodes, dim3(nblk(m)), dim3(T256), 0, st, sval.as<uint32_t>(), m,
                       rng.as<int2>(), kid.as<int2>(), t->keys.as<uint64_t>(), n, c_leaf,
                       map.as<int32_t>(), t->nodes.as<int4>(), t->parent.as<int32_t>(),
                       isleaf.as<int64_t>());
    scan_exclusive_i64(ctx, isleaf.as<int64_t>(), lpos.as<int64_t>(), m + 1);
    int64_t nl = read_i64(ctx, lpos.as<int64_t>() + m);
    t->n_leaves = nl;
    t->leaf_id.alloc(st, m * sizeof(int32_t));
    t->leaves.alloc(st, nl * sizeof(int32_t));
    hipLaunchKernelGGL(k_leaves, dim3(nblk(m)), dim3(T256), 0, st, isleaf.as<int64_t>(),
                       lpos.as<int64_t>(), m, t->leaf_id.as<int32_t>(), t->leaves.as<int32_t>());
    t->leaf_of.alloc(st, n * sizeof(int32_t));
    t->bbox.alloc(st, 6 * m * sizeof(double));
    hipLaunchKernelGGL(k_leaf_box, dim3(nblk(nl * 64)), dim3(T256), 0, st,
                       t->leaves.as<int32_t>(), nl, t->nodes.as<int4>(), t->xs.as<double>(),
                       t->leaf_of.as<int32_t>(), t->bbox.as<double>());
    hipLaunchKernelGGL(k_inner_box, dim3(nblk(m * 64)), dim3(T256), 0, st, t->nodes.as<int4>(), m,
                       t->leaves.as<int32_t>(), nl, t->bbox.as<double>());
    HIP_OK(hipGetLastError());
  } catch (...) {
    delete t;
    throw;
  }
  *out = t;
  HH_API_END(ctx)
}

void hh_tree_free(hh_tree t) { delete t; }

hh_status hh_tree_info(hh_tree t, int64_t* n, int64_t* n_nodes, int64_t* n_leaves) {
  if (!t) return HH_ERR_INVALID_ARG;
  if (n) *n = t->n;
  if (n_nodes) *n_nodes = t->n_nodes;
  if (n_leaves) *n_leaves = t->n_leaves;
  return HH_OK;
}

hh_status hh_tree_export(hh_tree t, int64_t* perm, uint64_t* keys, int32_t* nodes, double* bbox) {
  if (!t) return HH_ERR_INVALID_ARG;
  hh_ctx ctx = t->ctx;
  HH_API_BEGIN(ctx)
  if (perm) {
    std::vector<int32_t> p(t->n);
    read_bytes(ctx, p.data(), t->perm.p, t->n * sizeof(int32_t));
    for (int64_t i = 0; i < t->n; ++i) perm[i] = p[i];
  }
  if (keys) read_bytes(ctx, keys, t->keys.p, t->n * sizeof(uint64_t));
  if (nodes) read_bytes(ctx, nodes, t->nodes.p, t->n_nodes * sizeof(int4));
  if (bbox) read_bytes(ctx, bbox, t->bbox.p, t->n_nodes * 6 * sizeof(double));
  HH_API_END(ctx)
}

}  // extern "C"
