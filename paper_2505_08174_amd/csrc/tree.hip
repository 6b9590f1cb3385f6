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

#include <algorithm>

#include "api_guard.h"
#include "internal.h"

#pragma clang fp contract(off)

namespace {

constexpr int T256 = 256;

// Monotone map of doubles to unsigned integers (exact min/max with atomics).
__device__ __forceinline__ unsigned long long ord64(double d) {
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord64(unsigned long long u) {
  u = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
  return __longlong_as_double((long long)u);
}

__device__ __forceinline__ int sys_of(const int64_t* __restrict__ off, int nsys, int64_t i) {
  int a = 0, b = nsys - 1;   // largest s with off[s] <= i
  while (a < b) {
    int m = (a + b + 1) / 2;
    if (off[m] <= i) a = m; else b = m - 1;
  }
  return a;
}

// Exact per-system bounding boxes: wave reduction when a wave's particles
// belong to one system, ordered-integer atomics into mm[s][6].
__global__ __launch_bounds__(T256) void k_minmax_sys(const double* __restrict__ X, int64_t n,
                                                     const int64_t* __restrict__ off, int nsys,
                                                     unsigned long long* __restrict__ mm,
                                                     int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  const bool act = i < n;
  const int64_t ii = act ? i : n - 1;
  const int s = sys_of(off, nsys, ii);
  double v[3];
  bool nonfinite = false;
  for (int d = 0; d < 3; ++d) {
    v[d] = X[3 * ii + d];
    if (act && !isfinite(v[d])) nonfinite = true;
  }
  if (nonfinite) atomicOr(bad, 1);
  const int s0 = __shfl(s, 0, 64);
  const bool uni = __all(s == s0);
  if (uni) {
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = v[d];
      hi[d] = v[d];
      for (int o = 32; o > 0; o >>= 1) {
        lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
        hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
      }
    }
    if ((threadIdx.x & 63) == 0)
      for (int d = 0; d < 3; ++d) {
        atomicMin(&mm[6 * s + d], ord64(lo[d]));
        atomicMax(&mm[6 * s + 3 + d], ord64(hi[d]));
      }
  } else if (act) {
    for (int d = 0; d < 3; ++d) {
      atomicMin(&mm[6 * s + d], ord64(v[d]));
      atomicMax(&mm[6 * s + 3 + d], ord64(v[d]));
    }
  }
}

__global__ void k_mm_init(unsigned long long* __restrict__ mm, int nsys) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i < 6 * nsys) mm[i] = (i % 6) < 3 ? ~0ull : 0ull;
}

// Quantisation constants per system: lo[3], scale = 2^(21-e).
__global__ void k_sys_final(const unsigned long long* __restrict__ mm, int nsys,
                            double* __restrict__ q) {
  int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= nsys) return;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = unord64(mm[6 * s + d]);
    hi[d] = unord64(mm[6 * s + 3 + d]);
  }
  double E = fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
  int e = 0;
  if (E > 0.0) (void)frexp(E, &e);  // E = m 2^e, m in [0.5, 1): smallest e with 2^e > E
  q[4 * s] = lo[0]; q[4 * s + 1] = lo[1]; q[4 * s + 2] = lo[2];
  q[4 * s + 3] = ldexp(1.0, 21 - e);
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

__device__ __forceinline__ uint64_t morton_of(const double* __restrict__ x,
                                              const double* __restrict__ q) {
  const double cap = 2097151.0;
  double fx = fmin(floor((x[0] - q[0]) * q[3]), cap);
  double fy = fmin(floor((x[1] - q[1]) * q[3]), cap);
  double fz = fmin(floor((x[2] - q[2]) * q[3]), cap);
  return (spread3((uint64_t)fx) << 2) | (spread3((uint64_t)fy) << 1) | spread3((uint64_t)fz);
}

__global__ __launch_bounds__(T256) void k_morton(const double* __restrict__ X, int64_t n,
                                                 const int64_t* __restrict__ off, int nsys,
                                                 const double* __restrict__ q,
                                                 uint64_t* __restrict__ keys,
                                                 uint32_t* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= n) return;
  keys[i] = morton_of(X + 3 * i, q + 4 * sys_of(off, nsys, i));
  idx[i] = (uint32_t)i;
}

// Second key of the segmented sort: the system of each (key-sorted) particle.
__global__ __launch_bounds__(T256) void k_syskey(const uint32_t* __restrict__ idx, int64_t n,
                                                 const int64_t* __restrict__ off, int nsys,
                                                 uint64_t* __restrict__ k2) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p < n) k2[p] = (uint64_t)sys_of(off, nsys, idx[p]);
}

// Final order: Morton keys and systems at each sorted position.
__global__ __launch_bounds__(T256) void k_rekey(const double* __restrict__ X, int64_t n,
                                                const int64_t* __restrict__ off, int nsys,
                                                const double* __restrict__ q,
                                                const uint32_t* __restrict__ idx,
                                                uint64_t* __restrict__ keys,
                                                int32_t* __restrict__ sysk) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p >= n) return;
  const int64_t i = idx[p];
  const int s = sys_of(off, nsys, i);
  keys[p] = morton_of(X + 3 * i, q + 4 * s);
  sysk[p] = s;
}

__global__ __launch_bounds__(T256) void k_gather_check(const double* __restrict__ X, int64_t n,
                                                       const uint64_t* __restrict__ keys,
                                                       const int32_t* __restrict__ sysk,
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
  // identical positions of one system have identical keys: compare within
  // the run of equal (system, key)
  uint64_t k = keys[s];
  int32_t sy = sysk[s];
  for (int64_t t = s + 1; t < n && keys[t] == k && sysk[t] == sy; ++t) {
    if (t - s > 4096) { atomicOr(dup, 2); break; }
    uint32_t u = idx[t];
    if (X[3 * (int64_t)u] == x0 && X[3 * (int64_t)u + 1] == x1 && X[3 * (int64_t)u + 2] == x2) {
      atomicOr(dup, 1);
      break;
    }
  }
}

// Common-prefix length of the sorted (system, key, position) strings at
// positions i, j: sbits system bits, then 64 key bits, then 32 position bits.
__device__ __forceinline__ int delta(const uint64_t* __restrict__ k, const int32_t* __restrict__ sy,
                                     int sbits, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  if (sbits > 0) {
    int a = sy[i], b = sy[j];
    if (a != b) return __clz(a ^ b) - (32 - sbits);
  }
  uint64_t ka = k[i], kb = k[j];
  if (ka != kb) return sbits + __clzll((long long)(ka ^ kb));
  return sbits + 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// Binary radix tree (one thread per internal node i in [0, n-2]).
// rng[i] = (first, last) inclusive; kid[i] = (left, right) in the combined id
// space: internal node u -> u, sorted position s -> (n-1) + s.
__global__ __launch_bounds__(T256) void k_radix_tree(const uint64_t* __restrict__ k,
                                                     const int32_t* __restrict__ sy, int sbits,
                                                     int64_t n, int2* __restrict__ rng,
                                                     int2* __restrict__ kid,
                                                     int32_t* __restrict__ par) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= n - 1) return;
  int d = (delta(k, sy, sbits, n, i, i + 1) - delta(k, sy, sbits, n, i, i - 1)) >= 0 ? 1 : -1;
  int dmin = delta(k, sy, sbits, n, i, i - d);
  int64_t lmax = 2;
  while (delta(k, sy, sbits, n, i, i + lmax * d) > dmin) lmax *= 2;
  int64_t l = 0;
  for (int64_t t = lmax / 2; t >= 1; t /= 2)
    if (delta(k, sy, sbits, n, i, i + (l + t) * d) > dmin) l += t;
  int64_t j = i + l * d;
  int dnode = delta(k, sy, sbits, n, i, j);
  int64_t s = 0;
  int64_t t = l;
  do {
    t = (t + 1) / 2;
    if (delta(k, sy, sbits, n, i, i + (s + t) * d) > dnode) s += t;
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

// A node spans several systems when its first and last particle differ in
// system; such nodes only join system roots and are not part of the tree.
__device__ __forceinline__ bool mixed(const int2* __restrict__ rng, const int32_t* __restrict__ sy,
                                      int64_t n, int u) {
  int2 r = node_range(rng, n, u);
  return sy[r.x] != sy[r.y];
}

// cl: leaf size C_leaf of every system
__device__ __forceinline__ bool splittable(const int2* __restrict__ rng,
                                           const uint64_t* __restrict__ k,
                                           const int32_t* __restrict__ sy, int64_t n, int u,
                                           const int32_t* __restrict__ cl) {
  if (u >= n - 1) return false;
  int2 r = rng[u];
  return sy[r.x] == sy[r.y] && (r.y - r.x + 1) >= cl[sy[r.x]] && k[r.x] != k[r.y];
}

// kept: a system root (no parent, or a parent spanning systems) or a son of
// a splittable node.
__global__ __launch_bounds__(T256) void k_keep(const int2* __restrict__ rng,
                                               const int32_t* __restrict__ par,
                                               const uint64_t* __restrict__ k,
                                               const int32_t* __restrict__ sy, int64_t n,
                                               const int32_t* __restrict__ cl,
                                               int64_t* __restrict__ flag) {
  int64_t u = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (u >= 2 * n - 1) return;
  bool kept;
  if (mixed(rng, sy, n, (int)u)) kept = false;
  else if (par[u] < 0 || mixed(rng, sy, n, par[u])) kept = true;
  else kept = splittable(rng, k, sy, n, par[u], cl);
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
                                                const uint64_t* __restrict__ k,
                                                const int32_t* __restrict__ sy, int64_t n,
                                                const int32_t* __restrict__ cl,
                                                const int32_t* __restrict__ map,
                                                int4* __restrict__ nodes,
                                                int32_t* __restrict__ parent,
                                                int64_t* __restrict__ isleaf) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p >= m) return;
  int u = (int)sval[p];
  int2 r = node_range(rng, n, u);
  int4 nd = make_int4(r.x, r.y + 1, -1, -1);
  if (splittable(rng, k, sy, n, u, cl)) {
    int2 c = kid[u];
    nd.z = map[c.x];
    nd.w = map[c.y];
    parent[nd.z] = (int)p;
    parent[nd.w] = (int)p;
  }
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

// System roots: kept nodes without a parent, indexed by the system of their
// first particle.
__global__ __launch_bounds__(T256) void k_roots(const int4* __restrict__ nodes, int64_t m,
                                                const int32_t* __restrict__ parent,
                                                const int32_t* __restrict__ sysk,
                                                int32_t* __restrict__ roots) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p < m && parent[p] < 0) roots[sysk[nodes[p].x]] = (int32_t)p;
}

inline unsigned nblk(int64_t n, int t = T256) { return (unsigned)((n + t - 1) / t); }

// Refit: new positions in the kept order (xs[s] = X[perm[s]]).
// shift = 1 on a tree of 6N rows: row perm[s] belongs to particle perm[s] >> 1
__global__ __launch_bounds__(T256) void k_refit_gather(const double* __restrict__ X, int64_t n,
                                                       const int32_t* __restrict__ perm,
                                                       int shift, double* __restrict__ xs,
                                                       int* __restrict__ bad) {
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n) return;
  const int64_t o = perm[s] >> shift;
  const double x0 = X[3 * o], x1 = X[3 * o + 1], x2 = X[3 * o + 2];
  if (!isfinite(x0) || !isfinite(x1) || !isfinite(x2)) atomicOr(bad, 1);
  xs[3 * s] = x0;
  xs[3 * s + 1] = x1;
  xs[3 * s + 2] = x2;
}

// Rows of the 6N tree from the particle tree: sorted row s = 2p + r is row r
// (0: translation, 1: rotation) of sorted particle p, input row 2 perm[p] + r.
__global__ __launch_bounds__(T256) void k_six_rows(int64_t n2, const int32_t* __restrict__ perm1,
                                                   const uint64_t* __restrict__ keys1,
                                                   const double* __restrict__ xs1,
                                                   const int32_t* __restrict__ leaf_of1,
                                                   int32_t* __restrict__ perm,
                                                   uint64_t* __restrict__ keys,
                                                   double* __restrict__ xs,
                                                   int32_t* __restrict__ leaf_of) {
  int64_t s = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (s >= n2) return;
  const int64_t p = s >> 1;
  perm[s] = 2 * perm1[p] + (int32_t)(s & 1);
  keys[s] = keys1[p];
  xs[3 * s] = xs1[3 * p];
  xs[3 * s + 1] = xs1[3 * p + 1];
  xs[3 * s + 2] = xs1[3 * p + 2];
  leaf_of[s] = leaf_of1[p];
}

__global__ __launch_bounds__(T256) void k_six_nodes(int64_t m, int4* __restrict__ nodes) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= m) return;
  int4 v = nodes[i];
  v.x *= 2;
  v.y *= 2;
  nodes[i] = v;
}

// moves the storage of src into dst (both on the context stream)
void take(DevBuf& dst, DevBuf& src) {
  dst.release();
  dst.p = src.p;
  dst.bytes = src.bytes;
  dst.s = src.s;
  src.p = nullptr;
  src.bytes = 0;
}

}  // namespace

static void build_tree_impl(hh_ctx ctx, hh_tree_s* t, const double* X, int64_t n,
                            const std::vector<int64_t>& offs, const std::vector<int32_t>& cls) {
  hipStream_t st = ctx->stream;
  const int nsys = (int)offs.size() - 1;
  int sbits = 0;
  while ((1 << sbits) < nsys) ++sbits;
  t->ctx = ctx;
  t->n = n;
  t->c_leaf = *std::max_element(cls.begin(), cls.end());
  t->cl.alloc(st, nsys * sizeof(int32_t));
  HIP_OK(hipMemcpyAsync(t->cl.p, cls.data(), nsys * sizeof(int32_t), hipMemcpyHostToDevice, st));
  t->n_sys = nsys;
  t->offs_host = offs;
  t->offs.alloc(st, (nsys + 1) * sizeof(int64_t));
  HIP_OK(hipMemcpyAsync(t->offs.p, offs.data(), (nsys + 1) * sizeof(int64_t),
                        hipMemcpyHostToDevice, st));
  const int64_t* off = t->offs.as<int64_t>();
  // a1: per-system box, quantisation constants, Morton keys
  DevBuf mm, qc;
  mm.alloc(st, 6 * nsys * sizeof(unsigned long long));
  qc.alloc(st, 4 * nsys * sizeof(double));
  int* flags = (int*)ctx->scratch_flag.p;   // [0] non-finite, [1] duplicates
  HIP_OK(hipMemsetAsync(flags, 0, 4 * sizeof(int), st));
  hipLaunchKernelGGL(k_mm_init, dim3((6 * nsys + 255) / 256), dim3(256), 0, st,
                     mm.as<unsigned long long>(), nsys);
  hipLaunchKernelGGL(k_minmax_sys, dim3(nblk(n)), dim3(T256), 0, st, X, n, off, nsys,
                     mm.as<unsigned long long>(), flags);
  hipLaunchKernelGGL(k_sys_final, dim3((nsys + 255) / 256), dim3(256), 0, st,
                     mm.as<unsigned long long>(), nsys, qc.as<double>());
  t->keys.alloc(st, n * sizeof(uint64_t));
  DevBuf idx, sysk;
  idx.alloc(st, n * sizeof(uint32_t));
  sysk.alloc(st, n * sizeof(int32_t));
  hipLaunchKernelGGL(k_morton, dim3(nblk(n)), dim3(T256), 0, st, X, n, off, nsys,
                     qc.as<double>(), t->keys.as<uint64_t>(), idx.as<uint32_t>());
  HIP_OK(hipGetLastError());
  // a2: stable sort by key, then (several systems) stably by system
  radix_sort_u64(ctx, t->keys.as<uint64_t>(), idx.as<uint32_t>(), n, 63);
  if (nsys > 1) {
    hipLaunchKernelGGL(k_syskey, dim3(nblk(n)), dim3(T256), 0, st, idx.as<uint32_t>(), n, off,
                       nsys, t->keys.as<uint64_t>());
    radix_sort_u64(ctx, t->keys.as<uint64_t>(), idx.as<uint32_t>(), n, sbits);
  }
  hipLaunchKernelGGL(k_rekey, dim3(nblk(n)), dim3(T256), 0, st, X, n, off, nsys,
                     qc.as<double>(), idx.as<uint32_t>(), t->keys.as<uint64_t>(),
                     sysk.as<int32_t>());
  t->xs.alloc(st, 3 * n * sizeof(double));
  t->perm.alloc(st, n * sizeof(int32_t));
  hipLaunchKernelGGL(k_gather_check, dim3(nblk(n)), dim3(T256), 0, st, X, n,
                     t->keys.as<uint64_t>(), sysk.as<int32_t>(), idx.as<uint32_t>(),
                     t->xs.as<double>(), t->perm.as<int32_t>(), flags + 1);
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
                       t->keys.as<uint64_t>(), sysk.as<int32_t>(), sbits, n, rng.as<int2>(),
                       kid.as<int2>(), par.as<int32_t>());
  keep.alloc(st, (nt + 1) * sizeof(int64_t));
  kpos.alloc(st, (nt + 1) * sizeof(int64_t));
  HIP_OK(hipMemsetAsync(keep.as<int64_t>() + nt, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_keep, dim3(nblk(nt)), dim3(T256), 0, st, rng.as<int2>(),
                     par.as<int32_t>(), t->keys.as<uint64_t>(), sysk.as<int32_t>(), n,
                     t->cl.as<int32_t>(), keep.as<int64_t>());
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
  HIP_OK(hipMemsetAsync(t->parent.p, 0xff, m * sizeof(int32_t), st));
  DevBuf isleaf, lpos;
  isleaf.alloc(st, (m + 1) * sizeof(int64_t));
  lpos.alloc(st, (m + 1) * sizeof(int64_t));
  HIP_OK(hipMemsetAsync(isleaf.as<int64_t>() + m, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_nodes, dim3(nblk(m)), dim3(T256), 0, st, sval.as<uint32_t>(), m,
                     rng.as<int2>(), kid.as<int2>(), t->keys.as<uint64_t>(), sysk.as<int32_t>(),
                     n, t->cl.as<int32_t>(), map.as<int32_t>(), t->nodes.as<int4>(),
                     t->parent.as<int32_t>(),
                     isleaf.as<int64_t>());
  t->roots.alloc(st, nsys * sizeof(int32_t));
  hipLaunchKernelGGL(k_roots, dim3(nblk(m)), dim3(T256), 0, st, t->nodes.as<int4>(), m,
                     t->parent.as<int32_t>(), sysk.as<int32_t>(), t->roots.as<int32_t>());
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
  // work units of the MFMA near field (32-target chunks of every leaf), so
  // that no product on this tree allocates
  ensure_units(ctx, t);
}

extern "C" {

hh_status hh_build_tree(hh_ctx ctx, const double* X, int64_t n, int32_t c_leaf, hh_tree* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && X, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(n >= 1 && n < (1ll << 31) - 1, HH_ERR_INVALID_ARG, "n must be in [1, 2^31-2]");
  HH_REQUIRE(c_leaf >= 2, HH_ERR_INVALID_ARG, "c_leaf must be >= 2");
  PhaseTimer timer(ctx, HH_PHASE_TREE);
  hh_tree_s* t = new hh_tree_s();
  try {
    build_tree_impl(ctx, t, X, n, std::vector<int64_t>{0, n}, std::vector<int32_t>{c_leaf});
  } catch (...) {
    delete t;
    throw;
  }
  *out = t;
  HH_API_END(ctx)
}

hh_status hh_build_tree6(hh_ctx ctx, const double* X, int64_t n, int32_t c_leaf, hh_tree* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && X, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(n >= 1 && n < (1ll << 30) - 1, HH_ERR_INVALID_ARG, "n must be in [1, 2^30-2]");
  HH_REQUIRE(c_leaf >= 2 && c_leaf < (1 << 29), HH_ERR_INVALID_ARG,
             "c_leaf must be in [2, 2^29)");
  PhaseTimer timer(ctx, HH_PHASE_TREE);
  hipStream_t st = ctx->stream;
  hh_tree_s one;   // the particle tree
  hh_tree_s* t = new hh_tree_s();
  try {
    build_tree_impl(ctx, &one, X, n, std::vector<int64_t>{0, n}, std::vector<int32_t>{c_leaf});
    const int64_t n2 = 2 * n, m = one.n_nodes;
    t->ctx = ctx;
    t->six = true;
    t->n = n2;
    t->c_leaf = 2 * c_leaf;
    t->n_nodes = m;
    t->n_leaves = one.n_leaves;
    t->n_sys = 1;
    t->offs_host = {0, n2};
    t->offs.alloc(st, 2 * sizeof(int64_t));
    HIP_OK(hipMemcpyAsync(t->offs.p, t->offs_host.data(), 2 * sizeof(int64_t),
                          hipMemcpyHostToDevice, st));
    const int32_t cl2 = 2 * c_leaf;
    t->cl.alloc(st, sizeof(int32_t));
    HIP_OK(hipMemcpyAsync(t->cl.p, &cl2, sizeof(int32_t), hipMemcpyHostToDevice, st));
    t->perm.alloc(st, n2 * sizeof(int32_t));
    t->keys.alloc(st, n2 * sizeof(uint64_t));
    t->xs.alloc(st, 3 * n2 * sizeof(double));
    t->leaf_of.alloc(st, n2 * sizeof(int32_t));
    hipLaunchKernelGGL(k_six_rows, dim3(nblk(n2)), dim3(T256), 0, st, n2, one.perm.as<int32_t>(),
                       one.keys.as<uint64_t>(), one.xs.as<double>(), one.leaf_of.as<int32_t>(),
                       t->perm.as<int32_t>(), t->keys.as<uint64_t>(), t->xs.as<double>(),
                       t->leaf_of.as<int32_t>());
    take(t->nodes, one.nodes);
    hipLaunchKernelGGL(k_six_nodes, dim3(nblk(m)), dim3(T256), 0, st, m, t->nodes.as<int4>());
    HIP_OK(hipGetLastError());
    take(t->parent, one.parent);
    take(t->bbox, one.bbox);
    take(t->leaf_id, one.leaf_id);
    take(t->leaves, one.leaves);
    take(t->roots, one.roots);
    ensure_units(ctx, t);
    ctx_sync(ctx);   // the host values above stay valid until the copies ran
  } catch (...) {
    delete t;
    throw;
  }
  *out = t;
  HH_API_END(ctx)
}

static hh_status build_batch(hh_ctx ctx, const double* X, const int64_t* offsets, int32_t n_sys,
                             const int32_t* c_leafs, int32_t c_leaf, hh_tree* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && X && offsets, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(n_sys >= 1 && n_sys <= (1 << 20), HH_ERR_INVALID_ARG, "n_sys must be in [1, 2^20]");
  std::vector<int32_t> cls(n_sys, c_leaf);
  if (c_leafs) cls.assign(c_leafs, c_leafs + n_sys);
  for (int s = 0; s < n_sys; ++s)
    HH_REQUIRE(cls[s] >= 2, HH_ERR_INVALID_ARG, "c_leaf must be >= 2");
  std::vector<int64_t> offs(offsets, offsets + n_sys + 1);
  HH_REQUIRE(offs[0] == 0, HH_ERR_INVALID_ARG, "offsets[0] must be 0");
  for (int s = 0; s < n_sys; ++s)
    HH_REQUIRE(offs[s + 1] > offs[s], HH_ERR_INVALID_ARG, "every system needs >= 1 particle");
  const int64_t n = offs[n_sys];
  HH_REQUIRE(n < (1ll << 31) - 1, HH_ERR_INVALID_ARG, "total n must be < 2^31-1");
  PhaseTimer timer(ctx, HH_PHASE_TREE);
  hh_tree_s* t = new hh_tree_s();
  try {
    build_tree_impl(ctx, t, X, n, offs, cls);
  } catch (...) {
    delete t;
    throw;
  }
  *out = t;
  HH_API_END(ctx)
}

hh_status hh_build_tree_batch(hh_ctx ctx, const double* X, const int64_t* offsets, int32_t n_sys,
                              int32_t c_leaf, hh_tree* out) {
  return build_batch(ctx, X, offsets, n_sys, nullptr, c_leaf, out);
}

hh_status hh_build_tree_batch_leaf(hh_ctx ctx, const double* X, const int64_t* offsets,
                                   int32_t n_sys, const int32_t* c_leafs, hh_tree* out) {
  if (!c_leafs) {
    if (out) *out = nullptr;
    if (ctx) ctx->last_error = "NULL argument";
    return HH_ERR_INVALID_ARG;
  }
  return build_batch(ctx, X, offsets, n_sys, c_leafs, 2, out);
}

hh_status hh_tree_refit(hh_ctx ctx, hh_tree tree, const double* X) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(tree && X, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(tree->ctx == ctx, HH_ERR_INVALID_ARG, "tree belongs to another context");
  hipStream_t st = ctx->stream;
  const int64_t n = tree->n, m = tree->n_nodes, nl = tree->n_leaves;
  int* bad = (int*)ctx->scratch_flag.p;
  HIP_OK(hipMemsetAsync(bad, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_refit_gather, dim3(nblk(n)), dim3(T256), 0, st, X, n,
                     tree->perm.as<int32_t>(), tree->six ? 1 : 0, tree->xs.as<double>(), bad);
  hipLaunchKernelGGL(k_leaf_box, dim3(nblk(nl * 64)), dim3(T256), 0, st,
                     tree->leaves.as<int32_t>(), nl, tree->nodes.as<int4>(), tree->xs.as<double>(),
                     tree->leaf_of.as<int32_t>(), tree->bbox.as<double>());
  hipLaunchKernelGGL(k_inner_box, dim3(nblk(m * 64)), dim3(T256), 0, st, tree->nodes.as<int4>(),
                     m, tree->leaves.as<int32_t>(), nl, tree->bbox.as<double>());
  HIP_OK(hipGetLastError());
  HH_REQUIRE(read_i64(ctx, bad) == 0, HH_ERR_INVALID_ARG, "X holds a non-finite coordinate");
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
