// Block partition, Algorithm 1, with the admissibility condition Eq. (7).
//
// The recursion of Algorithm 1 is run breadth-first: a frontier of candidate
// blocks (tau, sigma) starts at (root, root); each level classifies every
// candidate (admissible -> P^G; both leaves -> P^H; else split the non-leaf
// side(s) into 2 or 4 sons) and compacts the three outcomes with prefix sums.
// The order of visits does not change the resulting sets, which are sorted by
// (tau, sigma) at the end.
//
// Eq. (7) on tight bounding boxes: diam^2 = (dx*dx + dy*dy) + dz*dz, the gap
// per axis g = max(0, lo_s - hi_t, lo_t - hi_s), dist^2 = (gx*gx + gy*gy) +
// gz*gz; admissible iff dist^2 > 0 and max(diam_t^2, diam_s^2) <= (eta*eta)
// dist^2. FP64, no contraction, fixed order (the result is exact-reproducible).
#include "api_guard.h"
#include "internal.h"

#pragma clang fp contract(off)

namespace {

constexpr int T256 = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + T256 - 1) / T256); }

__device__ __forceinline__ double diam2(const double* b) {
  double dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ double dist2(const double* t, const double* s) {
  double g[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) g[d] = fmax(0.0, fmax(s[d] - t[d + 3], t[d] - s[d + 3]));
  return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
}

// cls: 0 -> admissible (G), 1 -> leaf pair (H), 2 -> split
__global__ __launch_bounds__(T256) void k_classify(const int2* __restrict__ fr, int64_t nf,
                                                   const int4* __restrict__ nodes,
                                                   const double* __restrict__ bbox, double eta2,
                                                   int dense_mode, int64_t* __restrict__ cG,
                                                   int64_t* __restrict__ cH,
                                                   int64_t* __restrict__ cN) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= nf) return;
  int2 b = fr[i];
  int4 nt = nodes[b.x], ns = nodes[b.y];
  const double* bt = bbox + 6 * (int64_t)b.x;
  const double* bs = bbox + 6 * (int64_t)b.y;
  int64_t g = 0, h = 0, nx = 0;
  bool adm = false;
  if (!dense_mode) {
    double d2 = dist2(bt, bs);
    adm = d2 > 0.0 && fmax(diam2(bt), diam2(bs)) <= eta2 * d2;
  }
  bool lt = nt.z < 0, ls = ns.z < 0;
  if (adm) g = 1;
  else if (lt && ls) h = 1;
  else nx = (lt || ls) ? 2 : 4;
  cG[i] = g;
  cH[i] = h;
  cN[i] = nx;
}

__global__ __launch_bounds__(T256) void k_emit(const int2* __restrict__ fr, int64_t nf,
                                               const int4* __restrict__ nodes,
                                               const int64_t* __restrict__ cG,
                                               const int64_t* __restrict__ pG,
                                               const int64_t* __restrict__ cH,
                                               const int64_t* __restrict__ pH,
                                               const int64_t* __restrict__ cN,
                                               const int64_t* __restrict__ pN,
                                               int2* __restrict__ G, int2* __restrict__ H,
                                               int2* __restrict__ next) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= nf) return;
  int2 b = fr[i];
  if (cG[i]) { G[pG[i]] = b; return; }
  if (cH[i]) { H[pH[i]] = b; return; }
  int4 nt = nodes[b.x], ns = nodes[b.y];
  int64_t o = pN[i];
  if (ns.z < 0) {            // sigma is a leaf: split tau
    next[o] = make_int2(nt.z, b.y);
    next[o + 1] = make_int2(nt.w, b.y);
  } else if (nt.z < 0) {     // tau is a leaf: split sigma
    next[o] = make_int2(b.x, ns.z);
    next[o + 1] = make_int2(b.x, ns.w);
  } else {
    next[o] = make_int2(nt.z, ns.z);
    next[o + 1] = make_int2(nt.z, ns.w);
    next[o + 2] = make_int2(nt.w, ns.z);
    next[o + 3] = make_int2(nt.w, ns.w);
  }
  (void)cN;
}

__global__ __launch_bounds__(T256) void k_pack(const int2* __restrict__ L, int64_t m, int nb,
                                               uint64_t* __restrict__ key,
                                               uint32_t* __restrict__ val) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= m) return;
  int2 b = L[i];
  key[i] = ((uint64_t)b.x << nb) | (uint64_t)b.y;
  val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(T256) void k_unpack(const uint64_t* __restrict__ key, int64_t m,
                                                 int nb, int2* __restrict__ L) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (i >= m) return;
  uint64_t k = key[i];
  L[i] = make_int2((int)(k >> nb), (int)(k & ((1ull << nb) - 1)));
}

__global__ __launch_bounds__(T256) void k_near_ptr(const int2* __restrict__ H, int64_t nH,
                                                   const int32_t* __restrict__ leaf_id,
                                                   int64_t nl, int32_t* __restrict__ ptr) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p > nH) return;
  if (p == nH) { ptr[nl] = (int32_t)nH; return; }
  if (p == 0 || H[p - 1].x != H[p].x) ptr[leaf_id[H[p].x]] = (int32_t)p;
}

__global__ __launch_bounds__(T256) void k_far_ptr(const int2* __restrict__ G, int64_t nG,
                                                  int64_t m, int32_t* __restrict__ ptr) {
  int64_t p = (int64_t)blockIdx.x * T256 + threadIdx.x;
  if (p > m) return;
  int64_t a = 0, b = nG;
  while (a < b) {
    int64_t mid = (a + b) / 2;
    if (G[mid].x < p) a = mid + 1; else b = mid;
  }
  ptr[p] = (int32_t)a;
}

__global__ __launch_bounds__(T256) void k_pair_sizes(const int2* __restrict__ L, int64_t m,
                                                     const int4* __restrict__ nodes,
                                                     unsigned long long* __restrict__ sum) {
  int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x;
  unsigned long long v = 0;
  if (i < m) {
    int2 b = L[i];
    int4 a = nodes[b.x], c = nodes[b.y];
    v = (unsigned long long)(a.y - a.x) * (unsigned long long)(c.y - c.x);
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(sum, v);
}

__global__ void k_roots_frontier(const int32_t* __restrict__ roots, int nsys,
                                 int2* __restrict__ fr) {
  int s = blockIdx.x * 256 + threadIdx.x;
  if (s < nsys) fr[s] = make_int2(roots[s], roots[s]);
}

}  // namespace

static void sort_pairs(hh_ctx ctx, DevBuf& L, int64_t m, int nb) {
  if (m <= 1) return;
  hipStream_t st = ctx->stream;
  DevBuf key, val;
  key.alloc(st, m * sizeof(uint64_t));
  val.alloc(st, m * sizeof(uint32_t));
  hipLaunchKernelGGL(k_pack, dim3(nblk(m)), dim3(T256), 0, st, L.as<int2>(), m, nb,
                     key.as<uint64_t>(), val.as<uint32_t>());
  radix_sort_u64(ctx, key.as<uint64_t>(), val.as<uint32_t>(), m, 2 * nb);
  hipLaunchKernelGGL(k_unpack, dim3(nblk(m)), dim3(T256), 0, st, key.as<uint64_t>(), m, nb,
                     L.as<int2>());
  HIP_OK(hipGetLastError());
}

extern "C" {

hh_status hh_partition(hh_ctx ctx, hh_tree tree, double eta, int dense_mode, hh_part* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && tree, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(eta > 0.0 && eta < INFINITY, HH_ERR_INVALID_ARG, "eta must be > 0 (Eq. (7))");
  HH_REQUIRE(tree->ctx == ctx, HH_ERR_INVALID_ARG, "tree belongs to another context");
  hipStream_t st = ctx->stream;
  PhaseTimer timer(ctx, HH_PHASE_PARTITION);
  hh_part_s* p = new hh_part_s();
  try {
    p->ctx = ctx;
    p->tree = tree;
    const int4* nodes = tree->nodes.as<int4>();
    const double* bbox = tree->bbox.as<double>();
    double eta2 = eta * eta;
    std::vector<DevBuf*> gl, hl;
    std::vector<int64_t> gn, hn;
    // Algorithm 1 starts at (I, I) for every independent system
    DevBuf* fr = new DevBuf();
    const int nsys = tree->n_sys;
    fr->alloc(st, nsys * sizeof(int2));
    hipLaunchKernelGGL(k_roots_frontier, dim3((nsys + 255) / 256), dim3(256), 0, st,
                       tree->roots.as<int32_t>(), nsys, fr->as<int2>());
    int64_t nf = nsys;
    int64_t totG = 0, totH = 0;
    try {
      for (int level = 0; nf > 0; ++level) {
        HH_REQUIRE(level < 200, HH_ERR_CAPACITY, "partition deeper than 200 levels");
        DevBuf cG, cH, cN, pG, pH, pN;
        for (DevBuf* b : {&cG, &cH, &cN, &pG, &pH, &pN}) b->alloc(st, (nf + 1) * sizeof(int64_t));
        for (DevBuf* b : {&cG, &cH, &cN})
          HIP_OK(hipMemsetAsync(b->as<int64_t>() + nf, 0, sizeof(int64_t), st));
        hipLaunchKernelGGL(k_classify, dim3(nblk(nf)), dim3(T256), 0, st, fr->as<int2>(), nf,
                           nodes, bbox, eta2, dense_mode, cG.as<int64_t>(), cH.as<int64_t>(),
                           cN.as<int64_t>());
        scan_exclusive_i64(ctx, cG.as<int64_t>(), pG.as<int64_t>(), nf + 1);
        scan_exclusive_i64(ctx, cH.as<int64_t>(), pH.as<int64_t>(), nf + 1);
        scan_exclusive_i64(ctx, cN.as<int64_t>(), pN.as<int64_t>(), nf + 1);
        HIP_OK(hipMemcpyAsync(ctx->pinned, pG.as<int64_t>() + nf, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(ctx->pinned + 1, pH.as<int64_t>() + nf, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(ctx->pinned + 2, pN.as<int64_t>() + nf, 8, hipMemcpyDeviceToHost, st));
        ctx_sync(ctx);
        int64_t ng = ctx->pinned[0], nh = ctx->pinned[1], nn = ctx->pinned[2];
        HH_REQUIRE(totG + ng < (1ll << 31) && totH + nh < (1ll << 31) && nn < (1ll << 31),
                   HH_ERR_CAPACITY, "block lists exceed 2^31 entries");
        DevBuf* g = new DevBuf();
        DevBuf* h = new DevBuf();
        DevBuf* nx = new DevBuf();
        gl.push_back(g);
        hl.push_back(h);
        gn.push_back(ng);
        hn.push_back(nh);
        g->alloc(st, std::max<int64_t>(1, ng) * sizeof(int2));
        h->alloc(st, std::max<int64_t>(1, nh) * sizeof(int2));
        try {
          nx->alloc(st, std::max<int64_t>(1, nn) * sizeof(int2));
        } catch (...) {
          delete nx;
          throw;
        }
        hipLaunchKernelGGL(k_emit, dim3(nblk(nf)), dim3(T256), 0, st, fr->as<int2>(), nf, nodes,
                           cG.as<int64_t>(), pG.as<int64_t>(), cH.as<int64_t>(),
                           pH.as<int64_t>(), cN.as<int64_t>(), pN.as<int64_t>(), g->as<int2>(),
                           h->as<int2>(), nx->as<int2>());
        HIP_OK(hipGetLastError());
        delete fr;
        fr = nx;
        nf = nn;
        totG += ng;
        totH += nh;
      }
      p->nG = totG;
      p->nH = totH;
      p->G.alloc(st, std::max<int64_t>(1, totG) * sizeof(int2));
      p->H.alloc(st, std::max<int64_t>(1, totH) * sizeof(int2));
      int64_t og = 0, oh = 0;
      for (size_t i = 0; i < gl.size(); ++i) {
        if (gn[i])
          HIP_OK(hipMemcpyAsync(p->G.as<int2>() + og, gl[i]->p, gn[i] * sizeof(int2),
                                hipMemcpyDeviceToDevice, st));
        if (hn[i])
          HIP_OK(hipMemcpyAsync(p->H.as<int2>() + oh, hl[i]->p, hn[i] * sizeof(int2),
                                hipMemcpyDeviceToDevice, st));
        og += gn[i];
        oh += hn[i];
      }
    } catch (...) {
      delete fr;
      for (auto* b : gl) delete b;
      for (auto* b : hl) delete b;
      throw;
    }
    delete fr;
    for (auto* b : gl) delete b;
    for (auto* b : hl) delete b;
    int nb = 1;
    while ((1ll << nb) < tree->n_nodes) ++nb;
    sort_pairs(ctx, p->G, p->nG, nb);
    sort_pairs(ctx, p->H, p->nH, nb);
    p->near_ptr.alloc(st, (tree->n_leaves + 1) * sizeof(int32_t));
    p->far_ptr.alloc(st, (tree->n_nodes + 1) * sizeof(int32_t));
    hipLaunchKernelGGL(k_near_ptr, dim3(nblk(p->nH + 1)), dim3(T256), 0, st, p->H.as<int2>(),
                       p->nH, tree->leaf_id.as<int32_t>(), tree->n_leaves,
                       p->near_ptr.as<int32_t>());
    hipLaunchKernelGGL(k_far_ptr, dim3(nblk(tree->n_nodes + 1)), dim3(T256), 0, st,
                       p->G.as<int2>(), p->nG, tree->n_nodes, p->far_ptr.as<int32_t>());
    unsigned long long* sums = (unsigned long long*)ctx->scratch_flag.p;
    HIP_OK(hipMemsetAsync(sums, 0, 2 * sizeof(unsigned long long), st));
    if (p->nH)
      hipLaunchKernelGGL(k_pair_sizes, dim3(nblk(p->nH)), dim3(T256), 0, st, p->H.as<int2>(),
                         p->nH, nodes, sums);
    if (p->nG)
      hipLaunchKernelGGL(k_pair_sizes, dim3(nblk(p->nG)), dim3(T256), 0, st, p->G.as<int2>(),
                         p->nG, nodes, sums + 1);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(ctx->pinned, sums, 16, hipMemcpyDeviceToHost, st));
    ctx_sync(ctx);
    p->near_pairs = ctx->pinned[0];
    p->far_entries = ctx->pinned[1];
  } catch (...) {
    delete p;
    throw;
  }
  *out = p;
  HH_API_END(ctx)
}

void hh_part_free(hh_part p) { delete p; }

hh_status hh_part_info(hh_part p, int64_t* nG, int64_t* nH) {
  if (!p) return HH_ERR_INVALID_ARG;
  if (nG) *nG = p->nG;
  if (nH) *nH = p->nH;
  return HH_OK;
}

hh_status hh_part_stats(hh_part p, int64_t* near_pairs, int64_t* far_entries) {
  if (!p) return HH_ERR_INVALID_ARG;
  if (near_pairs) *near_pairs = p->near_pairs;
  if (far_entries) *far_entries = p->far_entries;
  return HH_OK;
}

hh_status hh_part_export(hh_part p, int32_t* G, int32_t* H) {
  if (!p) return HH_ERR_INVALID_ARG;
  hh_ctx ctx = p->ctx;
  HH_API_BEGIN(ctx)
  if (G) read_bytes(ctx, G, p->G.p, p->nG * sizeof(int2));
  if (H) read_bytes(ctx, H, p->H.p, p->nH * sizeof(int2));
  HH_API_END(ctx)
}

}  // extern "C"
