// Device-wide exclusive scan and stable LSD radix sort (8-bit digits).
//
// Radix pass: (1) each 256-thread block counts the digits of its 4096-item
// tile in LDS and writes a digit-major histogram; (2) one exclusive scan over
// all (digit, tile) counts gives every tile its output base per digit;
// (3) each block re-reads its tile in 16 rounds of 256 consecutive items and
// ranks each item among equal digits with 8 wave ballots (a wave-wide match),
// adding the counts of earlier waves and earlier rounds, which keeps the pass
// stable.
#include "internal.h"

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[SCAN_T / 64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan(v, lane);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int64_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_T / 64; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const int64_t* __restrict__ in,
                                                        int64_t n, int64_t* __restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  int64_t tot;
  (void)block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of `m` tile sums by one block, in place.
__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(int64_t* __restrict__ sums, int64_t m) {
  int64_t carry = 0;
  for (int64_t base = 0; base < m; base += SCAN_T) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < m ? sums[i] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, &tot);
    if (i < m) sums[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_down(const int64_t* __restrict__ in, int64_t n,
                                                      const int64_t* __restrict__ sums,
                                                      int64_t* __restrict__ out) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t ex = block_excl_scan(s, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

constexpr int RS_T = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_T * RS_ROUNDS;

__global__ __launch_bounds__(RS_T) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                     int shift, int64_t nblocks,
                                                     int64_t* __restrict__ hist) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + r * RS_T + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(RS_T) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, int64_t nblocks,
    const int64_t* __restrict__ offs) {
  __shared__ int64_t base[256];
  __shared__ int run[256];
  __shared__ int wcnt[RS_T / 64][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  run[threadIdx.x] = 0;
  for (int i = 0; i < RS_T / 64; ++i) wcnt[i][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t tile = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = tile + r * RS_T + threadIdx.x;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    uint32_t val = valid ? vin[i] : 0;
    int d = (int)((key >> shift) & 255);
    uint64_t vb = __ballot(valid);
    uint64_t m = valid ? vb : ~vb;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot((d >> b) & 1);
      m &= ((d >> b) & 1) ? bal : ~bal;
    }
    int rank = __popcll(m & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int64_t pos = base[d] + run[d] + rank;
      for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int ww = 0; ww < RS_T / 64; ++ww) {
      add += wcnt[ww][threadIdx.x];
      wcnt[ww][threadIdx.x] = 0;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

void scan_exclusive_i64(hh_ctx ctx, const int64_t* in, int64_t* out, int64_t n) {
  if (n <= 0) return;
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  DevBuf sums;
  sums.alloc(ctx->stream, tiles * sizeof(int64_t));
  hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(SCAN_T), 0, ctx->stream, in, n,
                     sums.as<int64_t>());
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(SCAN_T), 0, ctx->stream, sums.as<int64_t>(),
                     tiles);
  hipLaunchKernelGGL(k_scan_down, dim3(tiles), dim3(SCAN_T), 0, ctx->stream, in, n,
                     sums.as<int64_t>(), out);
  HIP_OK(hipGetLastError());
}

void radix_sort_u64(hh_ctx ctx, uint64_t* keys, uint32_t* vals, int64_t n, int bits) {
  if (n <= 1) return;
  int passes = (bits + 7) / 8;
  int64_t nblocks = (n + RS_TILE - 1) / RS_TILE;
  DevBuf k2, v2, hist;
  k2.alloc(ctx->stream, n * sizeof(uint64_t));
  v2.alloc(ctx->stream, n * sizeof(uint32_t));
  hist.alloc(ctx->stream, 256 * nblocks * sizeof(int64_t));
  uint64_t *ka = keys, *kb = k2.as<uint64_t>();
  uint32_t *va = vals, *vb = v2.as<uint32_t>();
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(RS_T), 0, ctx->stream, ka, n, shift,
                       nblocks, hist.as<int64_t>());
    scan_exclusive_i64(ctx, hist.as<int64_t>(), hist.as<int64_t>(), 256 * nblocks);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(RS_T), 0, ctx->stream, ka, va, kb,
                       vb, n, shift, nblocks, hist.as<int64_t>());
    HIP_OK(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    HIP_OK(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
  }
}
