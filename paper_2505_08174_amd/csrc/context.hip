// Context, device memory, kernel handles and host readbacks.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

#include "api_guard.h"
#include "devmath.h"
#include "internal.h"
#include "mlp_mfma.h"

void DevBuf::release() {
  if (p) {
    (void)hipFreeAsync(p, s);
    p = nullptr;
    bytes = 0;
  }
}

void DevBuf::alloc(hipStream_t stream, size_t nbytes) {
  release();
  s = stream;
  if (nbytes == 0) nbytes = 256;
  hipError_t e = hipMallocAsync(&p, nbytes, stream);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw hh_error{HH_ERR_OUT_OF_MEMORY,
                   "device allocation of " + std::to_string(nbytes) + " bytes failed"};
  }
  bytes = nbytes;
}

static hipEvent_t take_event(hh_ctx ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_OK(hipEventCreate(&e));
  return e;
}

PhaseTimer::PhaseTimer(hh_ctx c, int ph, bool on) : ctx(c), phase(ph) {
  if (!on || !ctx->profiling) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return;   // no timing events inside a captured graph
  a = take_event(ctx);
  (void)hipEventRecord(a, ctx->stream);
}

PhaseTimer::~PhaseTimer() {
  if (!a) return;
  hipEvent_t b = nullptr;
  try {
    b = take_event(ctx);
  } catch (...) {
    ctx->event_pool.push_back(a);
    return;
  }
  (void)hipEventRecord(b, ctx->stream);
  ctx->pending.push_back(PhaseRec{phase, a, b});
}

static void drain_phases(hh_ctx ctx) {
  if (ctx->pending.empty()) return;
  ctx_sync(ctx);
  for (auto& r : ctx->pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      ctx->phase_ms[r.phase] += ms;
      ctx->phase_cnt[r.phase] += 1;
    }
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->pending.clear();
}

size_t elem_size(int prec) { return prec == HH_FP64 ? 8 : 4; }

KParams make_kparams(hh_kernel k, bool fp64) {
  KParams kp;
  kp.kind = k->kind;
  kp.input_mode = k->input_mode;
  kp.a = k->a;
  kp.c8 = 1.0 / (8.0 * HH_PI * k->mu);
  kp.c6 = 1.0 / (6.0 * HH_PI * k->mu * k->a);
  kp.alpha1 = k->alpha1;
  kp.alpha2 = k->alpha2;
  kp.w = fp64 ? k->p64.p : k->p32.p;
  return kp;
}

// Device memory of hh_matvec_noalloc: the sorted forces and the near-field
// rows of one product. In host code this name is only a stand-in for the
// symbol; each device's address comes from hipGetSymbolAddress, taken once
// per device when the first context is created on it.
static __device__ __align__(256) unsigned char scratch[HH_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {nullptr};

// This device's copy of the scratch array (the device must be current).
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  HH_REQUIRE(device >= 0 && device < MAX_DEVICES, HH_ERR_INVALID_ARG, "device id out of range");
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HH_REQUIRE(p, HH_ERR_HIP, "no device address for the no-allocation scratch");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

__global__ void k_zero_words(int64_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}
}  // namespace

void zero_words(hh_ctx ctx, void* p, int64_t n) {
  if (n <= 0) return;
  const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)g), dim3(256), 0, ctx->stream, (int64_t*)p, n);
  HIP_OK(hipGetLastError());
}

void ctx_sync(hh_ctx ctx) { HIP_OK(hipStreamSynchronize(ctx->stream)); }

void read_bytes(hh_ctx ctx, void* host, const void* dev, size_t bytes) {
  if (bytes == 0) return;
  HIP_OK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
  ctx_sync(ctx);
}

int64_t read_i64(hh_ctx ctx, const void* dev_ptr) {
  HIP_OK(hipMemcpyAsync(ctx->pinned, dev_ptr, 8, hipMemcpyDeviceToHost, ctx->stream));
  ctx_sync(ctx);
  return ctx->pinned[0];
}

// BF16 round-to-nearest-even of a float, and back.
static uint16_t bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float bf16_val(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
// w = hi + lo with hi, lo BF16
static void bf16_split(double w, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne((float)w);
  lo = bf16_rne((float)(w - (double)bf16_val(hi)));
}

// K slot (8 h + u) of K step s <-> hidden feature, matching the MFMA result
// register order (row 8 (v / 4) + 4 h + v % 4 of register v, v = 8 (s % 2) + u
// of M tile s / 2).
static int kslot_feature(int s, int h, int u) {
  return 32 * (s / 2) + 16 * (s % 2) + 8 * (u / 4) + 4 * h + (u % 4);
}

// Fragment table of the BF16 MFMA MLP (layout in mlp_mfma.h): 16 bytes
// (8 BF16) per lane and fragment.
// Layers 1-3 (those followed by tanh) are stored scaled by 2 log2(e): the
// tile then takes tanh(x) = 1 - 2 / (2^y + 1) straight from the result y.
static std::vector<uint16_t> build_bf16_frags(const double* P0) {
  const int L1 = 0, L2 = L1 + 2 * 64, L3 = L2 + (2 * 4 * 2 + 2) * 64,
            L4 = L3 + (2 * 4 * 2 + 2) * 64, TOTAL = L4 + (4 * 2 + 1) * 64;
  std::vector<uint16_t> fr((size_t)TOTAL * 8, 0);
  auto at = [&](int frag, int u) -> uint16_t& { return fr[(size_t)frag * 8 + u]; };
  const double S = 2.0 / log(2.0);
  std::vector<double> Ps(P0, P0 + MLP_NP);
  for (int i = OFF_W1; i < OFF_W4; ++i) Ps[i] *= S;   // W1, b1, W2, b2, W3, b3
  const double* P = Ps.data();
  const double* W1 = P + OFF_W1;
  const double* b1 = P + OFF_B1;
  for (int mo = 0; mo < 2; ++mo)
    for (int lane = 0; lane < 64; ++lane) {
      int m = 32 * mo + (lane & 31), h = lane >> 5, f = L1 + mo * 64 + lane;
      uint16_t wh[3], wl[3], bh, bl;
      for (int d = 0; d < 3; ++d) bf16_split(W1[3 * m + d], wh[d], wl[d]);
      bf16_split(b1[m], bh, bl);
      if (h == 0) {
        for (int d = 0; d < 3; ++d) { at(f, d) = wh[d]; at(f, 3 + d) = wh[d]; }
        at(f, 6) = bh;
        at(f, 7) = bl;
      } else {
        for (int d = 0; d < 3; ++d) at(f, d) = wl[d];
      }
    }
  auto hidden = [&](int base, const double* W, const double* b, int nrow, int nmo) {
    for (int mo = 0; mo < nmo; ++mo)
      for (int lane = 0; lane < 64; ++lane) {
        int m = 32 * mo + (lane & 31), h = lane >> 5;
        for (int s = 0; s < 4; ++s)
          for (int part = 0; part < 2; ++part) {
            int f = base + ((mo * 4 + s) * 2 + part) * 64 + lane;
            for (int u = 0; u < 8; ++u) {
              if (m >= nrow) continue;
              uint16_t hi, lo;
              bf16_split(W[MLP_H * m + kslot_feature(s, h, u)], hi, lo);
              at(f, u) = part == 0 ? hi : lo;
            }
          }
        int fb = base + (nmo * 4 * 2) * 64 + mo * 64 + lane;
        if (h == 0 && m < nrow) {
          uint16_t hi, lo;
          bf16_split(b[m], hi, lo);
          at(fb, 0) = hi;
          at(fb, 1) = lo;
        }
      }
  };
  hidden(L2, P + OFF_W2, P + OFF_B2, 64, 2);
  hidden(L3, P + OFF_W3, P + OFF_B3, 64, 2);
  hidden(L4, P + OFF_W4, P + OFF_B4, 9, 1);
  return fr;
}

// Fragment table of the FP32 MFMA MLP (layout in mlp_mfma.h): one float per
// lane and K step. Layers 1-3 scaled by 2 log2(e) as for the BF16 table.
std::vector<float> build_f32_frags(const double* P0) {
  std::vector<float> fr((size_t)F32_FRAGS * 64, 0.0f);
  auto at = [&](int frag, int lane) -> float& { return fr[(size_t)frag * 64 + lane]; };
  const double S = 2.0 / log(2.0);
  const double* W1 = P0 + OFF_W1;
  const double* b1 = P0 + OFF_B1;
  // feature contracted by K slot h of step (mo, r)
  auto feat = [](int mo, int r, int h) { return 32 * mo + 8 * (r / 4) + 4 * h + (r % 4); };
  for (int mo = 0; mo < 2; ++mo)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = 32 * mo + (lane & 31), h = lane >> 5;
      at(F32_L1 + 2 * mo, lane) = (float)(S * W1[3 * m + h]);
      at(F32_L1 + 2 * mo + 1, lane) = (float)(S * (h == 0 ? W1[3 * m + 2] : b1[m]));
    }
  auto hidden = [&](int base, const double* W, const double* b) {
    for (int mp = 0; mp < 2; ++mp)
      for (int lane = 0; lane < 64; ++lane) {
        const int m = 32 * mp + (lane & 31), h = lane >> 5;
        for (int mo = 0; mo < 2; ++mo)
          for (int r = 0; r < 16; ++r)
            at(base + (mp * 2 + mo) * 16 + r, lane) = (float)(S * W[MLP_H * m + feat(mo, r, h)]);
        at(base + 64 + mp, lane) = h == 0 ? (float)(S * b[m]) : 0.0f;
      }
  };
  hidden(F32_L2, P0 + OFF_W2, P0 + OFF_B2);
  hidden(F32_L3, P0 + OFF_W3, P0 + OFF_B3);
  for (int lane = 0; lane < 64; ++lane) {
    const int m = lane & 31, h = lane >> 5;
    if (m >= 9) continue;
    for (int mo = 0; mo < 2; ++mo)
      for (int r = 0; r < 16; ++r)
        at(F32_L4 + mo * 16 + r, lane) = (float)P0[OFF_W4 + MLP_H * m + feat(mo, r, h)];
    if (h == 0) at(F32_L4 + 32, lane) = (float)P0[OFF_B4 + m];
  }
  return fr;
}

// Transposed weights of the FP32 MFMA backward (layout in backward_mfma.hip),
// unscaled: [W4^T: mo' 2][s 5], [W3^T: mo' 2][mo 2][r 16], [W2^T: same],
// then W1 by feature [d 3][64].
static std::vector<float> build_f32_bwd(const double* P0) {
  const int B4 = 0, B3 = 10, B2 = 74, B1 = 138, NF = 141;
  std::vector<float> fr((size_t)NF * 64, 0.0f);
  auto at = [&](int frag, int lane) -> float& { return fr[(size_t)frag * 64 + lane]; };
  auto feat = [](int mo, int r, int h) { return 32 * mo + 8 * (r / 4) + 4 * h + (r % 4); };
  for (int mp = 0; mp < 2; ++mp)
    for (int lane = 0; lane < 64; ++lane) {
      const int col = 32 * mp + (lane & 31), h = lane >> 5;
      for (int s = 0; s < 5; ++s) {
        const int m = 2 * s + h;
        if (m < 9) at(B4 + mp * 5 + s, lane) = (float)P0[OFF_W4 + MLP_H * m + col];
      }
      for (int mo = 0; mo < 2; ++mo)
        for (int r = 0; r < 16; ++r) {
          const int f = feat(mo, r, h);
          at(B3 + (mp * 2 + mo) * 16 + r, lane) = (float)P0[OFF_W3 + MLP_H * f + col];
          at(B2 + (mp * 2 + mo) * 16 + r, lane) = (float)P0[OFF_W2 + MLP_H * f + col];
        }
    }
  for (int d = 0; d < 3; ++d)
    for (int f = 0; f < 64; ++f) at(B1 + d, f) = (float)P0[OFF_W1 + 3 * f + d];
  return fr;
}

extern "C" {

hh_status hh_ctx_create(int device, void* stream, hh_ctx* out) {
  if (!out) return HH_ERR_INVALID_ARG;
  *out = nullptr;
  hh_ctx ctx = new (std::nothrow) hh_ctx_s();
  if (!ctx) return HH_ERR_OUT_OF_MEMORY;
  try {
    int n = 0;
    HIP_OK(hipGetDeviceCount(&n));
    HH_REQUIRE(device >= 0 && device < n, HH_ERR_INVALID_ARG, "no such HIP device");
    HIP_OK(hipSetDevice(device));
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    HIP_OK(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device));
    ctx->noalloc_scratch = scratch_address(device);
    HIP_OK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming));
    // keep freed blocks in the stream-ordered pool for reuse across steps
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    size_t fr = 0, tot = 0;
    HIP_OK(hipMemGetInfo(&fr, &tot));
    ctx->budget_bytes = (size_t)(0.4 * (double)fr);
    ctx->scratch_flag.alloc(ctx->stream, 64 * sizeof(int64_t));
    HIP_OK(hipHostMalloc((void**)&ctx->pinned, 64 * sizeof(int64_t), hipHostMallocDefault));
  } catch (const hh_error& e) {
    delete ctx;
    return e.st;
  } catch (const std::bad_alloc&) {
    delete ctx;
    return HH_ERR_OUT_OF_MEMORY;
  }
  *out = ctx;
  return HH_OK;
}

void hh_ctx_destroy(hh_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  ctx->scratch_flag.release();
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

const char* hh_last_error(hh_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

hh_status hh_ctx_set_stream(hh_ctx ctx, void* stream) {
  if (!ctx) return HH_ERR_INVALID_ARG;
  ctx->stream = (hipStream_t)stream;
  return HH_OK;
}

hh_status hh_ctx_set_budget(hh_ctx ctx, size_t bytes) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(bytes >= 4096, HH_ERR_INVALID_ARG, "budget must be at least 4096 bytes");
  ctx->budget_bytes = bytes;
  HH_API_END(ctx)
}

hh_status hh_ctx_set_team_min(hh_ctx ctx, int32_t team_min) {
  HH_API_BEGIN(ctx)
  HH_REQUIRE(team_min >= 64 && team_min <= (1 << 30), HH_ERR_INVALID_ARG,
             "team_min must be in [64, 2^30]");
  int cls = 0;
  while ((1 << cls) < team_min) ++cls;
  ctx->team_cls = cls;
  HH_API_END(ctx)
}

hh_status hh_ctx_set_profiling(hh_ctx ctx, int on) {
  HH_API_BEGIN(ctx)
  ctx->profiling = on != 0;
  HH_API_END(ctx)
}

hh_status hh_ctx_phase_times(hh_ctx ctx, double* ms, int64_t* count, int reset) {
  HH_API_BEGIN(ctx)
  drain_phases(ctx);
  for (int i = 0; i < HH_NPHASE; ++i) {
    if (ms) ms[i] = ctx->phase_ms[i];
    if (count) count[i] = ctx->phase_cnt[i];
    if (reset) {
      ctx->phase_ms[i] = 0;
      ctx->phase_cnt[i] = 0;
    }
  }
  HH_API_END(ctx)
}

hh_status hh_synchronize(hh_ctx ctx) {
  HH_API_BEGIN(ctx)
  ctx_sync(ctx);
  HH_API_END(ctx)
}

hh_status hh_kernel_create_rpy(hh_ctx ctx, double a, double mu, hh_kernel* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out, HH_ERR_INVALID_ARG, "out is NULL");
  HH_REQUIRE(a > 0 && mu > 0 && isfinite(a) && isfinite(mu), HH_ERR_INVALID_ARG,
             "RPY kernel needs a > 0 and mu > 0");
  hh_kernel k = new hh_kernel_s();
  k->ctx = ctx;
  k->kind = KIND_RPY;
  k->a = a;
  k->mu = mu;
  k->alpha1 = 1.0 / (6.0 * M_PI * mu * a);
  k->alpha2 = k->alpha1;
  *out = k;
  HH_API_END(ctx)
}

hh_status hh_kernel_create_rpy6(hh_ctx ctx, double a, double mu, hh_kernel* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out, HH_ERR_INVALID_ARG, "out is NULL");
  HH_REQUIRE(a > 0 && mu > 0 && isfinite(a) && isfinite(mu), HH_ERR_INVALID_ARG,
             "RPY kernel needs a > 0 and mu > 0");
  hh_kernel k = new hh_kernel_s();
  k->ctx = ctx;
  k->kind = KIND_RPY6;
  k->a = a;
  k->mu = mu;
  k->alpha1 = 1.0 / (6.0 * M_PI * mu * a);
  k->alpha2 = 1.0 / (8.0 * M_PI * mu * a * a * a);
  *out = k;
  HH_API_END(ctx)
}

hh_status hh_kernel_create_mlp(hh_ctx ctx, const double* params, int input_mode, double a,
                               double mu, hh_kernel* out) {
  if (out) *out = nullptr;
  HH_API_BEGIN(ctx)
  HH_REQUIRE(out && params, HH_ERR_INVALID_ARG, "NULL argument");
  HH_REQUIRE(input_mode == HH_MLP_INPUT_DIRECTION || input_mode == HH_MLP_INPUT_DISPLACEMENT,
             HH_ERR_INVALID_ARG, "unknown MLP input mode");
  HH_REQUIRE(a > 0 && mu > 0, HH_ERR_INVALID_ARG, "MLP kernel needs a > 0 and mu > 0");
  for (int i = 0; i < MLP_NP; ++i)
    HH_REQUIRE(isfinite(params[i]), HH_ERR_INVALID_ARG, "non-finite MLP parameter");
  hh_kernel_s* k = new hh_kernel_s();
  try {
    k->ctx = ctx;
    k->kind = KIND_MLP;
    k->input_mode = input_mode;
    k->a = a;
    k->mu = mu;
    k->alpha1 = 1.0 / (6.0 * M_PI * mu * a);
    k->alpha2 = k->alpha1;
    k->host_params.assign(params, params + MLP_NP);
    std::vector<float> p32(params, params + MLP_NP);
    std::vector<uint16_t> fr = build_bf16_frags(params);
    k->pbf.alloc(ctx->stream, fr.size() * sizeof(uint16_t));
    HIP_OK(hipMemcpyAsync(k->pbf.p, fr.data(), fr.size() * sizeof(uint16_t),
                          hipMemcpyHostToDevice, ctx->stream));
    std::vector<float> f32 = build_f32_frags(params);
    k->pf32.alloc(ctx->stream, f32.size() * sizeof(float));
    HIP_OK(hipMemcpyAsync(k->pf32.p, f32.data(), f32.size() * sizeof(float),
                          hipMemcpyHostToDevice, ctx->stream));
    std::vector<float> f32t = build_f32_bwd(params);
    k->pf32t.alloc(ctx->stream, f32t.size() * sizeof(float));
    HIP_OK(hipMemcpyAsync(k->pf32t.p, f32t.data(), f32t.size() * sizeof(float),
                          hipMemcpyHostToDevice, ctx->stream));
    k->p64.alloc(ctx->stream, MLP_NP * sizeof(double));
    k->p32.alloc(ctx->stream, MLP_NP * sizeof(float));
    HIP_OK(hipMemcpyAsync(k->p64.p, params, MLP_NP * sizeof(double), hipMemcpyHostToDevice,
                          ctx->stream));
    HIP_OK(hipMemcpyAsync(k->p32.p, p32.data(), MLP_NP * sizeof(float), hipMemcpyHostToDevice,
                          ctx->stream));
    ctx_sync(ctx);
  } catch (...) {
    delete k;
    throw;
  }
  *out = k;
  HH_API_END(ctx)
}

void hh_kernel_free(hh_kernel k) {
  if (!k) return;
  delete k;
}

int hh_device_arch_ok(void) {
  hipDeviceProp_t p;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
  return strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

}  // extern "C"
