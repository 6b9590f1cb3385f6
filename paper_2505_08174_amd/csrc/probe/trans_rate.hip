// Throughput of the VALU transcendental operations that bound the MLP tile
// (v_exp_f32, v_rcp_f32) against FP32 FMA: every lane runs 16 independent
// chains of one operation, eight 256-thread workgroups per compute unit.
// Prints lane-operations per clock per CU at the nominal clock. Not part of
// the library; it supports the activation ceiling that bench.py reports.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o trans_rate trans_rate.hip && ./trans_rate
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHAINS 16

template <int OP>
__global__ __launch_bounds__(256) void k_chain(float* out, int iters, float s) {
  float x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = s * (threadIdx.x + c) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
      if (OP == 0) x[c] = __builtin_amdgcn_exp2f(x[c]);
      else if (OP == 1) x[c] = __builtin_amdgcn_rcpf(x[c]);
      else x[c] = __builtin_fmaf(x[c], s, 0.5f);
    }
  }
  float r = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) r += x[c];
  out[blockIdx.x * 256 + threadIdx.x] = r;
}

int main() {
  int ncu = 0, khz = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, 0) != hipSuccess) {
    fprintf(stderr, "no HIP device\n");
    return 1;
  }
  const int blocks = ncu * 8, iters = 4096;
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return 1;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const char* name[3] = {"v_exp_f32", "v_rcp_f32", "v_fma_f32"};
  for (int rep = 0; rep < 2; ++rep)
    for (int op = 0; op < 3; ++op) {
      (void)hipEventRecord(a);
      if (op == 0) hipLaunchKernelGGL(k_chain<0>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f);
      if (op == 1) hipLaunchKernelGGL(k_chain<1>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f);
      if (op == 2) hipLaunchKernelGGL(k_chain<2>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f);
      (void)hipEventRecord(b);
      (void)hipEventSynchronize(b);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, a, b);
      const double ops = (double)blocks * 256 * iters * CHAINS;
      if (rep == 1)
        printf("%s: %.3f ms, %.3e lane-ops/s, %.1f lane-ops per clock per CU at %d MHz (%d CUs)\n",
               name[op], ms, ops / (ms * 1e-3), ops / (ms * 1e-3) / ncu / (khz * 1e3), khz / 1000,
               ncu);
    }
  (void)hipFree(out);
  return 0;
}
