// probe.hip -- issue-rate probes of the VALU instruction classes the
// kernels are built from, so that measured rooflines can be stated against
// what this chip sustains as well as against its published peak: fp64 FMA
// (the residue arithmetic below 2^42 and its transforms), v_mad_u64_u32 (the
// 64-bit integer products of the 60-bit primes) and 32-bit integer adds.
// Each lane runs kChains independent dependency chains, so the rate is
// bounded by issue, not by latency.
#include "internal.hpp"

namespace sfhe {

constexpr int kChains = 8;

__global__ void __launch_bounds__(256) probe_fma_kernel(double* sink, int64_t iters, double a, double b) {
  double x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (double)(threadIdx.x + c);
  for (int64_t i = 0; i < iters; ++i)
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  double s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == 1.0) sink[threadIdx.x] = s;   // never true for the probe's inputs; keeps the chains live
}

__global__ void __launch_bounds__(256) probe_mad64_kernel(u64* sink, int64_t iters, u32 a, u64 b) {
  u64 x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x + c;
  for (int64_t i = 0; i < iters; ++i)
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (u64)(u32)x[c] * a + b;
  u64 s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c];
  if (s == 1) sink[threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) probe_add32_kernel(u32* sink, int64_t iters, u32 a) {
  u32 x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7 + c;
  for (int64_t i = 0; i < iters; ++i)
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (x[c] + a) ^ (u32)(c + 1);
  u32 s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == 1u) sink[threadIdx.x] = s;
}

}  // namespace sfhe

using namespace sfhe;

extern "C" {

int sfhe_probe_valu(int32_t kind, double* lane_ops_per_s) {
  if (!lane_ops_per_s || kind < 0 || kind > 2) { set_error("bad probe kind or NULL output"); return SFHE_E_INVALID_ARG; }
  *lane_ops_per_s = 0;
  hipDeviceProp_t prop;
  int dev = 0;
  SFHE_HIP(hipGetDevice(&dev));
  SFHE_HIP(hipGetDeviceProperties(&prop, dev));
  const int blocks = prop.multiProcessorCount * 32;   // 32 waves of 256 lanes' worth per CU
  const int64_t iters = 4096;
  void* sink = nullptr;
  SFHE_HIP(hipMalloc(&sink, 256 * sizeof(u64)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SFHE_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = SFHE_E_DEVICE;
  float ms = 0;
  for (int rep = 0; rep < 2 && !rc; ++rep) {   // the first run loads the code object
    (void)hipEventRecord(e0, nullptr);
    if (kind == 0)
      hipLaunchKernelGGL(probe_fma_kernel, dim3(blocks), dim3(256), 0, nullptr, (double*)sink, iters, 0.999999, 1e-9);
    else if (kind == 1)
      hipLaunchKernelGGL(probe_mad64_kernel, dim3(blocks), dim3(256), 0, nullptr, (u64*)sink, iters, 2654435761u,
                         12345ull);
    else
      hipLaunchKernelGGL(probe_add32_kernel, dim3(blocks), dim3(256), 0, nullptr, (u32*)sink, iters, 0x9E3779B9u);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = SFHE_E_DEVICE;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (rc) { set_error("probe launch failed"); return rc; }
  // the add probe issues two instructions (add, xor) per chain step
  const double per_step = kind == 2 ? 2.0 : 1.0;
  *lane_ops_per_s = (double)blocks * 256.0 * (double)iters * kChains * per_step / (ms * 1e-3);
  return SFHE_OK;
}

}  // extern "C"
