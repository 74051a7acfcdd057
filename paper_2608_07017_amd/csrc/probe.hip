// Issue-rate probe of the vector ALU: the lane-operation rate that bounds
// the walker (its roofline's peak).  Every lane runs eight independent
// dependency chains of one instruction kind over the whole chip, so the
// rate measured is the issue rate, not the latency.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wos.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 16;

template <int OP>
__global__ __launch_bounds__(kProbeBlock) void probe_kernel(int iters, uint32_t seed, uint32_t* out) {
  const uint32_t t = blockIdx.x * kProbeBlock + threadIdx.x;
  uint32_t u[kChains];
  float f[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    u[c] = t * 2654435761u + seed + c;
    f[c] = (float)(u[c] & 1023) * 1e-3f;
  }
  const float fa = 1.0000001f, fb = 1e-7f;
  const uint32_t ua = seed | 1u;
#pragma unroll 8
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      // an empty statement that takes the integer value in a vector register
      // after every step: it emits nothing, and keeps the compiler from
      // folding a chain of additions or products into one
      if constexpr (OP == WOS_PROBE_FMA_F32) {
        f[c] = __builtin_fmaf(f[c], fa, fb);
      } else if constexpr (OP == WOS_PROBE_ADD_U32) {
        u[c] = u[c] + ua;
        asm volatile("" : "+v"(u[c]));
      } else if constexpr (OP == WOS_PROBE_SIN_F32) {
        f[c] = __builtin_amdgcn_sinf(f[c]);
      } else if constexpr (OP == WOS_PROBE_MUL_U32) {
        u[c] = u[c] * ua;
        asm volatile("" : "+v"(u[c]));
      } else {  // WOS_PROBE_MUL_WIDE_U32: the 32 x 32 -> 64 product of Philox
        const uint64_t pr = (uint64_t)u[c] * ua;
        u[c] = (uint32_t)pr ^ (uint32_t)(pr >> 32);
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc ^= u[c] ^ __float_as_uint(f[c]);
  out[t] = acc;
}

}  // namespace

extern "C" wos_status wos_probe_valu(int32_t op, int32_t iters, double* lane_ops_per_s, void* stream_) {
  if (!lane_ops_per_s || iters < 1) return WOS_EINVAL;
  if (op < WOS_PROBE_FMA_F32 || op > WOS_PROBE_MUL_WIDE_U32) return WOS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream_);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return WOS_EDEVICE;
  const int blocks = cus * 32;  // 32 workgroups of 4 waves per compute unit
  const size_t threads = (size_t)blocks * kProbeBlock;
  uint32_t* out = nullptr;
  if (hipMalloc(&out, threads * sizeof(uint32_t)) != hipSuccess) return WOS_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  wos_status s = WOS_OK;
  float ms = 0.0f;
  auto launch = [&](int it) {
    switch (op) {
      case WOS_PROBE_FMA_F32: hipLaunchKernelGGL(probe_kernel<WOS_PROBE_FMA_F32>, dim3(blocks), dim3(kProbeBlock), 0, st, it, 7u, out); break;
      case WOS_PROBE_ADD_U32: hipLaunchKernelGGL(probe_kernel<WOS_PROBE_ADD_U32>, dim3(blocks), dim3(kProbeBlock), 0, st, it, 7u, out); break;
      case WOS_PROBE_SIN_F32: hipLaunchKernelGGL(probe_kernel<WOS_PROBE_SIN_F32>, dim3(blocks), dim3(kProbeBlock), 0, st, it, 7u, out); break;
      case WOS_PROBE_MUL_U32: hipLaunchKernelGGL(probe_kernel<WOS_PROBE_MUL_U32>, dim3(blocks), dim3(kProbeBlock), 0, st, it, 7u, out); break;
      default: hipLaunchKernelGGL(probe_kernel<WOS_PROBE_MUL_WIDE_U32>, dim3(blocks), dim3(kProbeBlock), 0, st, it, 7u, out); break;
    }
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    s = WOS_EDEVICE;
  } else {
    launch(1);  // warm-up
    (void)hipEventRecord(e0, st);
    launch(iters);
    (void)hipEventRecord(e1, st);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.0f))
      s = WOS_EDEVICE;
  }
  // one operation per chain step (the wide product: one 32 x 32 -> 64
  // multiply, its xor of the halves not counted)
  if (s == WOS_OK) *lane_ops_per_s = (double)threads * iters * kChains / (ms * 1e-3);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return s;
}
