// Column permutation of row-major matrices, in place, one row per
// workgroup: the row is staged in LDS and written back as
// X[i, j] = X[i, rank[j]].  The windowed walker tallies into columns numbered
// by Morton rank; this puts them back in the caller's order at the end of a
// build.  Bound by HBM (each row read and written once).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wos_kernels.hpp"

namespace wos {

namespace {

constexpr int kPermBlock = 1024;

// With cols a multiple of 4 and 16-byte aligned rows, a thread moves four
// consecutive values per access (fewer, larger transfers in flight).
__global__ __launch_bounds__(kPermBlock) void permute_cols_kernel(uint32_t* __restrict__ X, int cols,
                                                                  const int* __restrict__ rank, int vec4) {
  extern __shared__ __align__(16) uint32_t row[];
  uint32_t* x = X + (size_t)blockIdx.x * cols;
  if (vec4) {
    const int c4 = cols >> 2;
    const uint4* x4 = reinterpret_cast<const uint4*>(x);
    uint4* r4 = reinterpret_cast<uint4*>(row);
    for (int j = threadIdx.x; j < c4; j += kPermBlock) r4[j] = x4[j];
    __syncthreads();
    const int4* k4 = reinterpret_cast<const int4*>(rank);
    uint4* o4 = reinterpret_cast<uint4*>(x);
    for (int j = threadIdx.x; j < c4; j += kPermBlock) {
      const int4 k = k4[j];
      o4[j] = make_uint4(row[k.x], row[k.y], row[k.z], row[k.w]);
    }
    return;
  }
  for (int j = threadIdx.x; j < cols; j += kPermBlock) row[j] = x[j];
  __syncthreads();
  for (int j = threadIdx.x; j < cols; j += kPermBlock) x[j] = row[rank[j]];
}

}  // namespace

size_t permute_max_cols() { return 160 * 1024 / 4; }

hipError_t launch_permute_cols(void* X, int rows, int cols, const int* rank, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if ((size_t)cols > permute_max_cols()) return hipErrorInvalidValue;
  const size_t lds = sizeof(uint32_t) * (size_t)cols;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(permute_cols_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int vec4 = (cols % 4 == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)rank % 16 == 0) ? 1 : 0;
  hipLaunchKernelGGL(permute_cols_kernel, dim3(rows), dim3(kPermBlock), lds, st, static_cast<uint32_t*>(X), cols,
                     rank, vec4);
  return hipGetLastError();
}

}  // namespace wos
