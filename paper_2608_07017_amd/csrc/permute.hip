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

__global__ __launch_bounds__(kPermBlock) void permute_cols_kernel(uint32_t* __restrict__ X, int cols,
                                                                  const int* __restrict__ rank) {
  extern __shared__ __align__(16) uint32_t row[];
  uint32_t* x = X + (size_t)blockIdx.x * cols;
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
  hipLaunchKernelGGL(permute_cols_kernel, dim3(rows), dim3(kPermBlock), lds, st, static_cast<uint32_t*>(X), cols,
                     rank);
  return hipGetLastError();
}

}  // namespace wos
