// Direct application of the toolbox (the boxed reconstruction
// u = A q + H g, grad u_i = B_i q + K_i g): matrix-vector products that read
// each matrix once, so they are bound by HBM bandwidth.  One wavefront per
// output row; lanes stride along the row (coalesced 64-wide loads) and
// accumulate in FP64; the row sum is a wavefront reduction.
#include <hip/hip_runtime.h>

#include "wos_kernels.hpp"

namespace wos {

namespace {

constexpr int kApplyBlock = 256;
constexpr int kWaves = kApplyBlock / 64;

template <typename T>
__global__ __launch_bounds__(kApplyBlock) void apply_kernel(const T* __restrict__ M, int rows,
                                                            int cols_m, const double* __restrict__ x,
                                                            const T* __restrict__ N, int cols_n,
                                                            const double* __restrict__ y,
                                                            double* __restrict__ out, int batch) {
  const int lane = threadIdx.x & 63;
  const int64_t row_global = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (row_global >= (int64_t)rows * batch) return;
  const int b = (int)(row_global / rows);
  const int i = (int)(row_global - (int64_t)b * rows);
  const T* mrow = M + ((size_t)b * rows + i) * (size_t)cols_m;
  const T* nrow = N + ((size_t)b * rows + i) * (size_t)cols_n;
  double acc = 0.0;
  for (int j = lane; j < cols_m; j += 64) acc += (double)mrow[j] * x[j];
  for (int j = lane; j < cols_n; j += 64) acc += (double)nrow[j] * y[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) out[row_global] = acc;
}

template <typename T>
hipError_t launch(const T* M, int rows, int cols_m, const double* x, const T* N, int cols_n,
                  const double* y, double* out, int batch, hipStream_t stream) {
  const int64_t total = (int64_t)rows * batch;
  const int grid = (int)((total + kWaves - 1) / kWaves);
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(apply_kernel<T>, dim3(grid), dim3(kApplyBlock), 0, stream, M, rows, cols_m, x,
                     N, cols_n, y, out, batch);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_f32(const float* M, int rows, int cols_m, const double* x, const float* N,
                            int cols_n, const double* y, double* out, int batch, hipStream_t stream) {
  return launch<float>(M, rows, cols_m, x, N, cols_n, y, out, batch, stream);
}

hipError_t launch_apply_f64(const double* M, int rows, int cols_m, const double* x,
                            const double* N, int cols_n, const double* y, double* out, int batch,
                            hipStream_t stream) {
  return launch<double>(M, rows, cols_m, x, N, cols_n, y, out, batch, stream);
}

}  // namespace wos
