// Kernels of the solution operators (C ABI wos_operator_*): the batched
// application u[r] = U z[r], z[r] = [f[r]; g[r]], of a dense operator to up
// to eight right-hand sides per launch, and the small elementwise steps of
// the operator's preparation.
//
// The application streams U from HBM once per launch.  A wavefront owns
// kRows rows of U and one slice of its columns; each lane walks the slice
// with stride 64 (coalesced rows), holds kRows x NB FP64 accumulators and
// reads each z value once for the kRows rows.  Slices of the same rows add
// their partial sums into the (zeroed) outputs with FP64 atomics; the number
// of slices is chosen so that the launch has a few thousand wavefronts.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wos_operator.hpp"

namespace wos {

namespace {

constexpr int kRows = 8;     // rows of U per wavefront
constexpr int kWaves = 4;    // wavefronts per workgroup
constexpr int kTargetWaves = 4096;

int nblocks(size_t count, int block) {
  size_t g = (count + block - 1) / block;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

// Output row r of the operator: rows [0, grad_rows) are grad u (d x n, in
// that order), rows [grad_rows, grad_rows + n) are u.
__device__ __forceinline__ double* out_slot(const OpBatch& bt, int b, int r, int grad_rows) {
  if (r < grad_rows) return bt.gu[b] ? bt.gu[b] + r : nullptr;
  return bt.u[b] + (r - grad_rows);
}

template <typename TS, int NB>
__global__ __launch_bounds__(64 * kWaves) void op_apply_kernel(const TS* __restrict__ U, int rows, int cols, int ld,
                                                               int n, int grad_rows, int slices, int slice_cols,
                                                               OpBatch bt) {
  const int wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int rg = wave / slices, sl = wave - rg * slices;
  const int r0 = rg * kRows;
  if (r0 >= rows) return;
  const int c0 = sl * slice_cols, c1 = min(cols, c0 + slice_cols);
  const int nr = min(kRows, rows - r0);

  double acc[kRows][NB];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = 0.0;

  const TS* Ur = U + (size_t)r0 * ld;
  for (int j = c0 + lane; j < c1; j += 64) {
    double z[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) z[b] = j < n ? bt.f[b][j] : bt.g[b][j - n];
    double uv[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) uv[r] = r < nr ? (double)Ur[(size_t)r * ld + j] : 0.0;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[r][b] = fma(uv[r], z[b], acc[r][b]);
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = acc[r][b];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      acc[r][b] = v;
    }
  // lane k writes the (row, rhs) pair k, k + 64, ...
  for (int k = lane; k < kRows * NB; k += 64) {
    const int r = k / NB, b = k - r * NB;
    if (r >= nr) continue;
    double v = 0.0;
#pragma unroll
    for (int rr = 0; rr < kRows; ++rr)
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
        if (rr * NB + bb == k) v = acc[rr][bb];
    double* o = out_slot(bt, b, r0 + r, grad_rows);
    if (!o) continue;
    if (slices == 1)
      *o = v;
    else
      atomicAdd(o, v);
  }
}

__global__ void op_zero_kernel(int rows, int n, int grad_rows, int nb, OpBatch bt) {
  const int total = rows * nb;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int b = e / rows, r = e - b * rows;
    double* o = out_slot(bt, b, r, grad_rows);
    if (o) *o = 0.0;
  }
}

template <typename TS>
hipError_t apply_t(const TS* U, int rows, int cols, int ld, int n, int grad_rows, int nb, const OpBatch& bt,
                   hipStream_t st) {
  const int groups = (rows + kRows - 1) / kRows;
  int slices = std::max(1, std::min((kTargetWaves + groups - 1) / groups, (cols + 255) / 256));
  const int slice_cols = ((cols + slices - 1) / slices + 63) / 64 * 64;
  slices = (cols + slice_cols - 1) / slice_cols;
  if (slices > 1)
    hipLaunchKernelGGL(op_zero_kernel, dim3(nblocks((size_t)rows * nb, 256)), dim3(256), 0, st, rows, n, grad_rows,
                       nb, bt);
  const dim3 grid((unsigned)(((size_t)groups * slices + kWaves - 1) / kWaves)), block(64 * kWaves);
  switch (nb) {
#define WOS_OP_CASE(NB)                                                                                            \
  case NB:                                                                                                         \
    hipLaunchKernelGGL((op_apply_kernel<TS, NB>), grid, block, 0, st, U, rows, cols, ld, n, grad_rows, slices,      \
                       slice_cols, bt);                                                                            \
    break;
    WOS_OP_CASE(1)
    WOS_OP_CASE(2)
    WOS_OP_CASE(3)
    WOS_OP_CASE(4)
    WOS_OP_CASE(5)
    WOS_OP_CASE(6)
    WOS_OP_CASE(7)
    WOS_OP_CASE(8)
#undef WOS_OP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// X[i][j] *= alpha w[j]  (rows x cols, leading dimension ld)
__global__ void scale_cols_kernel(double* __restrict__ X, int rows, int cols, int ld, const double* __restrict__ w,
                                  double alpha) {
  const size_t total = (size_t)rows * cols;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const size_t i = e / cols, j = e % cols;
    X[i * ld + j] *= alpha * w[j];
  }
}

// Y[i][j] += X[i][j]  (Y FP64 with leading dimension ldy; X dense rows x cols)
template <typename TX>
__global__ void add_block_kernel(double* __restrict__ Y, int rows, int cols, int ldy, const TX* __restrict__ X) {
  const size_t total = (size_t)rows * cols;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const size_t i = e / cols, j = e % cols;
    Y[i * ldy + j] += (double)X[e];
  }
}

__global__ void narrow_kernel(size_t count, const double* __restrict__ x, float* __restrict__ y) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) y[i] = (float)x[i];
}

}  // namespace

hipError_t launch_op_apply(bool f32, const void* U, int rows, int cols, int ld, int n, int grad_rows, int nb,
                           const OpBatch& bt, hipStream_t st) {
  if (nb < 1 || nb > kOpBatch || rows < 1 || cols < 1) return hipErrorInvalidValue;
  if (f32) return apply_t<float>(static_cast<const float*>(U), rows, cols, ld, n, grad_rows, nb, bt, st);
  return apply_t<double>(static_cast<const double*>(U), rows, cols, ld, n, grad_rows, nb, bt, st);
}

hipError_t launch_scale_cols(double* X, int rows, int cols, int ld, const double* w, double alpha, hipStream_t st) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(nblocks((size_t)rows * cols, 256)), dim3(256), 0, st, X, rows, cols, ld,
                     w, alpha);
  return hipGetLastError();
}

hipError_t launch_add_block(double* Y, int rows, int cols, int ldy, bool x_f64, const void* X, hipStream_t st) {
  const dim3 g(nblocks((size_t)rows * cols, 256)), b(256);
  if (x_f64)
    hipLaunchKernelGGL(add_block_kernel<double>, g, b, 0, st, Y, rows, cols, ldy, static_cast<const double*>(X));
  else
    hipLaunchKernelGGL(add_block_kernel<float>, g, b, 0, st, Y, rows, cols, ldy, static_cast<const float*>(X));
  return hipGetLastError();
}

hipError_t launch_narrow(size_t count, const double* x, float* y, hipStream_t st) {
  hipLaunchKernelGGL(narrow_kernel, dim3(nblocks(count, 256)), dim3(256), 0, st, count, x, y);
  return hipGetLastError();
}

}  // namespace wos
