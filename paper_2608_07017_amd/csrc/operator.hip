// Kernels of the solution operators (C ABI wos_operator_*): the batched
// application u[r] = U z[r], z[r] = [f[r]; g[r]], of a dense operator to up
// to eight right-hand sides per launch, and the small elementwise steps of
// the operator's preparation.
//
// The application streams U from HBM once per launch.  A wavefront owns KR
// rows of U (8, or 4 for batches wider than four) and one slice of its
// columns; each lane loads two consecutive elements of each row at a time
// (rows are padded to a multiple of four elements, so the loads are
// aligned), holds KR x NB FP64 accumulators and reads each z value once for
// the KR rows.  Slices of the same rows add
// their partial sums into the (zeroed) outputs with FP64 atomics; the number
// of slices is chosen so that the launch has a few thousand wavefronts.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wos_operator.hpp"

namespace wos {

namespace {

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

// VEC = 2 consecutive elements of one row of U in one load (8 bytes for
// FP32, 16 for FP64; rows are aligned: the row stride is a multiple of four
// and the column a multiple of VEC).  Wider FP32 loads were slower: each
// column also needs NB loads of z, which then dominate.
template <typename TS>
struct VecLoad;
template <>
struct VecLoad<float> {
  static constexpr int N = 2;
  __device__ __forceinline__ static void load(const float* p, float (&v)[2]) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    v[0] = q.x;
    v[1] = q.y;
  }
};
template <>
struct VecLoad<double> {
  static constexpr int N = 2;
  __device__ __forceinline__ static void load(const double* p, double (&v)[2]) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    v[0] = q.x;
    v[1] = q.y;
  }
};

template <typename TS, int NB, int KR>
__global__ __launch_bounds__(64 * kWaves) void op_apply_kernel(const TS* __restrict__ U, int rows, int cols, int ld,
                                                               int n, int grad_rows, int slices, int slice_cols,
                                                               OpBatch bt) {
  constexpr int VEC = VecLoad<TS>::N;
  const int wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int rg = wave / slices, sl = wave - rg * slices;
  const int r0 = rg * KR;
  if (r0 >= rows) return;
  const int c0 = sl * slice_cols, c1 = min(cols, c0 + slice_cols);
  const int nr = min(KR, rows - r0);

  double acc[KR][NB];
#pragma unroll
  for (int r = 0; r < KR; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[r][b] = 0.0;

  const TS* Ur = U + (size_t)r0 * ld;
  for (int j = c0 + lane * VEC; j < c1; j += 64 * VEC) {
    TS uv[KR][VEC];
    if (j + VEC <= c1) {
#pragma unroll
      for (int r = 0; r < KR; ++r) {
        if (r < nr) {
          VecLoad<TS>::load(Ur + (size_t)r * ld + j, uv[r]);
        } else {
#pragma unroll
          for (int c = 0; c < VEC; ++c) uv[r][c] = TS(0);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < KR; ++r)
#pragma unroll
        for (int c = 0; c < VEC; ++c) uv[r][c] = (r < nr && j + c < c1) ? Ur[(size_t)r * ld + j + c] : TS(0);
    }
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      const int jc = min(j + c, cols - 1);  // columns past c1 have uv = 0
      double z[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) z[b] = jc < n ? bt.f[b][jc] : bt.g[b][jc - n];
#pragma unroll
      for (int r = 0; r < KR; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = fma((double)uv[r][c], z[b], acc[r][b]);
    }
  }
#pragma unroll
  for (int r = 0; r < KR; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = acc[r][b];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      acc[r][b] = v;
    }
  // lane k writes the (row, rhs) pair k, k + 64, ...
  for (int k = lane; k < KR * NB; k += 64) {
    const int r = k / NB, b = k - r * NB;
    if (r >= nr) continue;
    double v = 0.0;
#pragma unroll
    for (int rr = 0; rr < KR; ++rr)
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

template <typename TS, int NB>
hipError_t apply_nb(const TS* U, int rows, int cols, int ld, int n, int grad_rows, const OpBatch& bt,
                    hipStream_t st) {
  // rows per wavefront: eight for narrow batches, four for wide ones, which
  // keeps the accumulators within about 64 registers
  constexpr int KR = NB <= 4 ? 8 : 4;
  constexpr int VEC = VecLoad<TS>::N;
  const int groups = (rows + KR - 1) / KR;
  const int chunk = 64 * VEC;  // columns one pass of a wavefront covers
  int slices = std::max(1, std::min((kTargetWaves + groups - 1) / groups, (cols + chunk - 1) / chunk));
  const int slice_cols = ((cols + slices - 1) / slices + chunk - 1) / chunk * chunk;
  slices = (cols + slice_cols - 1) / slice_cols;
  if (slices > 1)
    hipLaunchKernelGGL(op_zero_kernel, dim3(nblocks((size_t)rows * NB, 256)), dim3(256), 0, st, rows, n, grad_rows,
                       NB, bt);
  const dim3 grid((unsigned)(((size_t)groups * slices + kWaves - 1) / kWaves)), block(64 * kWaves);
  hipLaunchKernelGGL((op_apply_kernel<TS, NB, KR>), grid, block, 0, st, U, rows, cols, ld, n, grad_rows, slices,
                     slice_cols, bt);
  return hipGetLastError();
}

template <typename TS>
hipError_t apply_t(const TS* U, int rows, int cols, int ld, int n, int grad_rows, int nb, const OpBatch& bt,
                   hipStream_t st) {
  switch (nb) {
    case 1: return apply_nb<TS, 1>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 2: return apply_nb<TS, 2>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 3: return apply_nb<TS, 3>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 4: return apply_nb<TS, 4>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 5: return apply_nb<TS, 5>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 6: return apply_nb<TS, 6>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 7: return apply_nb<TS, 7>(U, rows, cols, ld, n, grad_rows, bt, st);
    case 8: return apply_nb<TS, 8>(U, rows, cols, ld, n, grad_rows, bt, st);
    default: return hipErrorInvalidValue;
  }
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
