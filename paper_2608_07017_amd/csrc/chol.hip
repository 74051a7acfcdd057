// Blocked Cholesky factorisation N = L L^T (lower, row-major, in place) and
// the triangular solves with L, in FP32 or FP64, for the regularised normal
// equations of the solve path.
//
// Right-looking, panel width 64: the 64 x 64 diagonal block is factored by
// one workgroup in LDS, the panel below it is solved against that block
// (one thread per row, the block's factor in LDS), and the trailing matrix
// is updated by the MFMA GEMM (the full square; only its lower part is read
// later).  A non-positive pivot is replaced by a tiny one and reported in
// `info` (first failing column + 1), so a singular input never produces
// NaNs.
//
// Triangular solves, one right-hand side: the blocks are taken in order;
// the block's right-hand side is first reduced by the blocks already solved
// (a GEMV over the block's 64 rows, many workgroups) and then solved by one
// wavefront against the diagonal block.
#include <hip/hip_runtime.h>

#include "wos_solve_kernels.hpp"

namespace wos {

namespace {

constexpr int NB = 64;

__device__ __forceinline__ float dev_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dev_sqrt(double x) { return sqrt(x); }
template <typename T>
__device__ __forceinline__ T tiny_pivot();
template <>
__device__ __forceinline__ float tiny_pivot<float>() { return 1e-30f; }
template <>
__device__ __forceinline__ double tiny_pivot<double>() { return 1e-300; }

// factor the diagonal block A[k0 .. k0+b)^2 in place (b <= NB)
template <typename T>
__global__ __launch_bounds__(256) void potrf_diag_kernel(T* __restrict__ A, int lda, int k0, int b,
                                                          int* __restrict__ info) {
  __shared__ T s[NB][NB + 1];
  __shared__ T s_d;
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    s[i][j] = A[(size_t)(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    if (tid == 0) {
      T d = s[j][j];
      if (!(d > T(0))) {
        if (*info == 0) *info = k0 + j + 1;
        d = tiny_pivot<T>();
      }
      s_d = dev_sqrt(d);
      s[j][j] = s_d;
    }
    __syncthreads();
    const T d = s_d;
    for (int i = j + 1 + tid; i < b; i += 256) s[i][j] /= d;
    __syncthreads();
    // trailing update of the block: s[i][c] -= s[i][j] s[c][j], j < c <= i
    const int t = b - j - 1;
    for (int e = tid; e < t * t; e += 256) {
      const int i = j + 1 + e / t, c = j + 1 + e % t;
      if (c <= i) s[i][c] -= s[i][j] * s[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    A[(size_t)(k0 + i) * lda + k0 + j] = (j <= i) ? s[i][j] : T(0);
  }
}

// rows r in [k0 + b, n): x L11^T = A[r, k0 .. k0+b) solved in place
template <typename T>
__global__ __launch_bounds__(256) void trsm_panel_kernel(T* __restrict__ A, int lda, int n, int k0, int b) {
  __shared__ T L[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    L[i][j] = A[(size_t)(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  const int r = k0 + b + blockIdx.x * 256 + tid;
  if (r >= n) return;
  T* row = A + (size_t)r * lda + k0;
  for (int c = 0; c < b; ++c) {
    T v = row[c];
    for (int t = 0; t < c; ++t) v -= row[t] * L[c][t];
    row[c] = v / L[c][c];
  }
}

// y[r] -= sum_c L[r][c] x[c] for r in [r0, r0 + rows), c in [c0, c0 + cols)
// (trans = false), or y[c] -= sum_r L[r][c] x[r] over those ranges (trans):
// one wavefront per output element group
template <typename T>
__global__ __launch_bounds__(256) void trsv_update_kernel(const T* __restrict__ L, int lda, int r0, int rows,
                                                          int c0, int cols, const T* __restrict__ x,
                                                          T* __restrict__ y, int trans) {
  const int lane = threadIdx.x & 63;
  const int out = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nout = trans ? cols : rows;
  if (out >= nout) return;
  T acc = T(0);
  if (!trans) {
    const T* Lr = L + (size_t)(r0 + out) * lda + c0;
    for (int c = lane; c < cols; c += 64) acc += Lr[c] * x[c0 + c];
  } else {
    for (int r = lane; r < rows; r += 64) acc += L[(size_t)(r0 + r) * lda + c0 + out] * x[r0 + r];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    if (!trans)
      y[r0 + out] -= acc;
    else
      y[c0 + out] -= acc;
  }
}

// solve the diagonal block [k0, k0 + b) in place on y: L_kk z = y (lower)
// or L_kk^T z = y (upper); one wavefront
template <typename T>
__global__ __launch_bounds__(64) void trsv_diag_kernel(const T* __restrict__ L, int lda, int k0, int b,
                                                       T* __restrict__ y, int trans) {
  const int lane = threadIdx.x;
  T v = lane < b ? y[k0 + lane] : T(0);
  if (!trans) {
    for (int i = 0; i < b; ++i) {
      T zi = __shfl(v, i);
      zi /= L[(size_t)(k0 + i) * lda + k0 + i];
      if (lane == i) v = zi;
      if (lane > i && lane < b) v -= L[(size_t)(k0 + lane) * lda + k0 + i] * zi;
    }
  } else {
    for (int i = b - 1; i >= 0; --i) {
      T zi = __shfl(v, i);
      zi /= L[(size_t)(k0 + i) * lda + k0 + i];
      if (lane == i) v = zi;
      if (lane < i) v -= L[(size_t)(k0 + i) * lda + k0 + lane] * zi;
    }
  }
  if (lane < b) y[k0 + lane] = v;
}

template <typename T>
hipError_t gemm_t(bool ta, bool tb, int M, int N, int K, T alpha, const T* A, int lda, const T* B, int ldb, T beta,
                  T* C, int ldc, hipStream_t st);
template <>
hipError_t gemm_t<double>(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                          const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  return mfma_gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}
template <>
hipError_t gemm_t<float>(bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda,
                         const float* B, int ldb, float beta, float* C, int ldc, hipStream_t st) {
  return mfma_gemm_f32(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}

template <typename T>
hipError_t potrf(T* A, int n, int lda, int* info, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int b = min(NB, n - k0);
    hipLaunchKernelGGL(potrf_diag_kernel<T>, dim3(1), dim3(256), 0, st, A, lda, k0, b, info);
    const int rest = n - k0 - b;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_panel_kernel<T>, dim3((rest + 255) / 256), dim3(256), 0, st, A, lda, n, k0, b);
      T* L21 = A + (size_t)(k0 + b) * lda + k0;
      T* A22 = A + (size_t)(k0 + b) * lda + k0 + b;
      hipError_t e = gemm_t<T>(false, true, rest, rest, b, T(-1), L21, lda, L21, lda, T(1), A22, lda, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

// y <- (L L^T)^{-1} y
template <typename T>
hipError_t potrs(const T* L, int n, int lda, T* y, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += NB) {  // forward: L z = y
    const int b = min(NB, n - k0);
    if (k0 > 0)
      hipLaunchKernelGGL(trsv_update_kernel<T>, dim3((b + 3) / 4), dim3(256), 0, st, L, lda, k0, b, 0, k0, y, y, 0);
    hipLaunchKernelGGL(trsv_diag_kernel<T>, dim3(1), dim3(64), 0, st, L, lda, k0, b, y, 0);
  }
  const int last = ((n - 1) / NB) * NB;
  for (int k0 = last; k0 >= 0; k0 -= NB) {  // backward: L^T x = z
    const int b = min(NB, n - k0);
    const int below = n - (k0 + b);
    if (below > 0)
      hipLaunchKernelGGL(trsv_update_kernel<T>, dim3((b + 3) / 4), dim3(256), 0, st, L, lda, k0 + b, below, k0, b, y,
                         y, 1);
    hipLaunchKernelGGL(trsv_diag_kernel<T>, dim3(1), dim3(64), 0, st, L, lda, k0, b, y, 1);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t cholesky_f64(double* A, int n, int lda, int* info, hipStream_t st) { return potrf<double>(A, n, lda, info, st); }
hipError_t cholesky_f32(float* A, int n, int lda, int* info, hipStream_t st) { return potrf<float>(A, n, lda, info, st); }
hipError_t cholesky_solve_f64(const double* L, int n, int lda, double* y, hipStream_t st) {
  return potrs<double>(L, n, lda, y, st);
}
hipError_t cholesky_solve_f32(const float* L, int n, int lda, float* y, hipStream_t st) {
  return potrs<float>(L, n, lda, y, st);
}

}  // namespace wos
