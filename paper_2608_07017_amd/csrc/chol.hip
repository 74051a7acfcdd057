// Blocked Cholesky factorisation N = L L^T (lower, row-major, in place) and
// the triangular solves with L, in FP32 or FP64, for the regularised normal
// equations of the solve path.
//
// Recursive: the block is halved at a multiple of 64 rows, the leading half
// is factored and inverted, the off-diagonal block of the factor and the
// Schur complement update are MFMA GEMMs (inner dimension half the block),
// the trailing half is factored and inverted, and the off-diagonal block of
// the inverse is two more GEMMs; 64 x 64 diagonal blocks are factored in
// LDS by one workgroup of four wavefronts (itself blocked by panels of eight
// columns: one wavefront factors a panel, all four apply its rank-8 update)
// and inverted by one of them.  A non-positive pivot is replaced by a tiny
// one and reported in `info` (first failing column + 1), so a singular
// input never produces NaNs.
//
// The solves with the factor use its explicit inverse X = L^{-1}: each
// solve (L L^T)^{-1} r = X^T (X r) is then two matrix-vector products.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Factor the diagonal block A[k0 .. k0+b)^2 in place (b <= NB) and write
// the inverse of its factor to the same block of X (zero above the
// diagonal).  Four wavefronts, lane l owning row l: the factor is blocked
// by panels of eight columns (see below), then wavefront 0 inverts it, one
// column per lane in registers.
template <typename T>
__global__ __launch_bounds__(256) void potrf_diag_kernel(T* __restrict__ A, int lda, int k0, int b,
                                                          T* __restrict__ X, int ldx, int* __restrict__ info) {
  __shared__ T s[NB][NB + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    s[i][j] = (i < b && j < b) ? A[(size_t)(k0 + i) * lda + k0 + j] : (i == j ? T(1) : T(0));
  }
  __syncthreads();
  // blocked by panels of PW columns: wavefront 0 factors a panel (rows in
  // lanes, columns in order, the panel's own updates inside the
  // wavefront), then all wavefronts apply its rank-PW update to the
  // columns right of it; two barriers per panel
  constexpr int PW = 8;
  int bad = 0;
  for (int jb = 0; jb < NB; jb += PW) {
    if (wave == 0) {
      for (int t = 0; t < PW; ++t) {
        const int j = jb + t;
        T d = s[j][j];
        if (!(d > T(0))) {
          if (bad == 0 && j < b) bad = j + 1;
          d = tiny_pivot<T>();
        }
        d = dev_sqrt(d);
        const T lij = lane > j ? s[lane][j] / d : (lane == j ? d : T(0));
        s[lane][j] = lij;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int c = j + 1; c < jb + PW; ++c)
          if (lane >= c) s[lane][c] -= lij * s[c][j];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    __syncthreads();
    T li[PW];
#pragma unroll
    for (int t = 0; t < PW; ++t) li[t] = s[lane][jb + t];
    for (int c = jb + PW + wave; c <= lane; c += 4) {
      T v = s[lane][c];
#pragma unroll
      for (int t = 0; t < PW; ++t) v -= li[t] * s[c][jb + t];
      s[lane][c] = v;
    }
    __syncthreads();
  }
  if (tid == 0 && bad && *info == 0) *info = k0 + bad;
  if (wave == 0) {
    // inverse of the lower factor, one column per lane kept in registers
    // (forward substitution with the factor's rows read from LDS)
    T xc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      T v = (i == lane) ? T(1) : T(0);
#pragma unroll
      for (int t = 0; t < i; ++t) v -= s[i][t] * xc[t];
      xc[i] = (i >= lane && i < b && lane < b) ? v / s[i][i] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (i < b && lane < b) X[(size_t)(k0 + i) * ldx + k0 + lane] = xc[i];
  }
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    A[(size_t)(k0 + i) * lda + k0 + j] = (j <= i) ? s[i][j] : T(0);
  }
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

// dst (rows x cols, ldd) = src (rows x cols, lds)
template <typename T>
__global__ void copy_block_kernel(const T* __restrict__ src, int lds, T* __restrict__ dst, int ldd, int rows,
                                  int cols) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / cols, j = e % cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

// Factor A[n0:n1, n0:n1] = L L^T in place and write X = L^{-1} to the same
// block of X, by recursive halving at a multiple of NB:
//   L11, X11 of the leading half;  L21 = A21 X11^T;  A22 -= L21 L21^T;
//   L22, X22 of the trailing half;  X21 = -X22 (L21 X11);
// the leaves are the one-workgroup diagonal kernel.  Apart from the leaves
// every step is a GEMM whose inner dimension is half the block, so the
// factorisation and the inverse run mostly as large MFMA products.
template <typename T>
hipError_t chol_inv_rec(T* A, int lda, int n0, int n1, T* X, int ldx, T* work, int* info, hipStream_t st) {
  const int nb = (n1 - n0 + NB - 1) / NB;
  if (nb <= 1) {
    hipLaunchKernelGGL(potrf_diag_kernel<T>, dim3(1), dim3(256), 0, st, A, lda, n0, n1 - n0, X, ldx, info);
    return hipGetLastError();
  }
  const int h = n0 + (nb / 2) * NB;
  const int r = n1 - h, c = h - n0;
  T* A21 = A + (size_t)h * lda + n0;
  T* A22 = A + (size_t)h * lda + h;
  T* X11 = X + (size_t)n0 * ldx + n0;
  T* X21 = X + (size_t)h * ldx + n0;
  T* X22 = X + (size_t)h * ldx + h;
  hipError_t e = chol_inv_rec<T>(A, lda, n0, h, X, ldx, work, info, st);
  if (e != hipSuccess) return e;
  // L21 = A21 X11^T, kept in the (still unused) X21 block
  e = gemm_t<T>(false, true, r, c, c, T(1), A21, lda, X11, ldx, T(0), X21, ldx, st);
  if (e != hipSuccess) return e;
  e = gemm_t<T>(false, true, r, r, c, T(-1), X21, ldx, X21, ldx, T(1), A22, lda, st);
  if (e != hipSuccess) return e;
  const size_t tot = (size_t)r * c;
  hipLaunchKernelGGL(copy_block_kernel<T>, dim3((unsigned)std::min<size_t>((tot + 255) / 256, 4096)), dim3(256), 0,
                     st, X21, ldx, A21, lda, r, c);
  e = chol_inv_rec<T>(A, lda, h, n1, X, ldx, work, info, st);
  if (e != hipSuccess) return e;
  // X21 = -X22 (L21 X11)
  e = gemm_t<T>(false, false, r, c, c, T(1), A21, lda, X11, ldx, T(0), work, c, st);
  if (e != hipSuccess) return e;
  return gemm_t<T>(false, false, r, c, r, T(-1), X22, ldx, work, c, T(0), X21, ldx, st);
}

template <typename T>
hipError_t chol_inv(T* A, int n, int lda, T* X, int ldx, T* work, int* info, hipStream_t st) {
  hipError_t e = hipMemsetAsync(X, 0, sizeof(T) * (size_t)n * ldx, st);  // the blocks above the diagonal
  if (e != hipSuccess) return e;
  e = chol_inv_rec<T>(A, lda, 0, n, X, ldx, work, info, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

size_t chol_work_elems(int n) {
  const int nb = (n + NB - 1) / NB;
  const size_t h = (size_t)(nb / 2) * NB;
  return std::max<size_t>((size_t)n * NB, h * ((size_t)n - std::min<size_t>(h, n)));
}

hipError_t cholesky_inverse_f64(double* A, int n, int lda, double* X, double* work, int* info, hipStream_t st) {
  return chol_inv<double>(A, n, lda, X, n, work, info, st);
}
hipError_t cholesky_inverse_f32(float* A, int n, int lda, float* X, float* work, int* info, hipStream_t st) {
  return chol_inv<float>(A, n, lda, X, n, work, info, st);
}

}  // namespace wos
