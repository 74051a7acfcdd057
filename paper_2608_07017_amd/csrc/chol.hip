// Blocked Cholesky factorisation N = L L^T (lower, row-major, in place) and
// the triangular solves with L, in FP32 or FP64, for the regularised normal
// equations of the solve path.
//
// Right-looking, panel width 64: the 64 x 64 diagonal block is factored in
// LDS by four wavefronts (itself blocked by panels of eight columns: one
// wavefront factors a panel, all four apply its rank-8 update), and one of
// them inverts the factor (kept in Dinv, one 64 x 64 block per panel); the panel below is then L21 = A21 L11^{-T}, an MFMA
// GEMM with that inverse, and the trailing matrix is updated by the MFMA
// GEMM (the full square; only its lower part is read later).  A
// non-positive pivot is replaced by a tiny one and reported in `info`
// (first failing column + 1), so a singular input never produces NaNs.
//
// The solves with the factor use its explicit inverse X = L^{-1}, built by
// recursive halving, [L11 0; L21 L22]^{-1} = [X11 0; -X22 L21 X11 X22],
// down to the diagonal inverses, so that most of its work is in large MFMA
// GEMMs; each solve (L L^T)^{-1} r = X^T (X r) is then two matrix-vector
// products.
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
// the inverse of its factor to Dinv (NB x NB, row-major, zero above the
// diagonal).  Four wavefronts, lane l owning row l: the factor is blocked
// by panels of eight columns (see below), then wavefront 0 inverts it, one
// column per lane in registers.
template <typename T>
__global__ __launch_bounds__(256) void potrf_diag_kernel(T* __restrict__ A, int lda, int k0, int b,
                                                          T* __restrict__ Dinv, int* __restrict__ info) {
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
    for (int i = 0; i < NB; ++i) Dinv[i * NB + lane] = xc[i];
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

template <typename T>
__global__ void copy_panel_kernel(const T* __restrict__ P, int rows, int b, T* __restrict__ A, int lda) {
  const size_t total = (size_t)rows * b;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
    A[(e / b) * lda + e % b] = P[e];
}

template <typename T>
hipError_t potrf(T* A, int n, int lda, T* Dinv, T* work, int* info, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int b = min(NB, n - k0);
    T* Dk = Dinv + (size_t)(k0 / NB) * NB * NB;
    hipLaunchKernelGGL(potrf_diag_kernel<T>, dim3(1), dim3(256), 0, st, A, lda, k0, b, Dk, info);
    const int rest = n - k0 - b;
    if (rest > 0) {
      // panel: L21 = A21 L11^{-T} = A21 Dk^T into `work` (rest x b), then
      // the trailing update A22 -= L21 L21^T, then L21 back into A
      T* A21 = A + (size_t)(k0 + b) * lda + k0;
      hipError_t e = gemm_t<T>(false, true, rest, b, b, T(1), A21, lda, Dk, NB, T(0), work, b, st);
      if (e != hipSuccess) return e;
      T* A22 = A + (size_t)(k0 + b) * lda + k0 + b;
      e = gemm_t<T>(false, true, rest, rest, b, T(-1), work, b, work, b, T(1), A22, lda, st);
      if (e != hipSuccess) return e;
      const size_t tot = (size_t)rest * b;
      hipLaunchKernelGGL(copy_panel_kernel<T>, dim3((unsigned)std::min<size_t>((tot + 255) / 256, 4096)), dim3(256),
                         0, st, work, rest, b, A21, lda);
    }
  }
  return hipGetLastError();
}

// X = L^{-1} (lower, zeros above the diagonal) from the factor and the
// inverses of its diagonal blocks, by recursive halving at multiples of NB:
// X[h:, :h] = -X[h:, h:] (L[h:, :h] X[:h, :h]).
template <typename T>
__global__ void place_diag_inverse_kernel(const T* __restrict__ Dinv, int n, T* __restrict__ X, int ldx) {
  const int kb = blockIdx.x, k0 = kb * NB;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    if (k0 + i < n && k0 + j < n) X[(size_t)(k0 + i) * ldx + k0 + j] = Dinv[(size_t)kb * NB * NB + e];
  }
}

template <typename T>
hipError_t trtri_rec(const T* L, int lda, int n0, int n1, T* X, int ldx, T* work, hipStream_t st) {
  const int nb = (n1 - n0 + NB - 1) / NB;
  if (nb <= 1) return hipSuccess;  // diagonal block: placed beforehand
  const int h = n0 + (nb / 2) * NB;
  hipError_t e = trtri_rec<T>(L, lda, n0, h, X, ldx, work, st);
  if (e != hipSuccess) return e;
  e = trtri_rec<T>(L, lda, h, n1, X, ldx, work, st);
  if (e != hipSuccess) return e;
  const int r = n1 - h, c = h - n0;
  // work (r x c) = L[h:n1, n0:h] X[n0:h, n0:h]
  e = gemm_t<T>(false, false, r, c, c, T(1), L + (size_t)h * lda + n0, lda, X + (size_t)n0 * ldx + n0, ldx, T(0),
                work, c, st);
  if (e != hipSuccess) return e;
  // X[h:n1, n0:h] = -X[h:n1, h:n1] work
  return gemm_t<T>(false, false, r, c, r, T(-1), X + (size_t)h * ldx + h, ldx, work, c, T(0),
                   X + (size_t)h * ldx + n0, ldx, st);
}

template <typename T>
hipError_t trtri(const T* L, int n, int lda, const T* Dinv, T* X, int ldx, T* work, hipStream_t st) {
  hipError_t e = hipMemsetAsync(X, 0, sizeof(T) * (size_t)n * ldx, st);
  if (e != hipSuccess) return e;
  const int nb = (n + NB - 1) / NB;
  hipLaunchKernelGGL(place_diag_inverse_kernel<T>, dim3(nb), dim3(256), 0, st, Dinv, n, X, ldx);
  e = trtri_rec<T>(L, lda, 0, n, X, ldx, work, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

size_t chol_work_elems(int n) {
  const int nb = (n + NB - 1) / NB;
  const size_t h = (size_t)(nb / 2) * NB;
  return std::max<size_t>((size_t)n * NB, h * ((size_t)n - std::min<size_t>(h, n)));
}

hipError_t cholesky_f64(double* A, int n, int lda, double* Dinv, double* work, int* info, hipStream_t st) {
  return potrf<double>(A, n, lda, Dinv, work, info, st);
}
hipError_t cholesky_f32(float* A, int n, int lda, float* Dinv, float* work, int* info, hipStream_t st) {
  return potrf<float>(A, n, lda, Dinv, work, info, st);
}
hipError_t tri_inverse_f64(const double* L, int n, int lda, const double* Dinv, double* X, double* work,
                           hipStream_t st) {
  return trtri<double>(L, n, lda, Dinv, X, n, work, st);
}
hipError_t tri_inverse_f32(const float* L, int n, int lda, const float* Dinv, float* X, float* work,
                           hipStream_t st) {
  return trtri<float>(L, n, lda, Dinv, X, n, work, st);
}

}  // namespace wos
