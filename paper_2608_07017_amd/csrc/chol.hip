// Blocked Cholesky factorisation N = L L^T (lower, row-major, in place) and
// the triangular solves with L, in FP32 or FP64, for the regularised normal
// equations of the solve path.
//
// Recursive: the block is halved at a multiple of 64 rows, the leading half
// is factored and inverted, the off-diagonal block of the factor and the
// Schur complement update are MFMA GEMMs (inner dimension half the block),
// the trailing half is factored and inverted, and the off-diagonal block of
// the inverse is two more GEMMs; 64 x 64 diagonal blocks are factored in
// LDS by one workgroup of four wavefronts (panels of 16 columns factored in
// one wavefront's registers, their updates and the inverse by 16 x 16 tiles
// on the matrix cores).  A non-positive pivot is replaced by a tiny
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

// 1 / sqrt(x) for a positive normal x: the hardware estimate refined by
// Newton steps y <- y (3/2 - (x/2) y^2) (one for FP32, two for FP64, each
// at least doubling the correct bits), within a few ulp of the exact value.
__device__ __forceinline__ float rsqrt_refined(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  const float h = 0.5f * x;
  y = y * (1.5f - h * y * y);
  return y;
}
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}
template <typename T>
__device__ __forceinline__ T tiny_pivot();
template <>
__device__ __forceinline__ float tiny_pivot<float>() { return 1e-30f; }
template <>
__device__ __forceinline__ double tiny_pivot<double>() { return 1e-300; }

// Broadcast lane `src` (a constant) of v to the whole wavefront.
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 16 x 16 x 4 MFMA in the operand precision (layouts in mfma_gemm.hip:
// A operand A[l % 16][l / 16], B operand B[l / 16][l % 16]).
__device__ __forceinline__ void tile_mfma(float a, float b, float (&acc)[4]) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  v4f c = {acc[0], acc[1], acc[2], acc[3]};
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  for (int r = 0; r < 4; ++r) acc[r] = c[r];
}
__device__ __forceinline__ void tile_mfma(double a, double b, double (&acc)[4]) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  v4d c = {acc[0], acc[1], acc[2], acc[3]};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  for (int r = 0; r < 4; ++r) acc[r] = c[r];
}
// row of result r of lane l in a 16 x 16 MFMA tile (column l % 16)
template <typename T>
__device__ __forceinline__ int tile_row(int l, int r) {
  return sizeof(T) == 8 ? (l >> 4) + 4 * r : 4 * (l >> 4) + r;
}

constexpr int TW = 16;  // tile side and panel width of the diagonal kernel

template <typename T>
using Blk = T[NB][NB + 1];  // one NB x NB block in LDS (rows padded)
template <typename T>
using Scr = T[4][TW][TW + 1];  // per-wavefront tile scratch

// Factor the NB x NB block s (in LDS, padded with the identity beyond its
// b x b part) as L L^T in place and write X = L^{-1} to sx; `bad` becomes
// the first non-positive pivot + 1 (0 if none) among the first b columns.
// Entries of s and sx above the diagonal are left undefined (those inside
// the diagonal tiles of sx are zero).  All four wavefronts of the
// workgroup call it; it ends with a barrier.
//
// Factor, by panels of TW columns: wavefront 0 factors the panel with row
// jb + l in lane l, the panel in registers and the pivots and multipliers
// broadcast across lanes (no LDS round trip inside the panel); then the
// TW x TW tiles right of and below the panel take the rank-TW update
// C -= L_ip L_jp^T on the matrix cores (at most two tiles per wavefront).
//
// Inverse X = L^{-1}, by tiles: the four diagonal tiles are inverted by
// forward substitution (one wavefront each, one column per lane), then
// each block row I of the off-diagonal tiles is X_IJ = -X_II sum_K L_IK X_KJ
// (J <= K < I), the tiles of one block row in parallel.
template <typename T>
__device__ void factor_inv_lds(Blk<T>& s, Blk<T>& sx, Scr<T>& st, int b, int& bad) {
  constexpr int NT = NB / TW;  // tiles per side
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  bad = 0;
  for (int p = 0; p < NT; ++p) {
    const int jb = p * TW;
    if (wave == 0) {
      const int row = jb + lane;
      const bool live = row < NB;
      T r[TW];
#pragma unroll
      for (int t = 0; t < TW; ++t) r[t] = live ? s[row][jb + t] : T(0);
      // per column: pivot, scaled column, then the update of column t + 1
      // (the next pivot's critical path) before the others; the
      // scheduling barrier keeps the broadcasts of one column from being
      // hoisted into the next (SGPR pressure)
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        T d = lane_bcast(r[t], t);
        const bool ok = d > T(0);
        bad = (!ok && bad == 0 && jb + t < b) ? jb + t + 1 : bad;
        d = ok ? d : tiny_pivot<T>();
        const T inv = rsqrt_refined(d);
        const T l = lane > t ? r[t] * inv : (lane == t ? d * inv : T(0));
        r[t] = l;
        if (t + 1 < TW) r[t + 1] -= l * lane_bcast(l, t + 1);
#pragma unroll
        for (int c = t + 2; c < TW; ++c) r[c] -= l * lane_bcast(l, c);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (live) {
#pragma unroll
        for (int t = 0; t < TW; ++t) s[row][jb + t] = r[t];
      }
    }
    __syncthreads();
    // trailing tiles (I, J), p < J <= I < NT: wavefront w takes tiles
    // w and w + 4 of that list
    const int nrest = NT - 1 - p;
    const int ntiles = nrest * (nrest + 1) / 2;
    for (int k = wave; k < ntiles; k += 4) {
      int J = p + 1, rem = k;
      while (rem >= NT - J) {
        rem -= NT - J;
        ++J;
      }
      const int I = J + rem;
      T acc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = s[I * TW + tile_row<T>(lane, r)][J * TW + li];
#pragma unroll
      for (int q = 0; q < TW / 4; ++q) {
        const T a = -s[I * TW + li][jb + 4 * q + lk];
        const T bb = s[J * TW + li][jb + 4 * q + lk];
        tile_mfma(a, bb, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) s[I * TW + tile_row<T>(lane, r)][J * TW + li] = acc[r];
    }
    __syncthreads();
  }
  // diagonal tiles of the inverse: wavefront I inverts L_II, column li in
  // lanes li (the other lanes repeat the work of lane li)
  {
    // right-looking: row t of the column is final once the rows above it
    // have been subtracted, then it is subtracted from the rows below
    const int I = wave, o = I * TW;
    const T invd = T(1) / s[o + li][o + li];
    T xc[TW];
#pragma unroll
    for (int i = 0; i < TW; ++i) xc[i] = (i == li) ? T(1) : T(0);
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      xc[t] *= lane_bcast(invd, t);
#pragma unroll
      for (int i = t + 1; i < TW; ++i) xc[i] -= s[o + i][o + t] * xc[t];
    }
    if (lk == 0) {
#pragma unroll
      for (int i = 0; i < TW; ++i) sx[o + i][o + li] = xc[i];
    }
  }
  __syncthreads();
  // block rows of the off-diagonal tiles
  for (int I = 1; I < NT; ++I) {
    if (wave < I) {
      const int J = wave;
      T acc[4] = {T(0), T(0), T(0), T(0)};
      for (int K = J; K < I; ++K) {
#pragma unroll
        for (int q = 0; q < TW / 4; ++q)
          tile_mfma(s[I * TW + li][K * TW + 4 * q + lk], sx[K * TW + 4 * q + lk][J * TW + li], acc);
      }
      T(*w)[TW + 1] = st[wave];
#pragma unroll
      for (int r = 0; r < 4; ++r) w[tile_row<T>(lane, r)][li] = acc[r];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      T out[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < TW / 4; ++q) tile_mfma(-sx[I * TW + li][I * TW + 4 * q + lk], w[4 * q + lk][li], out);
#pragma unroll
      for (int r = 0; r < 4; ++r) sx[I * TW + tile_row<T>(lane, r)][J * TW + li] = out[r];
    }
    __syncthreads();
  }
}

// Load the rows x cols block of G at (r0, c0) into the NB x NB LDS block
// s, padded with the identity (pad_identity) or zeros; every load is
// issued before the first LDS store (addresses clamped into the block).
template <typename T>
__device__ void load_block(Blk<T>& s, const T* __restrict__ G, int ld, int r0, int c0, int rows, int cols,
                           bool pad_identity) {
  const int tid = threadIdx.x;
  T v[NB * NB / 256];
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) {
    const int e = tid + 256 * q;
    const int i = min(e / NB, rows - 1), j = min(e % NB, cols - 1);
    v[q] = G[(size_t)(r0 + i) * ld + c0 + j];
  }
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) {
    const int e = tid + 256 * q;
    const int i = e / NB, j = e % NB;
    s[i][j] = (i < rows && j < cols) ? v[q] : ((pad_identity && i == j) ? T(1) : T(0));
  }
}

// Store the rows x cols part of the LDS block s to G at (r0, c0); with
// `lower` the entries above the diagonal are stored as zeros.
template <typename T>
__device__ void store_block(const Blk<T>& s, T* __restrict__ G, int ld, int r0, int c0, int rows, int cols,
                            bool lower) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) {
    const int e = tid + 256 * q;
    const int i = e / NB, j = e % NB;
    if (i < rows && j < cols) G[(size_t)(r0 + i) * ld + c0 + j] = (!lower || j <= i) ? s[i][j] : T(0);
  }
}

// acc (the wavefront's 32 x 32 quadrant of an NB x NB product, 2 x 2 MFMA
// tiles) += sum_k a(m, k) b(k, n) over k < NB, the operands read from LDS
// through the accessors.  Quadrant of wavefront w: rows 32 (w / 2), columns
// 32 (w % 2); tile (i, j) result r of lane l is element
// (32 (w / 2) + 16 i + tile_row(l, r), 32 (w % 2) + 16 j + l % 16).
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void lds_product(FA a, FB b, T (&acc)[2][2][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  for (int k = 0; k < NB; k += 4) {
    T av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = a(wm + 16 * i + li, k + lk);
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = b(k + lk, wn + 16 * j + li);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) tile_mfma(av[i], bv[j], acc[i][j]);
  }
}

// Visit the elements of the wavefront's quadrant held in acc.
template <typename T, typename F>
__device__ __forceinline__ void quadrant_each(T (&acc)[2][2][4], F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) f(wm + 16 * i + tile_row<T>(lane, r), wn + 16 * j + li, acc[i][j][r]);
}

// Factor the diagonal block A[k0 .. k0+n)^2 (n <= 2 NB) in place and write
// the inverse of its factor to the same block of X (whose part above the
// diagonal the caller has zeroed), in one workgroup of four wavefronts
// with the block in LDS: with halves 1 (the first NB rows) and 2,
//   L11, X11 of block 11;  L21 = A21 X11^T;  A22 -= L21 L21^T;
//   L22, X22 of block 22;  X21 = -X22 (L21 X11),
// the four products on the matrix cores.  Only the lower triangle of A is
// read; the part above the diagonal of the block is left as it was.
template <typename T>
__global__ __launch_bounds__(256) void potrf_node_kernel(T* __restrict__ A, int lda, int k0, int n,
                                                          T* __restrict__ X, int ldx, int* __restrict__ info) {
  __shared__ Blk<T> S0, S1, S2, S3;
  __shared__ Scr<T> st;
  const int b1 = min(n, NB), b2 = n - NB;
  const int k1 = k0 + NB;
  load_block(S0, A, lda, k0, k0, b1, b1, true);
  __syncthreads();
  int bad1 = 0, bad2 = 0;
  factor_inv_lds(S0, S1, st, b1, bad1);
  store_block(S0, A, lda, k0, k0, b1, b1, true);
  store_block(S1, X, ldx, k0, k0, b1, b1, true);
  if (b2 > 0) {
    // L21 = A21 X11^T (X11 lower: entries above its diagonal read as 0)
    load_block(S2, A, lda, k1, k0, b2, NB, false);
    __syncthreads();
    T acc[2][2][4] = {};
    lds_product<T>([&](int m, int k) { return S2[m][k]; },
                   [&](int k, int c) { return k <= c ? S1[c][k] : T(0); }, acc);
    __syncthreads();  // S0 (L11) stored, S2 (A21) read
    quadrant_each(acc, [&](int m, int c, T v) { S0[m][c] = v; });
    __syncthreads();
    store_block(S0, A, lda, k1, k0, b2, NB, false);
    // A22 -= L21 L21^T, then L22, X22
    load_block(S2, A, lda, k1, k1, b2, b2, true);
    __syncthreads();
    quadrant_each(acc, [&](int m, int c, T& v) { v = S2[m][c]; });
    lds_product<T>([&](int m, int k) { return -S0[m][k]; }, [&](int k, int c) { return S0[c][k]; }, acc);
    __syncthreads();
    quadrant_each(acc, [&](int m, int c, T v) { S2[m][c] = v; });
    __syncthreads();
    factor_inv_lds(S2, S3, st, b2, bad2);
    store_block(S2, A, lda, k1, k1, b2, b2, true);
    store_block(S3, X, ldx, k1, k1, b2, b2, true);
    // T = L21 X11 (into S1 once X11 is read), X21 = -X22 T
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = T(0);
    lds_product<T>([&](int m, int k) { return S0[m][k]; }, [&](int k, int c) { return k >= c ? S1[k][c] : T(0); },
                   acc);
    __syncthreads();  // S1 (X11) stored and read
    quadrant_each(acc, [&](int m, int c, T v) { S1[m][c] = v; });
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = T(0);
    lds_product<T>([&](int m, int k) { return k <= m ? -S3[m][k] : T(0); }, [&](int k, int c) { return S1[k][c]; },
                   acc);
    quadrant_each(acc, [&](int m, int c, T v) {
      if (m < b2) X[(size_t)(k1 + m) * ldx + k0 + c] = v;
    });
  }
  if (threadIdx.x == 0 && *info == 0 && (bad1 || bad2)) *info = bad1 ? k0 + bad1 : k1 + bad2;
}

template <typename T>
hipError_t gemm_t(bool ta, bool tb, int M, int N, int K, T alpha, const T* A, int lda, const T* B, int ldb, T beta,
                  T* C, int ldc, hipStream_t st, bool lower = false);
template <>
hipError_t gemm_t<double>(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                          const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st, bool lower) {
  return lower ? mfma_gemm_lower_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st)
               : mfma_gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}
template <>
hipError_t gemm_t<float>(bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda,
                         const float* B, int ldb, float beta, float* C, int ldc, hipStream_t st, bool lower) {
  return lower ? mfma_gemm_lower_f32(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st)
               : mfma_gemm_f32(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
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
// block of X, by recursive halving at a multiple of LEAF:
//   L11, X11 of the leading half;  L21 = A21 X11^T;  A22 -= L21 L21^T;
//   L22, X22 of the trailing half;  X21 = -X22 (L21 X11);
// the leaves (at most LEAF = 2 NB rows) are the one-workgroup node kernel,
// which takes the same steps inside LDS.  Apart from the leaves every step
// is a GEMM whose inner dimension is half the block, so the factorisation
// and the inverse run mostly as large MFMA products.
constexpr int LEAF = 2 * NB;

template <typename T>
hipError_t chol_inv_rec(T* A, int lda, int n0, int n1, T* X, int ldx, T* work, int* info, hipStream_t st) {
  const int nb = (n1 - n0 + LEAF - 1) / LEAF;
  if (nb <= 1) {
    hipLaunchKernelGGL(potrf_node_kernel<T>, dim3(1), dim3(256), 0, st, A, lda, n0, n1 - n0, X, ldx, info);
    return hipGetLastError();
  }
  const int h = n0 + (nb / 2) * LEAF;
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
  e = gemm_t<T>(false, true, r, r, c, T(-1), X21, ldx, X21, ldx, T(1), A22, lda, st, true);  // lower part read
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
  // the largest r x c block of the recursion is the top level's
  const int nb = (n + LEAF - 1) / LEAF;
  const size_t h = (size_t)(nb / 2) * LEAF;
  return std::max<size_t>((size_t)n * NB, h * ((size_t)n - std::min<size_t>(h, n)));
}

hipError_t cholesky_inverse_f64(double* A, int n, int lda, double* X, double* work, int* info, hipStream_t st) {
  return chol_inv<double>(A, n, lda, X, n, work, info, st);
}
hipError_t cholesky_inverse_f32(float* A, int n, int lda, float* X, float* work, int* info, hipStream_t st) {
  return chol_inv<float>(A, n, lda, X, n, work, info, st);
}

}  // namespace wos
