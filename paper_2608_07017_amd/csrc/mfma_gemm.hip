// Dense GEMM on the matrix cores: C = alpha op(A) op(B) + beta C, row-major,
// op = identity or transpose, in FP32 (v_mfma_f32_16x16x4f32) or FP64
// (v_mfma_f64_16x16x4f64), accumulating in the operand precision.  Used by
// the solve path for the assembly of Lambda and Sigma, the normal matrix
// Lambda^T Lambda and the trailing updates of the Cholesky factorisation.
//
// Tiling: a 256-thread workgroup (four wavefronts) owns a 64 x 64 tile of
// C; each wavefront a 32 x 32 quarter made of 2 x 2 MFMA blocks of 16 x 16.
// K advances in slabs of 16 staged in LDS (row-major 16 x 64 slabs of
// op(A)^T and op(B), padded against bank conflicts).
//
// MFMA 16x16x4 operand layout (wave64, lane l): the A operand holds
// A[l % 16][l / 16], the B operand B[l / 16][l % 16]; the 4 results of lane
// l are D[4 (l / 16) + r][l % 16] for FP32 and D[l / 16 + 4 r][l % 16] for
// FP64, r = 0..3 (both checked on gfx950).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "wos_solve_kernels.hpp"

namespace wos {

namespace {

constexpr int GT = 64;   // C tile
constexpr int GK = 16;   // K slab
constexpr int GPAD = 4;  // LDS row padding (elements)

template <typename T>
__device__ __forceinline__ void mfma_16x16x4(T a, T b, T (&acc)[4]);

template <>
__device__ __forceinline__ void mfma_16x16x4<float>(float a, float b, float (&acc)[4]) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  v4f c = {acc[0], acc[1], acc[2], acc[3]};
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  acc[0] = c[0];
  acc[1] = c[1];
  acc[2] = c[2];
  acc[3] = c[3];
}

template <>
__device__ __forceinline__ void mfma_16x16x4<double>(double a, double b, double (&acc)[4]) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  v4d c = {acc[0], acc[1], acc[2], acc[3]};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  acc[0] = c[0];
  acc[1] = c[1];
  acc[2] = c[2];
  acc[3] = c[3];
}

// element (r, c) of op(X) for an X of leading dimension ld
template <bool TRANS, typename S>
__device__ __forceinline__ S op_at(const S* X, int ld, int r, int c) {
  return TRANS ? X[(size_t)c * ld + r] : X[(size_t)r * ld + c];
}

// C (M x N) = alpha op(A) (M x K) op(B) (K x N) + beta C.  Operands may be
// stored in a narrower type SA / SB than the arithmetic type T.
template <typename T, typename SA, typename SB, bool TA, bool TB>
__global__ __launch_bounds__(256) void mfma_gemm_kernel(int M, int N, int K, T alpha, const SA* __restrict__ A,
                                                        int lda, const SB* __restrict__ B, int ldb, T beta,
                                                        T* __restrict__ C, int ldc, int lower) {
  __shared__ T sA[GK][GT + GPAD];  // sA[k][i] = op(A)[m0 + i][k0 + k]
  __shared__ T sB[GK][GT + GPAD];  // sB[k][j] = op(B)[k0 + k][n0 + j]
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  if (lower && n0 >= m0 + GT) return;  // tile above the diagonal
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // wavefront's quarter
  const int li = lane & 15, lk = lane >> 4;

  T acc[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = T(0);

  for (int k0 = 0; k0 < K; k0 += GK) {
    // stage the slabs: 16 x 64 elements each, 4 per thread
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e;
      int kk, ii;
      if (TA) {  // op(A)[i][k] = A[k][i]: consecutive threads walk i
        kk = idx / GT;
        ii = idx % GT;
      } else {  // consecutive threads walk k
        ii = idx / GK;
        kk = idx % GK;
      }
      const int gi = m0 + ii, gk = k0 + kk;
      sA[kk][ii] = (gi < M && gk < K) ? (T)op_at<TA>(A, lda, gi, gk) : T(0);
      int kb, jj;
      if (TB) {  // op(B)[k][j] = B[j][k]: consecutive threads walk k
        jj = idx / GK;
        kb = idx % GK;
      } else {
        kb = idx / GT;
        jj = idx % GT;
      }
      const int gj = n0 + jj, gkb = k0 + kb;
      sB[kb][jj] = (gj < N && gkb < K) ? (T)op_at<TB>(B, ldb, gkb, gj) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      T av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sA[ks + lk][wm + 16 * a + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sB[ks + lk][wn + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) mfma_16x16x4<T>(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm + 16 * a + (std::is_same<T, double>::value ? lk + 4 * r : 4 * lk + r);
        const int gj = n0 + wn + 16 * b + li;
        if (gi < M && gj < N) {
          T* dst = C + (size_t)gi * ldc + gj;
          *dst = alpha * acc[a][b][r] + (beta == T(0) ? T(0) : beta * *dst);
        }
      }
}

// The pipelined kernel for larger products: a 256-thread workgroup owns a
// (32 WM) x (32 WN) tile of C, each wavefront a (16 WM) x (16 WN) quarter
// of WM x WN MFMA blocks.  K advances in slabs of 16: the next slab is
// loaded from global memory into registers while the current one is
// multiplied out of LDS (two LDS buffers, one barrier per slab), with
// 16-byte loads wherever the stored rows are aligned, along M or N for a
// K-major operand and along K otherwise.
// PER consecutive elements from a 16-byte aligned address, in 16-byte loads
template <typename T, typename S, int PER>
__device__ __forceinline__ void load16(const S* src, T (&r)[PER]) {
  if constexpr (std::is_same<S, float>::value) {
#pragma unroll
    for (int c = 0; c < PER / 4; ++c) {
      const float4 q = reinterpret_cast<const float4*>(src)[c];
      r[4 * c] = (T)q.x;
      r[4 * c + 1] = (T)q.y;
      r[4 * c + 2] = (T)q.z;
      r[4 * c + 3] = (T)q.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < PER / 2; ++c) {
      const double2 q = reinterpret_cast<const double2*>(src)[c];
      r[2 * c] = (T)q.x;
      r[2 * c + 1] = (T)q.y;
    }
  }
}

// One operand's share of a K slab: P consecutive elements of one stored
// row.  K-major storage (op(A) = A^T with A K x M, or op(B) = B with B
// K x N): thread t takes slab row k = t / (BX / P) and the P columns from
// (t % (BX / P)) P.  Row-major storage along K (op(A) = A, op(B) = B^T):
// thread t takes stored row x = t / (GK / P) and the P values of k from
// (t % (GK / P)) P.  Out-of-range elements are zero.
template <typename T, typename S, int BX, int P, bool KMAJOR>
struct SlabPart {
  int x, k;  // stored-row / column offsets of this thread within the slab
  __device__ __forceinline__ SlabPart(int tid) {
    if (KMAJOR) {
      k = tid / (BX / P);
      x = (tid % (BX / P)) * P;
    } else {
      x = tid / (GK / P);
      k = (tid % (GK / P)) * P;
    }
  }
  // load from X (ld) for the tile at x0 (extent X_ext) and slab k0 (of K)
  __device__ __forceinline__ void load(const S* X, int ld, int x0, int xext, int k0, int K, int vec, T (&r)[P]) const {
    if (KMAJOR) {
      const int gk = k0 + k, gx = x0 + x;
      const S* src = X + (size_t)gk * ld + gx;
      if (vec && gk < K && gx + P <= xext) {
        load16<T, S, P>(src, r);
      } else {
#pragma unroll
        for (int e = 0; e < P; ++e) r[e] = (gk < K && gx + e < xext) ? (T)src[e] : T(0);
      }
    } else {
      const int gx = x0 + x, gk = k0 + k;
      const S* src = X + (size_t)gx * ld + gk;
      if (vec && gx < xext && gk + P <= K) {
        load16<T, S, P>(src, r);
      } else {
#pragma unroll
        for (int e = 0; e < P; ++e) r[e] = (gx < xext && gk + e < K) ? (T)src[e] : T(0);
      }
    }
  }
  // store into the slab buffer s[k][x]
  template <int LD>
  __device__ __forceinline__ void store(T (*sl)[LD], const T (&r)[P]) const {
    if (KMAJOR) {
#pragma unroll
      for (int e = 0; e < P; ++e) sl[k][x + e] = r[e];
    } else {
#pragma unroll
      for (int e = 0; e < P; ++e) sl[k + e][x] = r[e];
    }
  }
};

template <typename T, typename SA, typename SB, bool TA, bool TB, int WM, int WN>
__global__ __launch_bounds__(256) void mfma_gemm_pipe_kernel(int M, int N, int K, T alpha, const SA* __restrict__ A,
                                                             int lda, const SB* __restrict__ B, int ldb, T beta,
                                                             T* __restrict__ C, int ldc, int vec_a, int vec_b,
                                                             int lower) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int PA = BM * GK / 256, PB = BN * GK / 256;  // elements per thread per slab
  __shared__ T sA[2][GK][BM + GPAD];
  __shared__ T sB[2][GK][BN + GPAD];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (lower && n0 >= m0 + BM) return;  // tile above the diagonal
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 16 * WM, wn = (wave & 1) * 16 * WN;
  const int li = lane & 15, lk = lane >> 4;
  const SlabPart<T, SA, BM, PA, TA> pa(tid);   // op(A) K-major iff A is stored transposed
  const SlabPart<T, SB, BN, PB, !TB> pb(tid);  // op(B) K-major iff B is stored as is

  T acc[WM][WN][4];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = T(0);

  T ra[PA], rb[PB];
  pa.load(A, lda, m0, M, 0, K, vec_a, ra);
  pb.load(B, ldb, n0, N, 0, K, vec_b, rb);
  pa.store(sA[0], ra);
  pb.store(sB[0], rb);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += GK) {
    const bool more = k0 + GK < K;
    if (more) {  // in flight during this slab's MFMAs
      pa.load(A, lda, m0, M, k0 + GK, K, vec_a, ra);
      pb.load(B, ldb, n0, N, k0 + GK, K, vec_b, rb);
    }
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      T av[WM], bv[WN];
#pragma unroll
      for (int a = 0; a < WM; ++a) av[a] = sA[buf][ks + lk][wm + 16 * a + li];
#pragma unroll
      for (int b = 0; b < WN; ++b) bv[b] = sB[buf][ks + lk][wn + 16 * b + li];
#pragma unroll
      for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) mfma_16x16x4<T>(av[a], bv[b], acc[a][b]);
    }
    if (more) {
      pa.store(sA[buf ^ 1], ra);
      pb.store(sB[buf ^ 1], rb);
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm + 16 * a + (std::is_same<T, double>::value ? lk + 4 * r : 4 * lk + r);
        const int gj = n0 + wn + 16 * b + li;
        if (gi < M && gj < N) {
          T* dst = C + (size_t)gi * ldc + gj;
          *dst = alpha * acc[a][b][r] + (beta == T(0) ? T(0) : beta * *dst);
        }
      }
}

// every stored row of an operand starts on a 16-byte boundary
template <typename S>
bool rows_aligned(const S* X, int ld) {
  return ((uintptr_t)X % 16) == 0 && ((size_t)ld * sizeof(S)) % 16 == 0;
}

// Tile autotuner of the FP32 pipelined products: the first product of a
// shape class (transposes, triangle mode, M and N in tiles of 128, K to a
// power of two) that overwrites C (beta = 0) runs with both tilings, timed
// with HIP events on its stream, and the faster is kept for the class.
// Both tilings add the same products in the same order for every element
// of C, so the choice changes the time only, never a bit of the result.
// Other products of an untuned class take the occupancy rule below.
struct TileKey {
  int ta, tb, lower, mt, nt, kl;
  bool operator<(const TileKey& o) const {
    return std::tie(ta, tb, lower, mt, nt, kl) < std::tie(o.ta, o.tb, o.lower, o.mt, o.nt, o.kl);
  }
};
std::mutex g_tile_mu;
std::map<std::pair<int, TileKey>, int> g_tile;  // (device, class) -> 1: 128 x 128 tiles, 0: 64 x 64

template <typename T, typename SA, typename SB>
hipError_t gemm_dispatch(bool ta, bool tb, int M, int N, int K, T alpha, const SA* A, int lda, const SB* B, int ldb,
                         T beta, T* C, int ldc, hipStream_t st, bool lower = false, int force_wide = -1);

template <typename T, typename SA, typename SB>
int tuned_wide(bool ta, bool tb, int M, int N, int K, T alpha, const SA* A, int lda, const SB* B, int ldb, T beta,
               T* C, int ldc, hipStream_t st, bool lower, bool rule) {
  int kl = 0;
  while ((1 << (kl + 1)) <= K) ++kl;
  const TileKey key{ta ? 1 : 0, tb ? 1 : 0, lower ? 1 : 0, (M + 127) / 128, (N + 127) / 128, kl};
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> g(g_tile_mu);
    auto it = g_tile.find({dev, key});
    if (it != g_tile.end()) return it->second;
  }
  if (beta != T(0)) return rule ? 1 : 0;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return rule ? 1 : 0;
  float t_narrow = 0.0f, t_wide = 0.0f;
  bool ok = hipEventRecord(ev[0], st) == hipSuccess &&
            gemm_dispatch<T, SA, SB>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st, lower, 0) ==
                hipSuccess &&
            hipEventRecord(ev[1], st) == hipSuccess &&
            gemm_dispatch<T, SA, SB>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st, lower, 1) ==
                hipSuccess &&
            hipEventRecord(ev[2], st) == hipSuccess && hipEventSynchronize(ev[2]) == hipSuccess &&
            hipEventElapsedTime(&t_narrow, ev[0], ev[1]) == hipSuccess &&
            hipEventElapsedTime(&t_wide, ev[1], ev[2]) == hipSuccess;
  for (auto& e : ev) (void)hipEventDestroy(e);
  const int pick = ok ? (t_wide < t_narrow ? 1 : 0) : (rule ? 1 : 0);
  std::lock_guard<std::mutex> g(g_tile_mu);
  g_tile[{dev, key}] = pick;
  return ok ? -1 - pick : pick;  // -1 - pick: C already holds the product
}

template <typename T, typename SA, typename SB>
hipError_t gemm_dispatch(bool ta, bool tb, int M, int N, int K, T alpha, const SA* A, int lda, const SB* B, int ldb,
                         T beta, T* C, int ldc, hipStream_t st, bool lower, int force_wide) {
  const int lo = lower ? 1 : 0;
  if (M <= 0 || N <= 0) return hipSuccess;
  // larger products: the pipelined kernel, FP32 128 x 128 tiles, FP64
  // 64 x 64 (the accumulators and two LDS buffers of a larger FP64 tile
  // would not fit); products with a side of 64 or less (the lowest level
  // of the recursive Cholesky) keep the 64 x 64 kernel
  if (M > 64 && N > 64 && K >= GK) {
    const int va = rows_aligned(A, lda) ? 1 : 0, vb = rows_aligned(B, ldb) ? 1 : 0;
    // FP32 products too small to give 256 tiles of 128 x 128 take 64 x 64
    // tiles, four times as many workgroups
    // (in the lower-triangle mode the 128 x 128 tiles that remain must
    // still fill the chip four times over, else the last round runs
    // mostly empty)
    const size_t t128 = (size_t)((M + 127) / 128) * ((N + 127) / 128);
    bool wide = std::is_same<T, float>::value && (lower ? (t128 + (M + 127) / 128) / 2 >= 1024 : t128 >= 256);
    if constexpr (std::is_same<T, float>::value) {
      if (force_wide >= 0) {
        wide = force_wide != 0;
      } else {
        const int w = tuned_wide<T, SA, SB>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st, lower, wide);
        if (w < 0) return hipSuccess;  // the timing runs computed the product
        wide = w != 0;
      }
    }
#define WOS_PIPE(W_, TA_, TB_)                                                                                  \
  hipLaunchKernelGGL((mfma_gemm_pipe_kernel<T, SA, SB, TA_, TB_, W_, W_>),                                      \
                     dim3((N + 32 * W_ - 1) / (32 * W_), (M + 32 * W_ - 1) / (32 * W_)), dim3(256), 0, st, M, N, K, \
                     alpha, A, lda, B, ldb, beta, C, ldc, va, vb, lo)
#define WOS_PIPE_W(TA_, TB_) \
  if (wide)                  \
    WOS_PIPE(4, TA_, TB_);   \
  else                       \
    WOS_PIPE(2, TA_, TB_)
    if (ta && !tb) {
      WOS_PIPE_W(true, false);
    } else if (!ta && !tb) {
      WOS_PIPE_W(false, false);
    } else if (!ta && tb) {
      WOS_PIPE_W(false, true);
    } else {
      WOS_PIPE_W(true, true);
    }
#undef WOS_PIPE_W
#undef WOS_PIPE
    return hipGetLastError();
  }
  const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  if (!ta && !tb)
    hipLaunchKernelGGL((mfma_gemm_kernel<T, SA, SB, false, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, lo);
  else if (ta && !tb)
    hipLaunchKernelGGL((mfma_gemm_kernel<T, SA, SB, true, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, lo);
  else if (!ta && tb)
    hipLaunchKernelGGL((mfma_gemm_kernel<T, SA, SB, false, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, lo);
  else
    hipLaunchKernelGGL((mfma_gemm_kernel<T, SA, SB, true, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, lo);
  return hipGetLastError();
}

}  // namespace

hipError_t mfma_gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                         const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  return gemm_dispatch<double, double, double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}

hipError_t mfma_gemm_f32(bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda,
                         const float* B, int ldb, float beta, float* C, int ldc, hipStream_t st) {
  return gemm_dispatch<float, float, float>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}

// Only the tiles of C that reach the diagonal or below (M == N; for
// symmetric products whose upper triangle is never read)
hipError_t mfma_gemm_lower_f64(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                               const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  return gemm_dispatch<double, double, double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st, true);
}
hipError_t mfma_gemm_lower_f32(bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda,
                               const float* B, int ldb, float beta, float* C, int ldc, hipStream_t st) {
  return gemm_dispatch<float, float, float>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st, true);
}
hipError_t mfma_gemm_lower_f64_a32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
                                   const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  return gemm_dispatch<double, float, double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st, true);
}

// FP64 arithmetic on an FP32-stored left operand (the toolbox rows)
hipError_t mfma_gemm_f64_a32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
                             const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  return gemm_dispatch<double, float, double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}

// FP64 arithmetic on an FP32-stored right operand
hipError_t mfma_gemm_f64_b32(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                             const float* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  return gemm_dispatch<double, double, float>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}

}  // namespace wos
