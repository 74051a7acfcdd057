// BF16 shadows of a toolbox and the BF16 matrix-core products of the solve.
//
// Shadow layout.  The solve contracts the toolbox rows L = [B^(0); ...;
// B^(d-1); A] ((d+1) n x m) over the sites: Lambda = L^T (W L).  Matrix-core
// BF16 operands take eight consecutive values of the contracted index per
// lane, so the shadows hold L transposed, k-contiguous:
//   S_V (m x (d+1) n):  S_V[j][a n + i] = L[a n + i][j]   (B components, then A)
//   S_G (p x (d+1) n):  the same for [K; H]
// Values are rounded to nearest even from the FP32 value (an FP64 toolbox
// through FP32).
//
// Products: C (FP32) = alpha X Y^T + beta C with X (M x K), Y (N x K) BF16,
// k-contiguous, on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Lane l
// of a 16 x 16 x 32 block holds X[i = l % 16][k = 8 (l / 16) + e] and
// Y[j = l % 16][k = 8 (l / 16) + e], e = 0..7, and receives
// C[4 (l / 16) + r][l % 16], r = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <set>

#include "wos_solve_kernels.hpp"

namespace wos {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// S[c][off + r] = bf16(X[r][c]) for an X of rows x cols (row-major, ld
// cols); S has leading dimension lds.  64 x 64 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void shadow_t_kernel(const T* __restrict__ X, int rows, int cols,
                                                       uint16_t* __restrict__ S, size_t lds, int off) {
  __shared__ uint16_t tile[64][66];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += 4) {
    const int r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < rows && c < cols) ? bf16_rne((float)X[(size_t)r * cols + c]) : (uint16_t)0;
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int c = c0 + cc, r = r0 + tx;
    if (c < cols && r < rows) S[(size_t)c * lds + off + r] = tile[tx][cc];
  }
}

// RT[j][a n + i] = sum_b W_i[a][b] S[j][b n + i]: the weighted rows W L,
// transposed like the shadow, in BF16.  W_i is the per-site block of the
// weighted assembly (A(x_i) for the gradient components, -b(x_i) and c(x_i)
// for the value component, all times lambda_i).  A thread owns one site and
// a chunk of rows j.
template <int D>
__global__ __launch_bounds__(256) void weight_t_kernel(const uint16_t* __restrict__ S, size_t lds, int n, int m,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ Ac, const double* __restrict__ bc,
                                                       const double* __restrict__ cc, int rows_per_block,
                                                       uint16_t* __restrict__ RT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float W[D + 1][D + 1];
  const double li = lam[i];
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int b = 0; b <= D; ++b) {
      double v;
      if (a < D)
        v = b == D ? 0.0 : li * (Ac ? Ac[((size_t)i * D + a) * D + b] : (a == b ? 1.0 : 0.0));
      else
        v = b < D ? (bc ? -li * bc[(size_t)i * D + b] : 0.0) : (cc ? li * cc[i] : 0.0);
      W[a][b] = (float)v;
    }
  const int j0 = blockIdx.y * rows_per_block, j1 = min(m, j0 + rows_per_block);
  for (int j = j0; j < j1; ++j) {
    const uint16_t* s = S + (size_t)j * lds + i;
    float y[D + 1];
#pragma unroll
    for (int b = 0; b <= D; ++b) y[b] = bf16_f32(s[(size_t)b * n]);
    uint16_t* o = RT + (size_t)j * lds + i;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
      float v = 0.0f;
#pragma unroll
      for (int b = 0; b <= D; ++b) v += W[a][b] * y[b];
      o[(size_t)a * n] = bf16_rne(v);
    }
  }
}

// C = alpha X Y^T + beta C.  A workgroup of 64 WGM WGN lanes owns a TM x TN
// tile of C, each wavefront a (TM / WGM) x (TN / WGN) part of 16 x 16 MFMA
// blocks; K advances in slabs of BK = 64 staged in dynamic LDS (rows padded
// to 72 values, so that the 16-byte reads of a lane group fall in distinct
// banks; two buffers), the next slab's 16-byte global loads in flight during
// the current one's MFMAs (two k-steps of 32 per slab and barrier).  Two
// shapes: 256 x 256 with eight wavefronts of 64 x 128 (144 KiB of LDS, one
// workgroup per compute unit; the most reuse of each staged slab) for
// products of at least one tile per compute unit, 128 x 128 with four
// wavefronts of 64 x 64 (72 KiB, two per compute unit) below that.  Every
// element of C adds the same products in the same order in both.
constexpr int BK = 64, BPAD = 8;

template <int TM, int TN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_bf16_kernel(int M, int N, int K, float alpha,
                                                                      const uint16_t* __restrict__ X, size_t ldx,
                                                                      const uint16_t* __restrict__ Y, size_t ldy,
                                                                      float beta, float* __restrict__ C,
                                                                      size_t ldc, int vec) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int RP = NT / 8;  // rows per load pass: 8 threads of 8 values per 64-value row
  constexpr int PX = TM / RP, PY = TN / RP;
  constexpr int FM = TM / WGM / 16, FN = TN / WGN / 16;  // MFMA blocks per wavefront
  static_assert(TM % RP == 0 && TN % RP == 0 && FM > 0 && FN > 0, "tile shape");
  extern __shared__ __align__(16) uint16_t gsm[];
  uint16_t(*sX)[TM][BK + BPAD] = reinterpret_cast<uint16_t(*)[TM][BK + BPAD]>(gsm);
  uint16_t(*sY)[TN][BK + BPAD] = reinterpret_cast<uint16_t(*)[TN][BK + BPAD]>(gsm + 2 * TM * (BK + BPAD));
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave / WGN) * (TM / WGM), wn = (wave % WGN) * (TN / WGN);
  const int li = lane & 15, lk = (lane >> 4) * 8;
  // thread t loads rows t / 8 + RP e of a slab, k chunk (t % 8) 8
  const int lrow = tid >> 3, lkc = (tid & 7) * 8;
  const bool vc = vec != 0;
  auto load = [&](const uint16_t* Z, size_t ld, int z0, int zext, int k0, uint4* r, int P) {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int gz = z0 + lrow + RP * e, gk = k0 + lkc;
      const uint16_t* src = Z + (size_t)gz * ld + gk;
      if (vc && gz < zext && gk + 8 <= K) {
        r[e] = *reinterpret_cast<const uint4*>(src);
      } else {
        uint16_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (gz < zext && gk + q < K) ? src[q] : (uint16_t)0;
        r[e] = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                          v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16));
      }
    }
  };
  f32x4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  uint4 rx[PX], ry[PY];
  load(X, ldx, m0, M, 0, rx, PX);
  load(Y, ldy, n0, N, 0, ry, PY);
#pragma unroll
  for (int e = 0; e < PX; ++e) *reinterpret_cast<uint4*>(&sX[0][lrow + RP * e][lkc]) = rx[e];
#pragma unroll
  for (int e = 0; e < PY; ++e) *reinterpret_cast<uint4*>(&sY[0][lrow + RP * e][lkc]) = ry[e];
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) {
      load(X, ldx, m0, M, k0 + BK, rx, PX);
      load(Y, ldy, n0, N, k0 + BK, ry, PY);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      bf16x8 xv[FM], yv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) xv[a] = *reinterpret_cast<const bf16x8*>(&sX[buf][wm + 16 * a + li][ks + lk]);
#pragma unroll
      for (int b = 0; b < FN; ++b) yv[b] = *reinterpret_cast<const bf16x8*>(&sY[buf][wn + 16 * b + li][ks + lk]);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xv[a], yv[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int e = 0; e < PX; ++e) *reinterpret_cast<uint4*>(&sX[buf ^ 1][lrow + RP * e][lkc]) = rx[e];
#pragma unroll
      for (int e = 0; e < PY; ++e) *reinterpret_cast<uint4*>(&sY[buf ^ 1][lrow + RP * e][lkc]) = ry[e];
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm + 16 * a + (lane >> 4) * 4 + r;
        const int gj = n0 + wn + 16 * b + li;
        if (gi < M && gj < N) {
          float* dst = C + (size_t)gi * ldc + gj;
          *dst = alpha * acc[a][b][r] + (beta == 0.0f ? 0.0f : beta * *dst);
        }
      }
}

// y (K) = alpha S^T v + beta y for a BF16 S (rows x K, ld), v FP64: partial
// sums over row blocks (FP64), added in block order.
constexpr int kBfRowBlocks = 64;

// A thread owns 8 consecutive columns (one 16-byte load per row when the
// rows are 16-byte aligned).
__global__ __launch_bounds__(256) void gemv_t_bf16_part_kernel(const uint16_t* __restrict__ S, int rows, int K,
                                                               size_t ld, const double* __restrict__ v,
                                                               int rows_per_block, int vec, double* __restrict__ part) {
  const int k0 = 8 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (k0 >= K) return;
  const int r0 = blockIdx.y * rows_per_block, r1 = min(rows, r0 + rows_per_block);
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (vec && k0 + 8 <= K) {
    for (int r = r0; r < r1; ++r) {
      const uint4 q = *reinterpret_cast<const uint4*>(S + (size_t)r * ld + k0);
      const double vr = v[r];
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        s[2 * e] += (double)__uint_as_float(w[e] << 16) * vr;
        s[2 * e + 1] += (double)__uint_as_float(w[e] & 0xFFFF0000u) * vr;
      }
    }
  } else {
    for (int r = r0; r < r1; ++r) {
      const double vr = v[r];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (k0 + e < K) s[e] += (double)bf16_f32(S[(size_t)r * ld + k0 + e]) * vr;
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (k0 + e < K) part[(size_t)blockIdx.y * K + k0 + e] = s[e];
}

__global__ void gemv_t_bf16_reduce_kernel(int K, int nb, const double* __restrict__ part, double alpha, double beta,
                                          double* __restrict__ y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * K + k];
  y[k] = alpha * s + (beta == 0.0 ? 0.0 : beta * y[k]);
}

// out[c n + i] (c = 0..d) of the apply: y = S_V^T fbar + S_G^T g, split into
// grad u (d x n) and u (n)
__global__ void split_apply_kernel(int n, int d, const double* __restrict__ y, double* __restrict__ u,
                                   double* __restrict__ grad_u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[i] = y[(size_t)d * n + i];
  if (grad_u)
    for (int a = 0; a < d; ++a) grad_u[(size_t)a * n + i] = y[(size_t)a * n + i];
}

unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_shadow_t(bool f64, const void* X, int rows, int cols, uint16_t* S, size_t lds, int off,
                           hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const dim3 g(nblk(cols, 64), nblk(rows, 64)), b(256);
  if (f64)
    hipLaunchKernelGGL(shadow_t_kernel<double>, g, b, 0, st, (const double*)X, rows, cols, S, lds, off);
  else
    hipLaunchKernelGGL(shadow_t_kernel<float>, g, b, 0, st, (const float*)X, rows, cols, S, lds, off);
  return hipGetLastError();
}

hipError_t launch_weight_t_bf16(const uint16_t* S, int n, int m, int d, const double* lam, const double* Ac,
                                const double* bc, const double* cc, uint16_t* RT, hipStream_t st) {
  if (n <= 0 || m <= 0) return hipSuccess;
  const size_t lds = (size_t)(d + 1) * n;
  const int rpb = 64;
  const dim3 g(nblk(n, 256), nblk(m, rpb)), b(256);
  if (d == 2)
    hipLaunchKernelGGL(weight_t_kernel<2>, g, b, 0, st, S, lds, n, m, lam, Ac, bc, cc, rpb, RT);
  else
    hipLaunchKernelGGL(weight_t_kernel<3>, g, b, 0, st, S, lds, n, m, lam, Ac, bc, cc, rpb, RT);
  return hipGetLastError();
}

// One tile shape's launch; the LDS attribute (beyond the default 64 KiB of
// dynamic LDS) is set once per device.
template <int TM, int TN, int WGM, int WGN>
hipError_t launch_gemm_bf16(int M, int N, int K, float alpha, const uint16_t* X, size_t ldx, const uint16_t* Y,
                            size_t ldy, float beta, float* C, size_t ldc, bool vec, hipStream_t st) {
  auto kern = gemm_nt_bf16_kernel<TM, TN, WGM, WGN>;
  const size_t lds = 2 * (size_t)(TM + TN) * (BK + BPAD) * sizeof(uint16_t);
  {
    static std::mutex mu;
    static std::set<int> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g_(mu);
    if (!done.count(dev)) {
      const hipError_t e =
          hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      done.insert(dev);
    }
  }
  hipLaunchKernelGGL(kern, dim3(nblk(N, TN), nblk(M, TM)), dim3(64 * WGM * WGN), lds, st, M, N, K, alpha, X, ldx, Y,
                     ldy, beta, C, ldc, vec ? 1 : 0);
  return hipGetLastError();
}

hipError_t gemm_nt_bf16(int M, int N, int K, float alpha, const uint16_t* X, size_t ldx, const uint16_t* Y,
                        size_t ldy, float beta, float* C, size_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const bool vec = ((uintptr_t)X % 16) == 0 && ((uintptr_t)Y % 16) == 0 && ldx % 8 == 0 && ldy % 8 == 0;
  // the 256 x 256 tiles once there is at least one per compute unit
  if ((size_t)nblk(M, 256) * nblk(N, 256) >= 256)
    return launch_gemm_bf16<256, 256, 4, 2>(M, N, K, alpha, X, ldx, Y, ldy, beta, C, ldc, vec, st);
  return launch_gemm_bf16<128, 128, 2, 2>(M, N, K, alpha, X, ldx, Y, ldy, beta, C, ldc, vec, st);
}

size_t gemv_t_bf16_part_elems(int K) { return (size_t)kBfRowBlocks * (size_t)K; }

hipError_t launch_gemv_t_bf16(const uint16_t* S, int rows, int K, size_t ld, const double* v, double alpha,
                              double beta, double* y, double* part, hipStream_t st) {
  if (K <= 0) return hipSuccess;
  const int nb = std::max(1, std::min(kBfRowBlocks, (rows + 63) / 64));
  const int rpb = (rows + nb - 1) / nb;
  const int vec = ((uintptr_t)S % 16) == 0 && ld % 8 == 0;
  hipLaunchKernelGGL(gemv_t_bf16_part_kernel, dim3(nblk(K, 8 * 256), nb), dim3(256), 0, st, S, rows, K, ld, v, rpb,
                     vec, part);
  hipLaunchKernelGGL(gemv_t_bf16_reduce_kernel, dim3(nblk(K, 256)), dim3(256), 0, st, K, nb, (const double*)part,
                     alpha, beta, y);
  return hipGetLastError();
}

hipError_t launch_split_apply(int n, int d, const double* y, double* u, double* grad_u, hipStream_t st) {
  hipLaunchKernelGGL(split_apply_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, d, y, u, grad_u);
  return hipGetLastError();
}

}  // namespace wos
