// Kernels of the regularised (Tikhonov) solve of the assembled system and
// of its matrix-free FP64 operator, used for mixed-precision iterative
// refinement.
//
// With L = [B^(0); ..; B^(d-1); A] ((d+1) n x m) and, per site i, the
// (d+1) x (d+1) block W_i
//   W_i[a][b] = lambda_i A_ab(x_i)   (a, b < d),   W_i[a][d] = 0,
//   W_i[d][b] = -lambda_i b_b(x_i),  W_i[d][d] = lambda_i c(x_i),
// the system matrix of eq. linear_q is Lambda = L^T W L, Sigma = L^T W [K; H]
// and the right-hand side -A^T (lambda o f) - Sigma g = -L^T (e_d (lambda o f)
// + W [K; H] g).  Vectors over the (d+1) n rows are stored block by block
// (row block a, then site i).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "wos_solve_kernels.hpp"

namespace wos {

namespace {

int nblocks(size_t count, int block) {
  size_t g = (count + block - 1) / block;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

// R (rows (d+1) n, `cols` = m or m + p columns) = W applied to the row
// blocks of [B; A] (left columns) and [K; H] (right columns), in TO.
template <typename T, typename TO>
__global__ void weight_rows_any_kernel(const T* __restrict__ A, const T* __restrict__ B, const T* __restrict__ H,
                                       const T* __restrict__ K, const double* __restrict__ lam,
                                       const double* __restrict__ Ac, const double* __restrict__ bc,
                                       const double* __restrict__ cc, int n, int m, int p, int d, int cols,
                                       TO* __restrict__ R) {
  const size_t total = (size_t)(d + 1) * n * cols;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const size_t col = idx % cols;
    const size_t row = idx / cols;
    const int a = (int)(row / n);
    const int i = (int)(row % n);
    const bool left = col < (size_t)m;
    const size_t jj = left ? col : col - m;
    const size_t w = left ? (size_t)m : (size_t)p;
    const T* G = left ? B : K;
    const T* Z = left ? A : H;
    const double li = lam[i];
    double v = 0.0;
    if (a < d) {
      for (int b = 0; b < d; ++b) {
        const double ab = Ac ? Ac[((size_t)i * d + a) * d + b] : (a == b ? 1.0 : 0.0);
        if (ab != 0.0) v += li * ab * (double)G[((size_t)b * n + i) * w + jj];
      }
    } else {
      if (bc)
        for (int b = 0; b < d; ++b) v -= li * bc[(size_t)i * d + b] * (double)G[((size_t)b * n + i) * w + jj];
      if (cc) v += li * cc[i] * (double)Z[(size_t)i * w + jj];
    }
    R[idx] = (TO)v;
  }
}

// z (block vector) = W y (trans = 0) or W^T y (trans = 1), plus e_d (s o f)
// when f is given
__global__ void apply_w_kernel(int n, int d, const double* __restrict__ lam, const double* __restrict__ Ac,
                               const double* __restrict__ bc, const double* __restrict__ cc,
                               const double* __restrict__ y, int trans, const double* __restrict__ f,
                               double* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double li = lam[i];
  double yv[4] = {0, 0, 0, 0};
  for (int a = 0; a <= d; ++a) yv[a] = y[(size_t)a * n + i];
  auto wab = [&](int a, int b) -> double {  // W_i[a][b]
    if (a < d) {
      if (b == d) return 0.0;
      return li * (Ac ? Ac[((size_t)i * d + a) * d + b] : (a == b ? 1.0 : 0.0));
    }
    if (b < d) return bc ? -li * bc[(size_t)i * d + b] : 0.0;
    return cc ? li * cc[i] : 0.0;
  };
  for (int a = 0; a <= d; ++a) {
    double s = 0.0;
    for (int b = 0; b <= d; ++b) s += (trans ? wab(b, a) : wab(a, b)) * yv[b];
    if (a == d && f) s += li * f[i];
    z[(size_t)a * n + i] = s;
  }
}

// Transposed products y = X^T v over row blocks are summed deterministically:
// block b writes its column sums to part[b][:], then gemv_reduce_kernel adds
// the blocks in order (the result does not depend on the schedule).
//
// part[blockIdx.y][j] = sum_{r in chunk} X[r][j] v[r]
template <typename T>
__global__ __launch_bounds__(256) void gemv_t_split_kernel(const T* __restrict__ X, int rows, int cols, int ld,
                                                           const double* __restrict__ v, double* __restrict__ part,
                                                           int chunk) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  double acc = 0.0;
  for (int r = r0; r < r1; ++r) acc += (double)X[(size_t)r * ld + j] * v[r];
  part[(size_t)blockIdx.y * cols + j] = acc;
}

// Y[t][j] = alpha sum_b part[b][t][j] + beta Y[t][j]  (beta 0: Y not read)
__global__ __launch_bounds__(256) void gemv_reduce_kernel(const double* __restrict__ part, int nrb, int nv, int cols,
                                                          double alpha, double beta, double* __restrict__ Y, int ys) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y;
  if (j >= cols) return;
  double s = 0.0;
  for (int b = 0; b < nrb; ++b) s += part[((size_t)b * nv + t) * cols + j];
  double* y = Y + (size_t)t * ys + j;
  *y = alpha * s + (beta == 0.0 ? 0.0 : beta * *y);
}

// y[i] = alpha sum_j X[i][j] v[j] + beta y[i], one wavefront per row
template <typename T>
__global__ __launch_bounds__(256) void gemv_n_ld_kernel(const T* __restrict__ X, int rows, int cols, int ld,
                                                        const double* __restrict__ v, double alpha, double beta,
                                                        double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  double acc = 0.0;
  for (int j = lane; j < cols; j += 64) acc += (double)X[(size_t)row * ld + j] * v[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) y[row] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[row]);
}

// 16-byte loads of four consecutive FP32 elements
__device__ __forceinline__ void load4(const float* p, double (&x)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  x[0] = q.x;
  x[1] = q.y;
  x[2] = q.z;
  x[3] = q.w;
}

// y[j] += alpha sum_r X[r][j] v[r] for an FP32 X with rows aligned to 16
// bytes and cols % 4 == 0: lane l of wavefront w takes columns
// c0 + 4l .. c0 + 4l + 3 of rows r0 + w, r0 + w + 4, ... (16-byte loads, the
// wavefront reading 1 KB of one row at a time, four rows in flight); the
// four wavefronts' sums
// are added in LDS and each block writes its column sums for its `rpb` rows.
__global__ __launch_bounds__(256) void gemv_t4_kernel(const float* __restrict__ X, int rows, int cols, int ld,
                                                      const double* __restrict__ v, double* __restrict__ part,
                                                      int rpb) {
  __shared__ double sp[3][64][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 256 + 4 * lane;
  const int r0 = blockIdx.y * rpb, r1 = min(rows, r0 + rpb);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < cols) {
    int r = r0 + wave;
    for (; r + 12 < r1; r += 16) {  // four rows in flight per lane
      double xa[4], xb[4], xc[4], xd[4];
      load4(X + (size_t)r * ld + c, xa);
      load4(X + (size_t)(r + 4) * ld + c, xb);
      load4(X + (size_t)(r + 8) * ld + c, xc);
      load4(X + (size_t)(r + 12) * ld + c, xd);
      const double va = v[r], vb = v[r + 4], vc = v[r + 8], vd = v[r + 12];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(xd[q], vd, fma(xc[q], vc, fma(xb[q], vb, fma(xa[q], va, acc[q]))));
    }
    for (; r < r1; r += 4) {
      double xa[4];
      load4(X + (size_t)r * ld + c, xa);
      const double va = v[r];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(xa[q], va, acc[q]);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) sp[wave - 1][lane][q] = acc[q];
  }
  __syncthreads();
  if (wave == 0 && c < cols) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = acc[q] + sp[0][lane][q] + sp[1][lane][q] + sp[2][lane][q];
      part[(size_t)blockIdx.y * cols + c + q] = t;
    }
  }
}

// y[i] = alpha sum_j X[i][j] v[j] + beta y[i] for an FP32 X with rows
// aligned to 16 bytes and cols % 4 == 0: one wavefront per row, 16-byte
// loads (each lane four consecutive elements, the wavefront 1 KB at a time)
__global__ __launch_bounds__(256) void gemv_n4_kernel(const float* __restrict__ X, int rows, int cols, int ld,
                                                      const double* __restrict__ v, double alpha, double beta,
                                                      double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* xr = X + (size_t)row * ld;
  double acc = 0.0, acc2 = 0.0;
  int j = 4 * lane;
  for (; j + 256 < cols; j += 512) {  // two loads in flight per lane
    double xa[4], xb[4];
    load4(xr + j, xa);
    load4(xr + j + 256, xb);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc = fma(xa[q], v[j + q], acc);
      acc2 = fma(xb[q], v[j + 256 + q], acc2);
    }
  }
  if (j < cols) {
    double xa[4];
    load4(xr + j, xa);
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = fma(xa[q], v[j + q], acc);
  }
  acc += acc2;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) y[row] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[row]);
}

// The same two products for NV vectors at once (NV odd, 3..17: the 2k + 1
// points of a saddle-search iteration), so that X is read once for all:
// vector t is V + t vs, its result Y + t ys.
// Y[t][i] = sum_j X[i][j] V[t][j]; one wavefront per row.
template <int NV>
__global__ __launch_bounds__(256) void gemv_n4b_kernel(const float* __restrict__ X, int rows, int cols, int ld,
                                                       const double* __restrict__ V, int vs, double* __restrict__ Y,
                                                       int ys) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* xr = X + (size_t)row * ld;
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) acc[t] = 0.0;
  for (int j = 4 * lane; j < cols; j += 256) {
    double xa[4];
    load4(xr + j, xa);
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const double* vt = V + (size_t)t * vs + j;
      acc[t] = fma(xa[3], vt[3], fma(xa[2], vt[2], fma(xa[1], vt[1], fma(xa[0], vt[0], acc[t]))));
    }
  }
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    double a = acc[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) Y[(size_t)t * ys + row] = a;
  }
}

// part[b][t][j] = sum_{i in block b} X[i][j] V[t][i]: the layout of
// gemv_t4_kernel, the four wavefronts' sums added in LDS one vector at a time.
template <int NV>
__global__ __launch_bounds__(256) void gemv_t4b_kernel(const float* __restrict__ X, int rows, int cols, int ld,
                                                       const double* __restrict__ V, int vs, double* __restrict__ part,
                                                       int rpb) {
  __shared__ double sp[3][64][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 256 + 4 * lane;
  const int r0 = blockIdx.y * rpb, r1 = min(rows, r0 + rpb);
  double acc[NV][4];
#pragma unroll
  for (int t = 0; t < NV; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = 0.0;
  if (c < cols) {
    for (int r = r0 + wave; r < r1; r += 4) {
      double xa[4];
      load4(X + (size_t)r * ld + c, xa);
#pragma unroll
      for (int t = 0; t < NV; ++t) {
        const double vt = V[(size_t)t * vs + r];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[t][q] = fma(xa[q], vt, acc[t][q]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    if (wave > 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) sp[wave - 1][lane][q] = acc[t][q];
    }
    __syncthreads();
    if (wave == 0 && c < cols) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double s = acc[t][q] + sp[0][lane][q] + sp[1][lane][q] + sp[2][lane][q];
        part[((size_t)blockIdx.y * NV + t) * cols + c + q] = s;
      }
    }
    __syncthreads();
  }
}

// The same two batched products for any row layout and either precision:
// one wavefront per row (forward), one thread per column (transposed,
// coalesced across the workgroup, `rpb` rows per block, each block's column
// sums to the partial-sum buffer).
template <typename T, int NV>
__global__ __launch_bounds__(256) void gemv_nb_kernel(const T* __restrict__ X, int rows, int cols, int ld,
                                                      const double* __restrict__ V, int vs, double* __restrict__ Y,
                                                      int ys) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const T* xr = X + (size_t)row * ld;
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) acc[t] = 0.0;
  for (int j = lane; j < cols; j += 64) {
    const double x = (double)xr[j];
#pragma unroll
    for (int t = 0; t < NV; ++t) acc[t] = fma(x, V[(size_t)t * vs + j], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    double a = acc[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) Y[(size_t)t * ys + row] = a;
  }
}

template <typename T, int NV>
__global__ __launch_bounds__(256) void gemv_tb_kernel(const T* __restrict__ X, int rows, int cols, int ld,
                                                      const double* __restrict__ V, int vs, double* __restrict__ part,
                                                      int rpb) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.y * rpb, r1 = min(rows, r0 + rpb);
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) acc[t] = 0.0;
  for (int r = r0; r < r1; ++r) {
    const double x = (double)X[(size_t)r * ld + c];
#pragma unroll
    for (int t = 0; t < NV; ++t) acc[t] = fma(x, V[(size_t)t * vs + r], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < NV; ++t) part[((size_t)blockIdx.y * NV + t) * cols + c] = acc[t];
}

bool rows16(const void* X, int ld, int cols) {
  return ((uintptr_t)X % 16) == 0 && (ld % 4) == 0 && (cols % 4) == 0;
}

// Rows per block of the transposed products: `start` when that still gives
// 256 blocks, otherwise halved down to `floor` so that small products are
// not a few long loops; at most kMaxRowBlocks row blocks (the partial-sum
// buffer's bound).
int rows_per_block(int rows, int cols, int start, int floor) {
  const int cb = (cols + 255) / 256;
  int rpb = start;
  while (rpb > floor && (size_t)cb * ((rows + rpb - 1) / rpb) < 256) rpb /= 2;
  return std::max(rpb, (rows + kMaxRowBlocks - 1) / kMaxRowBlocks);
}

hipError_t reduce_parts(const double* part, int nrb, int nv, int cols, double alpha, double beta, double* Y, int ys,
                        hipStream_t st) {
  hipLaunchKernelGGL(gemv_reduce_kernel, dim3((cols + 255) / 256, nv), dim3(256), 0, st, part, nrb, nv, cols, alpha,
                     beta, Y, ys);
  return hipGetLastError();
}

// y = alpha X^T v + beta y for an FP32 X with 16-byte rows
hipError_t launch_gemv_t4(const float* X, int rows, int cols, int ld, const double* v, double alpha, double beta,
                          double* y, double* part, hipStream_t st) {
  const int rpb = rows_per_block(rows, cols, 512, 32);
  const int nrb = (rows + rpb - 1) / rpb;
  hipLaunchKernelGGL(gemv_t4_kernel, dim3((cols + 255) / 256, nrb), dim3(256), 0, st, X, rows, cols, ld, v, part,
                     rpb);
  return reduce_parts(part, nrb, 1, cols, alpha, beta, y, cols, st);
}

// the same for any rows: one thread per column, 128 rows per block
template <typename T>
hipError_t launch_gemv_t_split(const T* X, int rows, int cols, int ld, const double* v, double alpha, double beta,
                               double* y, double* part, hipStream_t st) {
  const int chunk = std::max(128, (rows + kMaxRowBlocks - 1) / kMaxRowBlocks);
  const int nrb = (rows + chunk - 1) / chunk;
  hipLaunchKernelGGL(gemv_t_split_kernel<T>, dim3((cols + 255) / 256, nrb), dim3(256), 0, st, X, rows, cols, ld, v,
                     part, chunk);
  return reduce_parts(part, nrb, 1, cols, alpha, beta, y, cols, st);
}

__global__ void scale_kernel(int n, double beta, double* __restrict__ y) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride)
    y[i] = beta == 0.0 ? 0.0 : beta * y[i];
}

// out = coef * max_i N[i][i]; one workgroup
template <typename T>
__global__ __launch_bounds__(256) void reg_from_diag_kernel(const T* __restrict__ N, int m, int ld, double coef,
                                                            double* __restrict__ out) {
  __shared__ double s[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) mx = fmax(mx, (double)N[(size_t)i * ld + i]);
  s[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = coef * s[0];
}

// Weighted column sums of squares, stage 1: part[c][j] = sum over the rows
// of chunk c of w[i mod wn] X[i][j]^2 (FP64 accumulation; w NULL: 1).  One
// thread per column, so a wavefront reads 64 consecutive values of a row.
template <typename T>
__global__ __launch_bounds__(256) void colsq_part_kernel(const T* __restrict__ X, int rows, int cols, int ld,
                                                         const double* __restrict__ w, int wn, int chunk,
                                                         double* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  double s = 0.0;
  for (int i = r0; i < r1; ++i) {
    const double x = (double)X[(size_t)i * ld + j];
    s += (w ? w[i % wn] : 1.0) * x * x;
  }
  part[(size_t)blockIdx.y * cols + j] = s;
}

// stage 2: out[j] (+)= sum_c part[c][j], the chunks in order (deterministic)
__global__ void colsq_sum_kernel(const double* __restrict__ part, int nch, int cols, int accumulate,
                                 double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double s = accumulate ? out[j] : 0.0;
  for (int c = 0; c < nch; ++c) s += part[(size_t)c * cols + j];
  out[j] = s;
}

// out = coef * max_j v[j]; one workgroup
__global__ __launch_bounds__(256) void reg_from_vec_kernel(const double* __restrict__ v, int m, double coef,
                                                          double* __restrict__ out) {
  __shared__ double s[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) mx = fmax(mx, v[i]);
  s[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = coef * s[0];
}

__global__ void set_scalar_kernel(double* __restrict__ out, double v) { out[0] = v; }

__global__ void unit_vector_kernel(int m, int j, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = i == j ? 1.0 : 0.0;
}

template <typename T>
__global__ void add_diag_kernel(T* __restrict__ N, int m, int ld, const double* __restrict__ reg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) N[(size_t)i * ld + i] += (T)reg[0];
}

// y (double) = x + s * z with s read from the device (reg) or 1
__global__ void axpy_reg_kernel(int n, const double* __restrict__ x, const double* __restrict__ reg, double sign,
                                const double* __restrict__ z, double* __restrict__ y) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const double s = sign * (reg ? reg[0] : 1.0);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) y[i] = x[i] + s * z[i];
}

__global__ void to_f32_kernel(int n, const double* __restrict__ x, float* __restrict__ y) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) y[i] = (float)x[i];
}

__global__ void add_f32_kernel(int n, const float* __restrict__ d, double* __restrict__ q) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) q[i] += (double)d[i];
}

// Y (rows x cols, TO) = diag(w) X
template <typename TI, typename TO>
__global__ void scale_rows_kernel(const TI* __restrict__ X, int rows, int cols, const double* __restrict__ w,
                                  TO* __restrict__ Y) {
  const size_t total = (size_t)rows * cols;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride)
    Y[e] = (TO)(w[e / cols] * (double)X[e]);
}

}  // namespace

hipError_t launch_scale_rows(bool f64_in, bool f32_out, const void* X, int rows, int cols, const double* w, void* Y,
                             hipStream_t st) {
  const dim3 g(nblocks((size_t)rows * cols, 256)), b(256);
  if (f64_in && !f32_out)
    hipLaunchKernelGGL((scale_rows_kernel<double, double>), g, b, 0, st, (const double*)X, rows, cols, w, (double*)Y);
  else if (f64_in && f32_out)
    hipLaunchKernelGGL((scale_rows_kernel<double, float>), g, b, 0, st, (const double*)X, rows, cols, w, (float*)Y);
  else if (!f64_in && !f32_out)
    hipLaunchKernelGGL((scale_rows_kernel<float, double>), g, b, 0, st, (const float*)X, rows, cols, w, (double*)Y);
  else
    hipLaunchKernelGGL((scale_rows_kernel<float, float>), g, b, 0, st, (const float*)X, rows, cols, w, (float*)Y);
  return hipGetLastError();
}

hipError_t launch_weight_rows_any(bool f64_in, bool f32_out, const void* A, const void* B, const void* H,
                                  const void* K, const double* lam, const double* Ac, const double* bc,
                                  const double* cc, int n, int m, int p, int d, int cols, void* R, hipStream_t st) {
  const size_t total = (size_t)(d + 1) * n * cols;
  const dim3 g(nblocks(total, 256)), b(256);
  if (f64_in && !f32_out)
    hipLaunchKernelGGL((weight_rows_any_kernel<double, double>), g, b, 0, st, (const double*)A, (const double*)B,
                       (const double*)H, (const double*)K, lam, Ac, bc, cc, n, m, p, d, cols, (double*)R);
  else if (f64_in && f32_out)
    hipLaunchKernelGGL((weight_rows_any_kernel<double, float>), g, b, 0, st, (const double*)A, (const double*)B,
                       (const double*)H, (const double*)K, lam, Ac, bc, cc, n, m, p, d, cols, (float*)R);
  else if (!f64_in && !f32_out)
    hipLaunchKernelGGL((weight_rows_any_kernel<float, double>), g, b, 0, st, (const float*)A, (const float*)B,
                       (const float*)H, (const float*)K, lam, Ac, bc, cc, n, m, p, d, cols, (double*)R);
  else
    hipLaunchKernelGGL((weight_rows_any_kernel<float, float>), g, b, 0, st, (const float*)A, (const float*)B,
                       (const float*)H, (const float*)K, lam, Ac, bc, cc, n, m, p, d, cols, (float*)R);
  return hipGetLastError();
}

hipError_t launch_apply_w(int n, int d, const double* lam, const double* Ac, const double* bc, const double* cc,
                          const double* y, bool trans, const double* f, double* z, hipStream_t st) {
  hipLaunchKernelGGL(apply_w_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, d, lam, Ac, bc, cc, y,
                     trans ? 1 : 0, f, z);
  return hipGetLastError();
}

size_t gemv_part_elems(int cols, int nv) { return (size_t)kMaxRowBlocks * (size_t)std::max(nv, 1) * (size_t)cols; }

hipError_t launch_gemv_t_ld(bool f64, const void* X, int rows, int cols, int ld, const double* v, double alpha,
                            double beta, double* y, double* part, hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  if (rows <= 0) {
    hipLaunchKernelGGL(scale_kernel, dim3(nblocks(cols, 256)), dim3(256), 0, st, cols, beta, y);
    return hipGetLastError();
  }
  if (!f64 && rows16(X, ld, cols)) return launch_gemv_t4((const float*)X, rows, cols, ld, v, alpha, beta, y, part, st);
  if (f64) return launch_gemv_t_split((const double*)X, rows, cols, ld, v, alpha, beta, y, part, st);
  return launch_gemv_t_split((const float*)X, rows, cols, ld, v, alpha, beta, y, part, st);
}

hipError_t launch_gemv_t_acc(bool f64, const void* X, int rows, int cols, int ld, const double* v, double alpha,
                             double* y, double* part, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  return launch_gemv_t_ld(f64, X, rows, cols, ld, v, alpha, 1.0, y, part, st);
}

hipError_t launch_gemv_n_ld(bool f64, const void* X, int rows, int cols, int ld, const double* v, double alpha,
                            double beta, double* y, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if (!f64 && rows16(X, ld, cols))
    hipLaunchKernelGGL(gemv_n4_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, (const float*)X, rows, cols, ld, v,
                       alpha, beta, y);
  else if (f64)
    hipLaunchKernelGGL(gemv_n_ld_kernel<double>, dim3((rows + 3) / 4), dim3(256), 0, st, (const double*)X, rows, cols,
                       ld, v, alpha, beta, y);
  else
    hipLaunchKernelGGL(gemv_n_ld_kernel<float>, dim3((rows + 3) / 4), dim3(256), 0, st, (const float*)X, rows, cols,
                       ld, v, alpha, beta, y);
  return hipGetLastError();
}

#define WOS_NV_CASES(M_) M_(3) M_(5) M_(7) M_(9) M_(11) M_(13) M_(15) M_(17)
#define WOS_NV_ALL(M_) \
  M_(1) M_(2) M_(3) M_(4) M_(5) M_(6) M_(7) M_(8) M_(9) M_(10) M_(11) M_(12) M_(13) M_(14) M_(15) M_(16) M_(17)

hipError_t launch_gemv_n4_batch(const float* X, int rows, int cols, int ld, const double* V, int vs, int nv,
                                double* Y, int ys, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if (!rows16(X, ld, cols)) return hipErrorInvalidValue;
  const dim3 g((rows + 3) / 4);
  switch (nv) {
#define WOS_CASE(N_)                                                                                           \
  case N_:                                                                                                     \
    hipLaunchKernelGGL(gemv_n4b_kernel<N_>, g, dim3(256), 0, st, X, rows, cols, ld, V, vs, Y, ys);             \
    break;
    WOS_NV_CASES(WOS_CASE)
#undef WOS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t gemv_batch_generic(bool trans, const T* X, int rows, int cols, int ld, const double* V, int vs, int nv,
                              double* Y, int ys, double* part, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (!trans) {
    const dim3 g((rows + 3) / 4);
    switch (nv) {
#define WOS_CASE(N_)                                                                                 \
  case N_:                                                                                           \
    hipLaunchKernelGGL((gemv_nb_kernel<T, N_>), g, dim3(256), 0, st, X, rows, cols, ld, V, vs, Y, ys); \
    break;
      WOS_NV_ALL(WOS_CASE)
#undef WOS_CASE
      default:
        return hipErrorInvalidValue;
    }
  } else {
    const int rpb = rows_per_block(rows, cols, 512, 16);
    const int nrb = (rows + rpb - 1) / rpb;
    const dim3 g((cols + 255) / 256, nrb);
    switch (nv) {
#define WOS_CASE(N_)                                                                                          \
  case N_:                                                                                                    \
    hipLaunchKernelGGL((gemv_tb_kernel<T, N_>), g, dim3(256), 0, st, X, rows, cols, ld, V, vs, part, rpb);      \
    break;
      WOS_NV_CASES(WOS_CASE)
#undef WOS_CASE
      default:
        return hipErrorInvalidValue;
    }
    return reduce_parts(part, nrb, nv, cols, 1.0, 1.0, Y, ys, st);
  }
  return hipGetLastError();
}

hipError_t launch_gemv_batch(bool f64, bool trans, const void* X, int rows, int cols, int ld, const double* V, int vs,
                             int nv, double* Y, int ys, double* part, hipStream_t st) {
  const bool odd = nv >= 3 && nv <= 17 && (nv & 1);  // the 4-wide kernels' counts
  if (!f64 && odd && rows16(X, ld, cols))
    return trans ? launch_gemv_t4_batch((const float*)X, rows, cols, ld, V, vs, nv, Y, ys, part, st)
                 : launch_gemv_n4_batch((const float*)X, rows, cols, ld, V, vs, nv, Y, ys, st);
  if (f64) return gemv_batch_generic<double>(trans, (const double*)X, rows, cols, ld, V, vs, nv, Y, ys, part, st);
  return gemv_batch_generic<float>(trans, (const float*)X, rows, cols, ld, V, vs, nv, Y, ys, part, st);
}

hipError_t launch_gemv_t4_batch(const float* X, int rows, int cols, int ld, const double* V, int vs, int nv,
                                double* Y, int ys, double* part, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if (!rows16(X, ld, cols)) return hipErrorInvalidValue;
  const int rpb = rows_per_block(rows, cols, 512, 32);
  const int nrb = (rows + rpb - 1) / rpb;
  const dim3 g((cols + 255) / 256, nrb);
  switch (nv) {
#define WOS_CASE(N_)                                                                                           \
  case N_:                                                                                                     \
    hipLaunchKernelGGL(gemv_t4b_kernel<N_>, g, dim3(256), 0, st, X, rows, cols, ld, V, vs, part, rpb);         \
    break;
    WOS_NV_CASES(WOS_CASE)
#undef WOS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return reduce_parts(part, nrb, nv, cols, 1.0, 1.0, Y, ys, st);
}
#undef WOS_NV_CASES
#undef WOS_NV_ALL

int colsq_chunks(int rows) { return std::max(1, std::min(kColsqChunks, (rows + 127) / 128)); }

hipError_t launch_colsq(bool f64, const void* X, int rows, int cols, int ld, const double* w, int wn, bool accumulate,
                        double* part, double* out, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int nch = colsq_chunks(rows);
  const int chunk = (rows + nch - 1) / nch;
  const dim3 g((cols + 255) / 256, nch);
  if (f64)
    hipLaunchKernelGGL(colsq_part_kernel<double>, g, dim3(256), 0, st, (const double*)X, rows, cols, ld, w,
                       std::max(wn, 1), chunk, part);
  else
    hipLaunchKernelGGL(colsq_part_kernel<float>, g, dim3(256), 0, st, (const float*)X, rows, cols, ld, w,
                       std::max(wn, 1), chunk, part);
  hipLaunchKernelGGL(colsq_sum_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, part, nch, cols,
                     accumulate ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_reg_from_vec(const double* v, int m, double coef, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reg_from_vec_kernel, dim3(1), dim3(256), 0, st, v, m, coef, out);
  return hipGetLastError();
}

hipError_t launch_set_scalar(double* out, double v, hipStream_t st) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st, out, v);
  return hipGetLastError();
}

hipError_t launch_unit_vector(int m, int j, double* x, hipStream_t st) {
  hipLaunchKernelGGL(unit_vector_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, j, x);
  return hipGetLastError();
}

hipError_t launch_reg_from_diag(bool f64, const void* N, int m, int ld, double coef, double* out, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(reg_from_diag_kernel<double>, dim3(1), dim3(256), 0, st, (const double*)N, m, ld, coef, out);
  else
    hipLaunchKernelGGL(reg_from_diag_kernel<float>, dim3(1), dim3(256), 0, st, (const float*)N, m, ld, coef, out);
  return hipGetLastError();
}

hipError_t launch_add_diag(bool f64, void* N, int m, int ld, const double* reg, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(add_diag_kernel<double>, dim3((m + 255) / 256), dim3(256), 0, st, (double*)N, m, ld, reg);
  else
    hipLaunchKernelGGL(add_diag_kernel<float>, dim3((m + 255) / 256), dim3(256), 0, st, (float*)N, m, ld, reg);
  return hipGetLastError();
}

hipError_t launch_axpy_reg(int n, const double* x, const double* reg, double sign, const double* z, double* y,
                           hipStream_t st) {
  hipLaunchKernelGGL(axpy_reg_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x, reg, sign, z, y);
  return hipGetLastError();
}

hipError_t launch_to_f32(int n, const double* x, float* y, hipStream_t st) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}

hipError_t launch_add_f32(int n, const float* dlt, double* q, hipStream_t st) {
  hipLaunchKernelGGL(add_f32_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, n, dlt, q);
  return hipGetLastError();
}

}  // namespace wos
