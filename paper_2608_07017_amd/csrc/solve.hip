// Linear-algebra kernels of the solve path (FP64): the coefficient-weighted
// row blocks of the assembly, the transposed GEMM that forms Lambda and
// Sigma, matrix-vector products, and the parallel cyclic Jacobi
// eigensolver behind the truncated-SVD solve.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wos_solve_kernels.hpp"

namespace wos {

namespace {

int blocks_for(size_t count, int block) {
  size_t g = (count + block - 1) / block;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

// ------------------------------------------------------ weighted row blocks
// For each cell i the paper's assembly (Sec. "Second order linear elliptic
// PDEs") needs sum_i lambda_i B_i^T A(x_i) B_i - A^T B^b + A^T diag(lambda c) A.
// Writing L = [B^(0); ..; B^(d-1); A] ((d+1) n x m), this is L^T R with
//   R_a = sum_b diag(lambda A_ab) B^(b)                      (a < d)
//   R_d = -sum_a diag(lambda b_a) B^(a) + diag(lambda c) A,
// and Sigma = L^T S with K, H in place of B, A.  Rows of R (first m columns)
// and S (last p columns) are built side by side in one (d+1) n x (m+p) array.
template <typename T>
__global__ void weight_rows_kernel(const T* __restrict__ A, const T* __restrict__ B,
                                   const T* __restrict__ H, const T* __restrict__ K,
                                   const double* __restrict__ lam, const double* __restrict__ Ac,
                                   const double* __restrict__ bc, const double* __restrict__ cc, int n,
                                   int m, int p, int d, double* __restrict__ R) {
  const size_t ncols = (size_t)m + p;
  const size_t total = (size_t)(d + 1) * n * ncols;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const size_t col = idx % ncols;
    const size_t row = idx / ncols;
    const int a = (int)(row / n);
    const int i = (int)(row % n);
    const bool left = col < (size_t)m;
    const size_t jj = left ? col : col - m;
    const size_t w = left ? (size_t)m : (size_t)p;
    const T* G = left ? B : K;   // gradient operator
    const T* Z = left ? A : H;   // value operator
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
    R[idx] = v;
  }
}

// ------------------------------------------------------------------- GEMM
// C (M x N, row-major, ldc) = L^T X where L is K x M given as (d+1) row
// blocks of n rows each (blocks 0..d-1 from `Lb` with block stride n*M, block
// d from `La`), X is K x N row-major (ldx).  FP64 with 64 x 64 output tiles,
// 16-deep k panels staged in LDS, 4 x 4 outputs per thread.
constexpr int TM = 64, TN = 64, TK = 16;

template <typename T>
__global__ __launch_bounds__(256) void gemm_tn_kernel(const T* __restrict__ Lb, const T* __restrict__ La,
                                                      int nblk, int n, int M, const double* __restrict__ X,
                                                      int ldx, int N, double* __restrict__ C, int ldc,
                                                      double alpha, double beta) {
  __shared__ double sL[TK][TM + 1];
  __shared__ double sX[TK][TN + 1];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const int Ktot = nblk * n;
  for (int k0 = 0; k0 < Ktot; k0 += TK) {
    for (int t = threadIdx.x; t < TK * TM; t += 256) {
      const int kk = t / TM, mm = t % TM;
      const int k = k0 + kk, mcol = m0 + mm;
      double v = 0.0;
      if (k < Ktot && mcol < M) {
        const int blk = k / n, row = k % n;
        const T* src = (blk < nblk - 1) ? Lb + (size_t)blk * n * M : La;
        v = (double)src[(size_t)row * M + mcol];
      }
      sL[kk][mm] = v;
    }
    for (int t = threadIdx.x; t < TK * TN; t += 256) {
      const int kk = t / TN, nn = t % TN;
      const int k = k0 + kk, ncol = n0 + nn;
      sX[kk][nn] = (k < Ktot && ncol < N) ? X[(size_t)k * ldx + ncol] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sL[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sX[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = m0 + ty + 16 * i;
    if (r >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + tx + 16 * j;
      if (c < N) {
        double* dst = C + (size_t)r * ldc + c;
        *dst = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * *dst);
      }
    }
  }
}

// ------------------------------------------------------------------- GEMV
// y[j] = alpha * sum_i X[i][j] v[i] + beta * y[j]   (X rows x cols, row-major)
template <typename T>
__global__ void gemv_t_kernel(const T* __restrict__ X, int rows, int cols, const double* __restrict__ v,
                              double alpha, double beta, double* __restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double acc = 0.0;
  for (int i = 0; i < rows; ++i) acc += (double)X[(size_t)i * cols + j] * v[i];
  y[j] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[j]);
}

// y[i] = alpha * sum_j X[i][j] v[j] + beta * y[i]: one wavefront per row
template <typename T>
__global__ __launch_bounds__(256) void gemv_n_kernel(const T* __restrict__ X, int rows, int cols,
                                                     const double* __restrict__ v, double alpha, double beta,
                                                     double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  double acc = 0.0;
  for (int j = lane; j < cols; j += 64) acc += (double)X[(size_t)row * cols + j] * v[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) y[row] = alpha * acc + (beta == 0.0 ? 0.0 : beta * y[row]);
}

__global__ void axpby_kernel(int n, double a, const double* __restrict__ x, double b,
                             const double* __restrict__ y, double* __restrict__ z) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride)
    z[i] = a * x[i] + b * (y ? y[i] : 0.0);
}

// out[i] = s * lam[i] * poly(u[i]) with poly = c0 + c1 u + c2 u^2 + c3 u^3 - f[i] * cf
__global__ void pointwise_kernel(int n, const double* __restrict__ lam, const double* __restrict__ u,
                                 const double* __restrict__ f, double c0, double c1, double c2, double c3,
                                 double cf, double* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) {
    const double x = u ? u[i] : 0.0;
    const double v = c0 + x * (c1 + x * (c2 + x * c3)) - (f ? cf * f[i] : 0.0);
    out[i] = (lam ? lam[i] : 1.0) * v;
  }
}

// Euler-Lagrange route (eq. gradJ): the site weights of grad J = L^T y,
// L = [B; A], for the energies of the paper's nonlinear examples, with
// s = |p_i|^2, p_i = grad u_i:
//   kind 0, p-Laplace (eq. plaplace)   F = s^(P/2) / P - f u,
//           dF/dp = s^((P-2)/2) p (0 where s = 0, the limit for P > 1),
//           dF/du = -f;
//   kind 1, minimal surface            F = sqrt(1 + s) - f u,
//           dF/dp = p / sqrt(1 + s), dF/du = -f;
//   kind 2, semilinear (Lap u + u^2 = f) F = s / 2 - u^3 / 3 + f u,
//           dF/dp = p, dF/du = f - u^2;
//   kind 3, weighted quadratic ("elliptic div min")
//           F = w (p.A p / 2 + c u^2 / 2 - f u), dF/dp = w A p,
//           dF/du = w (c u - f), with per-site w, A (d x d, row-major) and
//           c, each optional (1, I, 0).
// dF/dp weight factor c(s) with dF/dp = c p:
__device__ inline double energy_cp(int kind, double P, double s) {
  if (kind == 1) return 1.0 / sqrt(1.0 + s);
  if (kind == 2) return 1.0;
  return s > 0.0 ? pow(s, 0.5 * (P - 2.0)) : 0.0;
}

// All weights and the density at the result:
//   y[a n + i] = lambda_i c(s) p_a   (a < d),
//   y[d n + i] = lambda_i dF/du,
//   F[i]       = F(u_i, p_i).
// w A p for kind 3 at site i (pa: d components)
__device__ inline void weighted_Ap(int d, size_t i, const double* pa, const double* cA, double wi, double* q) {
  for (int a = 0; a < d; ++a) {
    double t = 0.0;
    for (int b = 0; b < d; ++b) t += (cA ? cA[(i * d + a) * d + b] : (a == b ? 1.0 : 0.0)) * pa[b];
    q[a] = wi * t;
  }
}

__global__ void energy_weights_kernel(int kind, int n, int d, double P, const double* __restrict__ lam,
                                      const double* __restrict__ u, const double* __restrict__ gu,
                                      const double* __restrict__ f, double* __restrict__ y,
                                      double* __restrict__ F, const double* __restrict__ cA,
                                      const double* __restrict__ cc, const double* __restrict__ cw) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) {
    if (kind == 3) {
      double pa[3] = {0.0, 0.0, 0.0}, q[3];
      for (int a = 0; a < d; ++a) pa[a] = gu[(size_t)a * n + i];
      const double wi = cw ? cw[i] : 1.0, ci = cc ? cc[i] : 0.0, li = lam[i], ui = u[i], fi = f[i];
      weighted_Ap(d, i, pa, cA, wi, q);
      double pq = 0.0;
      for (int a = 0; a < d; ++a) {
        y[(size_t)a * n + i] = li * q[a];
        pq += pa[a] * q[a];
      }
      y[(size_t)d * n + i] = li * wi * (ci * ui - fi);
      F[i] = 0.5 * pq + wi * (0.5 * ci * ui * ui - fi * ui);
      continue;
    }
    double s = 0.0;
    for (int a = 0; a < d; ++a) s += gu[(size_t)a * n + i] * gu[(size_t)a * n + i];
    const double c = energy_cp(kind, P, s);
    const double li = lam[i], ui = u[i], fi = f[i];
    for (int a = 0; a < d; ++a) y[(size_t)a * n + i] = li * c * gu[(size_t)a * n + i];
    double Fi;
    if (kind == 1) {
      y[(size_t)d * n + i] = -li * fi;
      Fi = sqrt(1.0 + s) - fi * ui;
    } else if (kind == 2) {
      y[(size_t)d * n + i] = li * (fi - ui * ui);
      Fi = 0.5 * s - ui * ui * ui / 3.0 + fi * ui;
    } else {
      y[(size_t)d * n + i] = -li * fi;
      Fi = (s > 0.0 ? pow(s, 0.5 * P) : 0.0) / P - fi * ui;
    }
    F[i] = Fi;
  }
}

// The weights inside the iteration: yB[a n + i] = lambda_i c(s) p_a with
// p = gB + kg (gB = B fbar, kg = K g fixed over the iteration); with uA
// (= A fbar) given, also yA[i] = lambda_i (f_i - u_i^2), u = uA + hg (hg =
// H g), the u-dependent dF/du of the semilinear energy.  Several points
// at once: point blockIdx.y reads gB + y sg and uA + y su and writes
// yB + y sy and yA + y sy.
__global__ void energy_wb_kernel(int kind, int n, int d, double P, const double* __restrict__ lam,
                                 const double* __restrict__ gB, const double* __restrict__ kg,
                                 double* __restrict__ yB, const double* __restrict__ uA,
                                 const double* __restrict__ hg, const double* __restrict__ f,
                                 double* __restrict__ yA, size_t sg, size_t su, size_t sy,
                                 const double* __restrict__ cA, const double* __restrict__ cc,
                                 const double* __restrict__ cw) {
  gB += blockIdx.y * sg;
  yB += blockIdx.y * sy;
  yA += blockIdx.y * sy;
  if (uA) uA += blockIdx.y * su;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) {
    double pa[3] = {0.0, 0.0, 0.0};
    double s = 0.0;
    for (int a = 0; a < d; ++a) {
      pa[a] = gB[(size_t)a * n + i] + (kg ? kg[(size_t)a * n + i] : 0.0);
      s += pa[a] * pa[a];
    }
    const double li = lam[i];
    if (kind == 3) {
      const double wi = cw ? cw[i] : 1.0;
      double q[3];
      weighted_Ap(d, i, pa, cA, wi, q);
      for (int a = 0; a < d; ++a) yB[(size_t)a * n + i] = li * q[a];
      if (uA) {
        const double ui = uA[i] + (hg ? hg[i] : 0.0);
        yA[i] = li * wi * ((cc ? cc[i] : 0.0) * ui - f[i]);
      }
      continue;
    }
    const double c = li * energy_cp(kind, P, s);
    for (int a = 0; a < d; ++a) yB[(size_t)a * n + i] = c * pa[a];
    if (uA) {
      const double ui = uA[i] + (hg ? hg[i] : 0.0);
      yA[i] = li * (f[i] - ui * ui);
    }
  }
}

// One Adam step (the appendix on the optimisation of J): m <- b1 m +
// (1 - b1) g, v <- b2 v + (1 - b2) g^2, fbar <- fbar - a_j m / (sqrt(v) + eps),
// with the bias-corrected step a_j computed on the host.  With `reset`,
// g is then set to it (the constant part of the next gradient, onto which
// the next one is accumulated).
__global__ void adam_kernel(int m, double* __restrict__ g, double b1, double b2, double eps, double aj_host,
                            const double* __restrict__ aj_dev, double* __restrict__ mv, double* __restrict__ vv,
                            double* __restrict__ fbar, const double* __restrict__ reset) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const double aj = aj_dev ? *aj_dev : aj_host;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < (size_t)m; j += stride) {
    const double gj = g[j];
    const double mj = b1 * mv[j] + (1.0 - b1) * gj;
    const double vj = b2 * vv[j] + (1.0 - b2) * gj * gj;
    mv[j] = mj;
    vv[j] = vj;
    fbar[j] -= aj * mj / (sqrt(vj) + eps);
    if (reset) g[j] = reset[j];
  }
}

// C[i][j] += sum_k Xrows... : Gram update C += X^T diag(w) X (X rows x cols)
// used for the Newton Hessian A^T diag(w) A.  64 x 64 tiles.
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(const T* __restrict__ X, int rows, int cols,
                                                   const double* __restrict__ w, double* __restrict__ C) {
  __shared__ double sA[TK][TM + 1];
  __shared__ double sB[TK][TN + 1];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < rows; k0 += TK) {
    for (int t = threadIdx.x; t < TK * TM; t += 256) {
      const int kk = t / TM, mm = t % TM;
      const int k = k0 + kk;
      sA[kk][mm] = (k < rows && m0 + mm < cols) ? (double)X[(size_t)k * cols + m0 + mm] * w[k] : 0.0;
      sB[kk][mm] = (k < rows && n0 + mm < cols) ? (double)X[(size_t)k * cols + n0 + mm] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = m0 + ty + 16 * i;
    if (r >= cols) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + tx + 16 * j;
      if (c < cols) C[(size_t)r * cols + c] += acc[i][j];
    }
  }
}

// C = X^T X for a square or rectangular row-major X (rows x cols), FP64 input
__global__ __launch_bounds__(256) void gram64_kernel(const double* __restrict__ X, int rows, int cols,
                                                     double* __restrict__ C) {
  __shared__ double sA[TK][TM + 1];
  __shared__ double sB[TK][TN + 1];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < rows; k0 += TK) {
    for (int t = threadIdx.x; t < TK * TM; t += 256) {
      const int kk = t / TM, mm = t % TM;
      const int k = k0 + kk;
      sA[kk][mm] = (k < rows && m0 + mm < cols) ? X[(size_t)k * cols + m0 + mm] : 0.0;
      sB[kk][mm] = (k < rows && n0 + mm < cols) ? X[(size_t)k * cols + n0 + mm] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = m0 + ty + 16 * i;
    if (r >= cols) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + tx + 16 * j;
      if (c < cols) C[(size_t)r * cols + c] = acc[i][j];
    }
  }
}

// ------------------------------------------------------ Jacobi eigensolver
// Cyclic Jacobi on a symmetric M x M matrix G (M even; a padded zero row
// and column make an odd size even).  Round r of a sweep pairs the indices
// by the round-robin ("circle") schedule: position 0 is fixed and the others
// rotate, position k plays position M-1-k.  All M/2 rotations of a round act
// on disjoint index pairs, so G <- J^T G J and V <- V J are applied to every
// 2 x 2 block at once.  Rotation of pair (p, q) (Rutishauser's formulas):
//   theta = (G_qq - G_pp) / (2 G_pq), t = sgn(theta) / (|theta| + sqrt(theta^2 + 1)),
//   c = 1 / sqrt(t^2 + 1), s = t c,  J = [[c, s], [-s, c]] on (p, q).
__device__ __forceinline__ int rr_player(int pos, int r, int M) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (M - 1);
}

__global__ void jacobi_rot_kernel(const double* __restrict__ G, int M, int r, double* __restrict__ rot,
                                  int* __restrict__ pq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M / 2) return;
  int p = rr_player(k, r, M), q = rr_player(M - 1 - k, r, M);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  const double gpp = G[(size_t)p * M + p], gqq = G[(size_t)q * M + q], gpq = G[(size_t)p * M + q];
  double c = 1.0, s = 0.0;
  if (gpq != 0.0 && fabs(gpq) > 1e-300) {
    const double theta = (gqq - gpp) / (2.0 * gpq);
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
  }
  rot[2 * k] = c;
  rot[2 * k + 1] = s;
  pq[2 * k] = p;
  pq[2 * k + 1] = q;
}

// one thread per (pair i, pair j) 2 x 2 block of G; the extra row blocks
// (pair i = M/2 .. M/2 + M/2 - 1 .. ) update V's columns: thread (i, j) with
// i >= M/2 handles V rows 2 (i - M/2), 2 (i - M/2) + 1 for pair j.
__global__ void jacobi_apply_kernel(double* __restrict__ G, double* __restrict__ V, int M,
                                    const double* __restrict__ rot, const int* __restrict__ pq) {
  const int half = M / 2;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= half) return;
  const int r = pq[2 * j], s = pq[2 * j + 1];
  const double cj = rot[2 * j], sj = rot[2 * j + 1];
  if (i < half) {
    const int p = pq[2 * i], q = pq[2 * i + 1];
    const double ci = rot[2 * i], si = rot[2 * i + 1];
    double* Gp = G + (size_t)p * M;
    double* Gq = G + (size_t)q * M;
    const double a = Gp[r], b = Gp[s], c = Gq[r], d = Gq[s];
    // rows: [p; q] <- [[ci, -si], [si, ci]] [p; q]
    const double a1 = ci * a - si * c, b1 = ci * b - si * d;
    const double c1 = si * a + ci * c, d1 = si * b + ci * d;
    // columns: [r, s] <- [r, s] [[cj, sj], [-sj, cj]]
    Gp[r] = cj * a1 - sj * b1;
    Gp[s] = sj * a1 + cj * b1;
    Gq[r] = cj * c1 - sj * d1;
    Gq[s] = sj * c1 + cj * d1;
  } else {
    const int row0 = 2 * (i - half);
    for (int row = row0; row < row0 + 2 && row < M; ++row) {
      double* Vr = V + (size_t)row * M;
      const double a = Vr[r], b = Vr[s];
      Vr[r] = cj * a - sj * b;
      Vr[s] = sj * a + cj * b;
    }
  }
}

// off = sum_{i != j} G_ij^2, diag = sum_i G_ii^2 (two doubles, atomics)
__global__ void offnorm_kernel(const double* __restrict__ G, int M, double* __restrict__ out) {
  __shared__ double so[256], sd[256];
  double off = 0.0, dg = 0.0;
  const size_t total = (size_t)M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const double v = G[idx];
    if (idx / M == idx % M)
      dg += v * v;
    else
      off += v * v;
  }
  so[threadIdx.x] = off;
  sd[threadIdx.x] = dg;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      so[threadIdx.x] += so[threadIdx.x + h];
      sd[threadIdx.x] += sd[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], so[0]);
    atomicAdd(&out[1], sd[0]);
  }
}

__global__ void set_identity_kernel(double* __restrict__ V, int M) {
  const size_t total = (size_t)M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x)
    V[idx] = (idx / M == idx % M) ? 1.0 : 0.0;
}

// copy an m x m matrix into the top-left of an M x M zero-padded one
__global__ void pad_copy_kernel(const double* __restrict__ src, int m, int lds, double* __restrict__ dst, int M) {
  const size_t total = (size_t)M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t r = idx / M, c = idx % M;
    dst[idx] = (r < (size_t)m && c < (size_t)m) ? src[r * lds + c] : 0.0;
  }
}

__global__ void diag_kernel(const double* __restrict__ G, int M, double* __restrict__ e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) e[i] = G[(size_t)i * M + i];
}

// G = (G + G^T) / 2
__global__ void symmetrize_kernel(double* __restrict__ G, int M) {
  const size_t total = (size_t)M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t r = idx / M, c = idx % M;
    if (r < c) {
      const double v = 0.5 * (G[r * M + c] + G[c * M + r]);
      G[r * M + c] = v;
      G[c * M + r] = v;
    }
  }
}

// out[0] = sum_i w_i x_i y_i (w = 1 when null): one workgroup, a fixed
// order of additions (the value does not depend on the schedule)
__global__ __launch_bounds__(1024) void dot_kernel(int n, const double* __restrict__ x, const double* __restrict__ y,
                                                   const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += (w ? w[i] : 1.0) * x[i] * y[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// out[0] = max_i |e_i| (as the bit pattern of a non-negative double, which
// orders like an unsigned integer); out must be zeroed
__global__ void absmax_kernel(int n, const double* __restrict__ e, unsigned long long* __restrict__ out) {
  unsigned long long best = 0ull;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(e[i]));
    best = b > best ? b : best;
  }
  atomicMax(out, best);
}

// out[0] = #{i : |e_i| > thr}
__global__ void count_above_kernel(int n, const double* __restrict__ e, double thr,
                                   unsigned long long* __restrict__ out) {
  unsigned long long c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    c += fabs(e[i]) > thr ? 1ull : 0ull;
  if (c) atomicAdd(out, c);
}

// Picard coefficient A(x_i) = (1 + u_i^2) I_d, n x d x d
__global__ void picard_coef_kernel(int n, int d, const double* __restrict__ u, double* __restrict__ Ac) {
  const size_t total = (size_t)n * d * d;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / (d * d), ab = idx % (d * d);
    const double ui = u[i];
    Ac[idx] = (ab / d == ab % d) ? 1.0 + ui * ui : 0.0;
  }
}

// z[j] *= filt(e_j): 1/e_j where |e_j| > thr, else 0
__global__ void tsvd_filter_kernel(int M, const double* __restrict__ e, double thr, double* __restrict__ z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const double ej = e[j];
  z[j] = (fabs(ej) > thr) ? z[j] / ej : 0.0;
}

}  // namespace

// ------------------------------------------------------------- launchers
hipError_t launch_weight_rows(bool f64, const void* A, const void* B, const void* H, const void* K,
                              const double* lam, const double* Ac, const double* bc, const double* cc, int n,
                              int m, int p, int d, double* R, hipStream_t st) {
  const size_t total = (size_t)(d + 1) * n * ((size_t)m + p);
  if (f64)
    hipLaunchKernelGGL(weight_rows_kernel<double>, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                       (const double*)A, (const double*)B, (const double*)H, (const double*)K, lam, Ac, bc, cc,
                       n, m, p, d, R);
  else
    hipLaunchKernelGGL(weight_rows_kernel<float>, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                       (const float*)A, (const float*)B, (const float*)H, (const float*)K, lam, Ac, bc, cc, n,
                       m, p, d, R);
  return hipGetLastError();
}

hipError_t launch_gemm_tn(bool f64, const void* Lb, const void* La, int nblk, int n, int M, const double* X,
                          int ldx, int N, double* C, int ldc, double alpha, double beta, hipStream_t st) {
  const dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  if (f64)
    hipLaunchKernelGGL(gemm_tn_kernel<double>, grid, dim3(256), 0, st, (const double*)Lb, (const double*)La,
                       nblk, n, M, X, ldx, N, C, ldc, alpha, beta);
  else
    hipLaunchKernelGGL(gemm_tn_kernel<float>, grid, dim3(256), 0, st, (const float*)Lb, (const float*)La, nblk,
                       n, M, X, ldx, N, C, ldc, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_gemv_t(bool f64, const void* X, int rows, int cols, const double* v, double alpha, double beta,
                         double* y, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(gemv_t_kernel<double>, dim3((cols + 255) / 256), dim3(256), 0, st, (const double*)X, rows,
                       cols, v, alpha, beta, y);
  else
    hipLaunchKernelGGL(gemv_t_kernel<float>, dim3((cols + 255) / 256), dim3(256), 0, st, (const float*)X, rows,
                       cols, v, alpha, beta, y);
  return hipGetLastError();
}

hipError_t launch_gemv_n(bool f64, const void* X, int rows, int cols, const double* v, double alpha, double beta,
                         double* y, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(gemv_n_kernel<double>, dim3((rows + 3) / 4), dim3(256), 0, st, (const double*)X, rows,
                       cols, v, alpha, beta, y);
  else
    hipLaunchKernelGGL(gemv_n_kernel<float>, dim3((rows + 3) / 4), dim3(256), 0, st, (const float*)X, rows, cols,
                       v, alpha, beta, y);
  return hipGetLastError();
}

hipError_t launch_axpby(int n, double a, const double* x, double b, const double* y, double* z, hipStream_t st) {
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, a, x, b, y, z);
  return hipGetLastError();
}

hipError_t launch_pointwise(int n, const double* lam, const double* u, const double* f, double c0, double c1,
                            double c2, double c3, double cf, double* out, hipStream_t st) {
  hipLaunchKernelGGL(pointwise_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, lam, u, f, c0, c1, c2, c3,
                     cf, out);
  return hipGetLastError();
}

hipError_t launch_energy_weights(int kind, int n, int d, double P, const double* lam, const double* u,
                                 const double* gu, const double* f, double* y, double* F, const EnergyCoef& co,
                                 hipStream_t st) {
  if (d < 1 || d > 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy_weights_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, kind, n, d, P, lam, u, gu, f,
                     y, F, co.A, co.c, co.w);
  return hipGetLastError();
}

hipError_t launch_energy_wb(int kind, int n, int d, double P, const double* lam, const double* gB, const double* kg,
                            double* yB, const double* uA, const double* hg, const double* f, double* yA,
                            const EnergyCoef& co, hipStream_t st) {
  if (d < 1 || d > 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy_wb_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, kind, n, d, P, lam, gB, kg, yB, uA,
                     hg, f, yA, (size_t)0, (size_t)0, (size_t)0, co.A, co.c, co.w);
  return hipGetLastError();
}

hipError_t launch_energy_wb_batch(int kind, int n, int d, double P, const double* lam, const double* GB,
                                  const double* kg, double* YB, const double* UA, const double* hg, const double* f,
                                  int nv, const EnergyCoef& co, hipStream_t st) {
  if (d < 1 || d > 3 || nv < 1 || nv > 65535) return hipErrorInvalidValue;
  const size_t dn = (size_t)d * n;
  // point t: gB = GB + t dn, uA = UA + t n, yB = YB + t (d + 1) n, yA = yB + d n
  hipLaunchKernelGGL(energy_wb_kernel, dim3(blocks_for(n, 256), nv), dim3(256), 0, st, kind, n, d, P, lam, GB, kg, YB,
                     UA, hg, f, YB + dn, dn, (size_t)n, dn + n, co.A, co.c, co.w);
  return hipGetLastError();
}

hipError_t launch_adam(int m, double* g, double b1, double b2, double eps, double aj, double* mv, double* vv,
                       double* fbar, const double* reset, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, g, b1, b2, eps, aj,
                     (const double*)nullptr, mv, vv, fbar, reset);
  return hipGetLastError();
}

hipError_t launch_adam_dev(int m, double* g, double b1, double b2, double eps, const double* aj, double* mv,
                           double* vv, double* fbar, const double* reset, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, g, b1, b2, eps, 0.0, aj, mv, vv,
                     fbar, reset);
  return hipGetLastError();
}

hipError_t launch_gram(bool f64, const void* X, int rows, int cols, const double* w, double* C, hipStream_t st) {
  const dim3 grid((cols + TN - 1) / TN, (cols + TM - 1) / TM);
  if (f64)
    hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, st, (const double*)X, rows, cols, w, C);
  else
    hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(256), 0, st, (const float*)X, rows, cols, w, C);
  return hipGetLastError();
}

hipError_t launch_gram64(const double* X, int rows, int cols, double* C, hipStream_t st) {
  const dim3 grid((cols + TN - 1) / TN, (cols + TM - 1) / TM);
  hipLaunchKernelGGL(gram64_kernel, grid, dim3(256), 0, st, X, rows, cols, C);
  return hipGetLastError();
}

hipError_t launch_jacobi_round(double* G, double* V, int M, int r, double* rot, int* pq, hipStream_t st) {
  const int half = M / 2;
  hipLaunchKernelGGL(jacobi_rot_kernel, dim3((half + 255) / 256), dim3(256), 0, st, G, M, r, rot, pq);
  hipLaunchKernelGGL(jacobi_apply_kernel, dim3((half + 255) / 256, half + half), dim3(256), 0, st, G, V, M, rot,
                     pq);
  return hipGetLastError();
}

hipError_t launch_offnorm(const double* G, int M, double* out2, hipStream_t st) {
  hipError_t e = hipMemsetAsync(out2, 0, 2 * sizeof(double), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(offnorm_kernel, dim3(blocks_for((size_t)M * M, 256) > 1024 ? 1024 : blocks_for((size_t)M * M, 256)),
                     dim3(256), 0, st, G, M, out2);
  return hipGetLastError();
}

hipError_t launch_set_identity(double* V, int M, hipStream_t st) {
  hipLaunchKernelGGL(set_identity_kernel, dim3(blocks_for((size_t)M * M, 256)), dim3(256), 0, st, V, M);
  return hipGetLastError();
}

hipError_t launch_pad_copy(const double* src, int m, int lds, double* dst, int M, hipStream_t st) {
  hipLaunchKernelGGL(pad_copy_kernel, dim3(blocks_for((size_t)M * M, 256)), dim3(256), 0, st, src, m, lds, dst, M);
  return hipGetLastError();
}

hipError_t launch_diag(const double* G, int M, double* e, hipStream_t st) {
  hipLaunchKernelGGL(diag_kernel, dim3((M + 255) / 256), dim3(256), 0, st, G, M, e);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* G, int M, hipStream_t st) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for((size_t)M * M, 256)), dim3(256), 0, st, G, M);
  return hipGetLastError();
}

hipError_t launch_dot(int n, const double* x, const double* y, const double* w, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, st, n, x, y, w, out);
  return hipGetLastError();
}

hipError_t launch_absmax(int n, const double* e, double* out, hipStream_t st) {
  hipError_t er = hipMemsetAsync(out, 0, sizeof(double), st);
  if (er != hipSuccess) return er;
  hipLaunchKernelGGL(absmax_kernel, dim3(std::min(64, (n + 255) / 256 + 1)), dim3(256), 0, st, n, e,
                     reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

hipError_t launch_count_above(int n, const double* e, double thr, double* out, hipStream_t st) {
  hipError_t er = hipMemsetAsync(out, 0, sizeof(double), st);
  if (er != hipSuccess) return er;
  hipLaunchKernelGGL(count_above_kernel, dim3(std::min(64, (n + 255) / 256 + 1)), dim3(256), 0, st, n, e, thr,
                     reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

hipError_t launch_picard_coef(int n, int d, const double* u, double* Ac, hipStream_t st) {
  hipLaunchKernelGGL(picard_coef_kernel, dim3(blocks_for((size_t)n * d * d, 256)), dim3(256), 0, st, n, d, u, Ac);
  return hipGetLastError();
}

hipError_t launch_tsvd_filter(int M, const double* e, double thr, double* z, hipStream_t st) {
  hipLaunchKernelGGL(tsvd_filter_kernel, dim3((M + 255) / 256), dim3(256), 0, st, M, e, thr, z);
  return hipGetLastError();
}

}  // namespace wos
