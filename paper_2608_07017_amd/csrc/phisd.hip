// Kernels of the saddle search (p-HiSD, the appendix on the optimisation of
// J) and of the Newton-Schulz inverse of its preconditioner M = A.
//
// The k <= 8 directions v_1..v_k are m-vectors stored one after another
// (V[i m + j]); the small dense algebra on them (inner products with k
// vectors, the updates of fbar and V, the Gram-Schmidt pass) runs in one
// workgroup of 1024 threads that loops over m.  The products with the
// toolbox matrices and with M^-1 are the GEMV kernels of the solver.
#include <hip/hip_runtime.h>

#include "wos_solve_kernels.hpp"

namespace wos {
namespace {

constexpr int kHisdThreads = 1024;

// Sum over the workgroup; every thread gets the result.
__device__ double block_sum(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();  // lds may still be read by a previous call
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  return s;
}

// fbar <- fbar - eta (w - 2 sum_i v_i (v_i^T M w)), where M w = gr (w =
// M^-1 gr), so v_i^T M w = v_i^T gr; then h = 1e-6 max(1, |fbar|_2).
__global__ __launch_bounds__(kHisdThreads) void hisd_fbar_kernel(int m, int k, const double* __restrict__ V,
                                                                 const double* __restrict__ gr,
                                                                 const double* __restrict__ w, double eta,
                                                                 double* __restrict__ fbar, double* __restrict__ h) {
  __shared__ double lds[16];
  double c[8];
  for (int i = 0; i < k; ++i) {
    double s = 0.0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) s += V[(size_t)i * m + j] * gr[j];
    c[i] = block_sum(s, lds);
  }
  double ss = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double r = w[j];
    for (int i = 0; i < k; ++i) r -= 2.0 * c[i] * V[(size_t)i * m + j];
    const double x = fbar[j] - eta * r;
    fbar[j] = x;
    ss += x * x;
  }
  ss = block_sum(ss, lds);
  if (threadIdx.x == 0) h[0] = 1e-6 * fmax(1.0, sqrt(ss));
}

// X[(2i) m + j] = fbar_j + h v_ij, X[(2i + 1) m + j] = fbar_j - h v_ij,
// and X[2k m + j] = fbar_j (the point itself, last).
__global__ void hisd_shift_kernel(int m, int k, const double* __restrict__ fbar, const double* __restrict__ V,
                                  const double* __restrict__ h, double* __restrict__ X) {
  const double hh = h[0];
  const size_t total = (size_t)k * m;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t i = t / m, j = t % m;
    const double v = V[t];
    X[2 * i * m + j] = fbar[j] + hh * v;
    X[(2 * i + 1) * m + j] = fbar[j] - hh * v;
    if (i == 0) X[2 * (size_t)k * m + j] = fbar[j];
  }
}

// HV_i = (G[2i] - G[2i + 1]) / (2h) for i < k, the central difference of
// grad J; and HV_k = G[2k], grad J at the point itself, so that one batched
// product with M^-1 serves both.
__global__ void hisd_hv_kernel(int m, int k, const double* __restrict__ G, const double* __restrict__ h,
                               double* __restrict__ HV) {
  const double inv = 0.5 / h[0];
  const size_t total = (size_t)(k + 1) * m;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t i = t / m, j = t % m;
    HV[t] = i < (size_t)k ? (G[2 * i * m + j] - G[(2 * i + 1) * m + j]) * inv : G[2 * (size_t)k * m + j];
  }
}

// Vn_i = v_i - tau (y_i - v_i (v_i^T M y_i) - 2 sum_{l<i} v_l (v_l^T M y_i))
// with y_i = M^-1 HV_i, so M y_i = HV_i.
__global__ __launch_bounds__(kHisdThreads) void hisd_v_kernel(int m, int k, const double* __restrict__ V,
                                                              const double* __restrict__ HV,
                                                              const double* __restrict__ Y, double tau,
                                                              double* __restrict__ Vn) {
  __shared__ double lds[16];
  for (int i = 0; i < k; ++i) {
    double c[8];
    for (int l = 0; l <= i; ++l) {
      double s = 0.0;
      for (int j = threadIdx.x; j < m; j += blockDim.x) s += V[(size_t)l * m + j] * HV[(size_t)i * m + j];
      c[l] = block_sum(s, lds);
    }
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      double p = Y[(size_t)i * m + j] - c[i] * V[(size_t)i * m + j];
      for (int l = 0; l < i; ++l) p -= 2.0 * c[l] * V[(size_t)l * m + j];
      Vn[(size_t)i * m + j] = V[(size_t)i * m + j] - tau * p;
    }
  }
}

// Gram-Schmidt in the form <x, y>_M = x^T M y, in the order v_1..v_k, with
// MV = M V on entry: v_i <- v_i - <v_l, v_i>_M v_l for l < i (and M v_i
// alongside, as M is linear), then both scaled by <v_i, v_i>_M^(-1/2).
// bad[0] is set to 1 when <v_i, v_i>_M is not positive, before or after the
// projections, or falls below 1e-24 of its value before them (v_i in the
// span of the previous directions, to rounding).
__global__ __launch_bounds__(kHisdThreads) void hisd_gs_kernel(int m, int k, double* __restrict__ V,
                                                               double* __restrict__ MV, int* __restrict__ bad) {
  __shared__ double lds[16];
  for (int i = 0; i < k; ++i) {
    double s0 = 0.0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) s0 += V[(size_t)i * m + j] * MV[(size_t)i * m + j];
    const double nn0 = block_sum(s0, lds);
    for (int l = 0; l < i; ++l) {
      double s = 0.0;
      for (int j = threadIdx.x; j < m; j += blockDim.x) s += V[(size_t)l * m + j] * MV[(size_t)i * m + j];
      const double c = block_sum(s, lds);
      for (int j = threadIdx.x; j < m; j += blockDim.x) {
        V[(size_t)i * m + j] -= c * V[(size_t)l * m + j];
        MV[(size_t)i * m + j] -= c * MV[(size_t)l * m + j];
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) s += V[(size_t)i * m + j] * MV[(size_t)i * m + j];
    const double nn = block_sum(s, lds);
    if (!(nn0 > 0.0) || !(nn > 1e-24 * nn0)) {
      if (threadIdx.x == 0) bad[0] = 1;
      return;
    }
    const double inv = 1.0 / sqrt(nn);
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      V[(size_t)i * m + j] *= inv;
      MV[(size_t)i * m + j] *= inv;
    }
    __syncthreads();
  }
}

// The eigenvectors (columns of the M x M matrix E_vec, eigenvalues e) of
// the k smallest eigenvalues among the first m, in ascending order, into
// Vout (k x m).  Padding columns j >= m are never taken.
__global__ __launch_bounds__(kHisdThreads) void hisd_select_kernel(int Mp, int m, int k, const double* __restrict__ e,
                                                                   const double* __restrict__ Evec,
                                                                   double* __restrict__ Vout) {
  __shared__ double sv[16];
  __shared__ int si[16];
  __shared__ int chosen[8];
  for (int t = 0; t < k; ++t) {
    double best = INFINITY;
    int bi = 0x7fffffff;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      bool used = false;
      for (int q = 0; q < t; ++q) used |= chosen[q] == j;
      const double x = e[j];
      if (!used && (x < best || (x == best && j < bi))) {
        best = x;
        bi = j;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_down(best, o, 64);
      const int oi = __shfl_down(bi, o, 64);
      if (ob < best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
      sv[wv] = best;
      si[wv] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = sv[0];
      int ii = si[0];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
        if (sv[q] < b || (sv[q] == b && si[q] < ii)) {
          b = sv[q];
          ii = si[q];
        }
      // every remaining eigenvalue NaN: take index t (in range) rather than
      // the sentinel
      chosen[t] = (ii >= 0 && ii < m) ? ii : t;
    }
    __syncthreads();
    const int c = chosen[t];
    for (int j = threadIdx.x; j < m; j += blockDim.x) Vout[(size_t)t * m + j] = Evec[(size_t)j * Mp + c];
    __syncthreads();
  }
}

// X = A^T (m x m, FP64), from A stored as T.
template <typename T>
__global__ void transpose_to_f64_kernel(const T* __restrict__ A, int m, double* __restrict__ X) {
  const size_t total = (size_t)m * m;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t i = t / m, j = t % m;
    X[t] = (double)A[j * m + i];
  }
}

// D <- I - D (m x m).
__global__ void identity_minus_kernel(int m, double* __restrict__ D) {
  const size_t total = (size_t)m * m;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t i = t / m, j = t % m;
    D[t] = (i == j ? 1.0 : 0.0) - D[t];
  }
}

// Y[t m + j] = c[j] for t < nv.
__global__ void hisd_broadcast_kernel(int m, int nv, const double* __restrict__ c, double* __restrict__ Y) {
  const size_t total = (size_t)nv * m;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x)
    Y[t] = c[t % m];
}

unsigned grid_for(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_hisd_fbar(int m, int k, const double* V, const double* gr, const double* w, double eta, double* fbar,
                            double* h, hipStream_t st) {
  if (k < 0 || k > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hisd_fbar_kernel, dim3(1), dim3(kHisdThreads), 0, st, m, k, V, gr, w, eta, fbar, h);
  return hipGetLastError();
}

hipError_t launch_hisd_shift(int m, int k, const double* fbar, const double* V, const double* h, double* X,
                             hipStream_t st) {
  hipLaunchKernelGGL(hisd_shift_kernel, dim3(grid_for((size_t)k * m)), dim3(256), 0, st, m, k, fbar, V, h, X);
  return hipGetLastError();
}

hipError_t launch_hisd_hv(int m, int k, const double* G, const double* h, double* HV, hipStream_t st) {
  hipLaunchKernelGGL(hisd_hv_kernel, dim3(grid_for((size_t)(k + 1) * m)), dim3(256), 0, st, m, k, G, h, HV);
  return hipGetLastError();
}

hipError_t launch_hisd_v(int m, int k, const double* V, const double* HV, const double* Y, double tau, double* Vn,
                         hipStream_t st) {
  if (k < 1 || k > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hisd_v_kernel, dim3(1), dim3(kHisdThreads), 0, st, m, k, V, HV, Y, tau, Vn);
  return hipGetLastError();
}

hipError_t launch_hisd_gs(int m, int k, double* V, double* MV, int* bad, hipStream_t st) {
  if (k < 1 || k > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hisd_gs_kernel, dim3(1), dim3(kHisdThreads), 0, st, m, k, V, MV, bad);
  return hipGetLastError();
}

hipError_t launch_hisd_select(int Mp, int m, int k, const double* e, const double* Evec, double* Vout,
                              hipStream_t st) {
  if (k < 1 || k > 8 || k > m || Mp < m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hisd_select_kernel, dim3(1), dim3(kHisdThreads), 0, st, Mp, m, k, e, Evec, Vout);
  return hipGetLastError();
}

hipError_t launch_transpose_to_f64(bool f64, const void* A, int m, double* X, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(transpose_to_f64_kernel<double>, dim3(grid_for((size_t)m * m)), dim3(256), 0, st,
                       (const double*)A, m, X);
  else
    hipLaunchKernelGGL(transpose_to_f64_kernel<float>, dim3(grid_for((size_t)m * m)), dim3(256), 0, st,
                       (const float*)A, m, X);
  return hipGetLastError();
}

hipError_t launch_hisd_broadcast(int m, int nv, const double* c, double* Y, hipStream_t st) {
  hipLaunchKernelGGL(hisd_broadcast_kernel, dim3(grid_for((size_t)nv * m)), dim3(256), 0, st, m, nv, c, Y);
  return hipGetLastError();
}

hipError_t launch_identity_minus(int m, double* D, hipStream_t st) {
  hipLaunchKernelGGL(identity_minus_kernel, dim3(grid_for((size_t)m * m)), dim3(256), 0, st, m, D);
  return hipGetLastError();
}

}  // namespace wos
