// Cell weights lambda_i = |W_i| / |D| by uniform points, and the small
// element-wise finishing kernels of a build.
//
// The volume points come from Philox tag 1 (counter (q mod 2^32, q >> 32,
// 0, 1) for block q; two points per block in d = 2, one in d = 3), each
// coordinate lo + (hi - lo) * u.  Everything here is FP64 with one rounding
// per operation (no fused multiply-add), so the inside test and the nearest
// site are decided exactly as a plain double-precision evaluation would:
// the per-site counts are integers and reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "wos_device.hpp"
#include "wos_kernels.hpp"

namespace wos {

namespace {

constexpr int kVolBlock = 256;
constexpr int kHistLdsMax = 15360;  // sites whose counts fit in LDS (60 KiB)

#pragma clang fp contract(off)

__device__ __forceinline__ bool inside_exact(const VolumeParams& P, const double* x) {
  switch (P.dom.kind) {
    case WOS_BALL: {
      double s = 0.0;
      for (int a = 0; a < P.dim; ++a) {
        const double t = x[a] - P.dom.c[a];
        const double tt = t * t;
        s = (a == 0) ? tt : s + tt;
      }
      return s < P.dom.rad * P.dom.rad;
    }
    case WOS_BOX: {
      bool in = true;
      for (int a = 0; a < P.dim; ++a) in = in && (x[a] > P.dom.lo[a]) && (x[a] < P.dom.hi[a]);
      return in;
    }
    case WOS_POLYGON: {
      bool odd = false;
      for (int e = 0; e < P.nvert; ++e) {
        const int f = (e + 1 == P.nvert) ? 0 : e + 1;
        const double a0 = P.verts[2 * e], a1 = P.verts[2 * e + 1];
        const double b0 = P.verts[2 * f], b1 = P.verts[2 * f + 1];
        const bool crosses = (a1 > x[1]) != (b1 > x[1]);
        if (crosses) {
          const double num = (x[1] - a1) * (b0 - a0);
          const double xint = a0 + num / (b1 - a1);
          if (x[0] < xint) odd = !odd;
        }
      }
      return odd;
    }
    default: {  // WOS_BOX_MINUS_BALL
      bool in = true;
      for (int a = 0; a < P.dim; ++a) in = in && (x[a] > P.dom.lo[a]) && (x[a] < P.dom.hi[a]);
      double s = 0.0;
      for (int a = 0; a < P.dim; ++a) {
        const double t = x[a] - P.dom.c[a];
        const double tt = t * t;
        s = (a == 0) ? tt : s + tt;
      }
      return in && (s > P.dom.rad * P.dom.rad);
    }
  }
}

__device__ __forceinline__ int nearest_exact(const GridDev<double>& g, int dim, const double* q) {
  int idx = 0;
  for (int a = 0; a < dim; ++a) {
    int c = (int)((q[a] - g.lo[a]) * g.inv_h[a]);
    c = min(max(c, 0), g.n[a] - 1);
    idx = idx * g.n[a] + c;
  }
  const int code = g.cell[idx];
  if (code >= 0) return code;
  const int* lst = g.list + (-code - 1);
  const int cnt = lst[0];
  const int stride = (dim == 2) ? 2 : 4;
  int bj = lst[1];
  double best = 1.0e300;
  for (int c = 0; c < cnt; ++c) {
    const int j = lst[1 + c];
    const double* y = g.pts + (size_t)j * stride;
    double d2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double t = q[a] - y[a];
      const double tt = t * t;
      d2 = (a == 0) ? tt : d2 + tt;
    }
    if (d2 < best) {
      best = d2;
      bj = j;
    }
  }
  return bj;
}

__global__ __launch_bounds__(kVolBlock) void volume_kernel(VolumeParams P) {
  __shared__ unsigned int hist[kHistLdsMax];
  __shared__ unsigned long long s_in;
  const bool use_lds = P.n <= kHistLdsMax;
  if (use_lds)
    for (int j = threadIdx.x; j < P.n; j += kVolBlock) hist[j] = 0u;
  if (threadIdx.x == 0) s_in = 0ull;
  __syncthreads();

  double ext[3];
  for (int a = 0; a < P.dim; ++a) ext[a] = P.dom.hi[a] - P.dom.lo[a];
  unsigned int my_in = 0;
  const int64_t stride = (int64_t)gridDim.x * kVolBlock;
  for (int64_t q = (int64_t)blockIdx.x * kVolBlock + threadIdx.x; q < P.nblocks; q += stride) {
    const uint4 w = philox((uint32_t)((uint64_t)q & 0xFFFFFFFFull), (uint32_t)((uint64_t)q >> 32), 0u,
                           kTagVolume, P.k0, P.k1);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    const int per = (P.dim == 2) ? 2 : 1;
    for (int t = 0; t < per; ++t) {
      const int64_t pid = q * per + t;
      if (pid >= P.npoints) break;
      double x[3];
      for (int a = 0; a < P.dim; ++a) {
        const double u = u01<double>(words[t * P.dim + a]);
        const double prod = ext[a] * u;
        x[a] = P.dom.lo[a] + prod;
      }
      if (!inside_exact(P, x)) continue;
      my_in += 1u;
      const int j = nearest_exact(P.gv, P.dim, x);
      if (use_lds)
        atomicAdd(&hist[j], 1u);
      else
        atomicAdd(&P.counts[j], 1ull);
    }
  }
  atomicAdd(&s_in, (unsigned long long)my_in);
  __syncthreads();
  if (use_lds)
    for (int j = threadIdx.x; j < P.n; j += kVolBlock)
      if (hist[j]) atomicAdd(&P.counts[j], (unsigned long long)hist[j]);
  if (threadIdx.x == 0) atomicAdd(P.inside, s_in);
}

#pragma clang fp contract(fast)

__global__ void lambda_kernel(const unsigned long long* counts, int n, double* lambda) {
  __shared__ unsigned long long part[256];
  unsigned long long s = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) s += counts[j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  const double tot = (double)part[0];
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    lambda[j] = (tot > 0.0) ? (double)counts[j] / tot : 0.0;
}

template <typename T>
__global__ void h_from_counts_kernel(const uint32_t* hc, size_t count, T inv_N, T* h) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    h[i] = T(hc[i]) * inv_N;
}

int grid_for(size_t count, int block) {
  size_t g = (count + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_volume(const VolumeParams& P, hipStream_t stream) {
  if (P.nblocks <= 0) return hipSuccess;
  int grid = (int)((P.nblocks + kVolBlock * 8 - 1) / (kVolBlock * 8));
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(volume_kernel, dim3(grid), dim3(kVolBlock), 0, stream, P);
  return hipGetLastError();
}

hipError_t launch_lambda(const unsigned long long* counts, int n, double* lambda, hipStream_t stream) {
  hipLaunchKernelGGL(lambda_kernel, dim3(1), dim3(256), 0, stream, counts, n, lambda);
  return hipGetLastError();
}

hipError_t launch_h_from_counts_f32(const uint32_t* hc, size_t count, float inv_N, float* h,
                                    hipStream_t stream) {
  hipLaunchKernelGGL(h_from_counts_kernel<float>, dim3(grid_for(count, 256)), dim3(256), 0, stream,
                     hc, count, inv_N, h);
  return hipGetLastError();
}

hipError_t launch_h_from_counts_f64(const uint32_t* hc, size_t count, double inv_N, double* h,
                                    hipStream_t stream) {
  hipLaunchKernelGGL(h_from_counts_kernel<double>, dim3(grid_for(count, 256)), dim3(256), 0, stream,
                     hc, count, inv_N, h);
  return hipGetLastError();
}

}  // namespace wos
