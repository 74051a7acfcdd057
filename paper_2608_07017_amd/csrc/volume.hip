// Cell weights lambda_i = |W_i| / |D| by uniform points, and the small
// element-wise finishing kernels of a build.
//
// The volume points are stratified over the bounding box: tiles^d equal
// tiles receive per_tile points each (both powers of two), point p in tile
// p / per_tile (row-major, last axis fastest), so the lanes of a
// wavefront share a tile and mostly a grid cell, and its grid-record loads
// coalesce.  The uniforms come from Philox tag 1 (counter (q mod 2^32,
// q >> 32, 0, 1) for block q; two points per block in d = 2, one in d = 3);
// coordinate a is lo + (hi - lo) * ((c_a + u_a) / tiles) for tile index c_a.
// Everything here is FP64 with one rounding per operation (no fused
// multiply-add), so the inside test and the nearest site are decided
// exactly as a plain double-precision evaluation would: the per-site counts
// are integers and reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "wos_device.hpp"
#include "wos_kernels.hpp"

namespace wos {

namespace {

constexpr int kVolBlock = 1024;
constexpr int kHistLdsMax = 8192;  // sites whose counts are binned in LDS (32 KiB, dynamic)

#pragma clang fp contract(off)

template <int D, int KIND>
__device__ __forceinline__ bool inside_exact(const VolumeParams& P, const double* x) {
  if constexpr (KIND == WOS_BALL) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double t = x[a] - P.dom.c[a];
      const double tt = t * t;
      s = (a == 0) ? tt : s + tt;
    }
    return s < P.dom.rad * P.dom.rad;
  } else if constexpr (KIND == WOS_BOX) {
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; ++a) in = in && (x[a] > P.dom.lo[a]) && (x[a] < P.dom.hi[a]);
    return in;
  } else if constexpr (KIND == WOS_POLYGON) {
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
  } else {  // WOS_BOX_MINUS_BALL
    bool in = true;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      in = in && (x[a] > P.dom.lo[a]) && (x[a] < P.dom.hi[a]);
      const double t = x[a] - P.dom.c[a];
      const double tt = t * t;
      s = (a == 0) ? tt : s + tt;
    }
    return in && (s > P.dom.rad * P.dom.rad);
  }
}

template <int D>
__device__ __forceinline__ double d2_exact(const double* pts, int j, const double* q) {
  const double* y = pts + (size_t)j * PtStride<D>::value;
  double d2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double t = q[a] - y[a];
    const double tt = t * t;
    d2 = (a == 0) ? tt : d2 + tt;
  }
  return d2;
}

template <int D>
__device__ __noinline__ int nearest_exact_list(const GridDev<double>& g, int code, const double* q) {
  const int* lst = g.list + (-code - 1);
  const int cnt = lst[0];
  int bj = lst[1];
  double best = d2_exact<D>(g.pts, bj, q);
  for (int c = 1; c < cnt; ++c) {
    const int j = lst[1 + c];
    const double d2 = d2_exact<D>(g.pts, j, q);
    if (d2 < best) {
      best = d2;
      bj = j;
    }
  }
  return bj;
}

// Exact FP64 nearest site from a loaded cell record (strict '<' over the
// ascending candidates, repeats of the first included: ties to the lowest
// index).
template <int D>
__device__ __forceinline__ int nearest_exact(const GridDev<double>& g, int4 r, const double* q) {
  if (r.x < 0) return nearest_exact_list<D>(g, r.x, q);
  int bj = r.x;
  double best = d2_exact<D>(g.pts, r.x, q);
  const double d1 = d2_exact<D>(g.pts, r.y, q);
  if (d1 < best) {
    best = d1;
    bj = r.y;
  }
  const double d2 = d2_exact<D>(g.pts, r.z, q);
  if (d2 < best) {
    best = d2;
    bj = r.z;
  }
  const double d3 = d2_exact<D>(g.pts, r.w, q);
  if (d3 < best) bj = r.w;
  return bj;
}

template <int D>
__device__ __forceinline__ int cell_exact(const GridDev<double>& g, const double* q) {
  int idx = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int c = (int)((q[a] - g.lo[a]) * g.inv_h[a]);
    c = min(max(c, 0), g.n[a] - 1);
    idx = idx * g.n[a] + c;
  }
  return idx;
}

template <int D, int KIND>
__global__ __launch_bounds__(kVolBlock) void volume_kernel(VolumeParams P) {
  extern __shared__ unsigned int hist[];  // n counters when n <= kHistLdsMax
  __shared__ unsigned long long s_in;
  const bool use_lds = P.n <= kHistLdsMax;
  if (use_lds)
    for (int j = threadIdx.x; j < P.n; j += kVolBlock) hist[j] = 0u;
  if (threadIdx.x == 0) s_in = 0ull;
  __syncthreads();

  double ext[D];
#pragma unroll
  for (int a = 0; a < D; ++a) ext[a] = P.dom.hi[a] - P.dom.lo[a];
  unsigned int my_in = 0;
  constexpr int PER = (D == 2) ? 2 : 1;  // points per Philox block
  const int64_t stride = (int64_t)gridDim.x * kVolBlock;
  for (int64_t q = (int64_t)blockIdx.x * kVolBlock + threadIdx.x; q < P.nblocks; q += stride) {
    const uint4 w = philox((uint32_t)((uint64_t)q & 0xFFFFFFFFull), (uint32_t)((uint64_t)q >> 32), 0u,
                           kTagVolume, P.k0, P.k1);
    double x[PER][D];
    bool ok[PER];
    int4 rec[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      // tile coordinates of point p = q PER + t
      const int64_t p = q * PER + t;
      const int64_t tile = p >> P.point_shift;
      const int64_t tmask = ((int64_t)1 << P.tile_shift) - 1;
      double c[D];
#pragma unroll
      for (int a = 0; a < D; ++a) c[a] = (double)((tile >> (P.tile_shift * (D - 1 - a))) & tmask);
      double u[D];
      if constexpr (D == 2) {
        u[0] = u01<double>(t == 0 ? w.x : w.z);
        u[1] = u01<double>(t == 0 ? w.y : w.w);
      } else {
        u[0] = u01<double>(w.x);
        u[1] = u01<double>(w.y);
        u[2] = u01<double>(w.z);
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double f = (c[a] + u[a]) * P.inv_tiles;  // both steps exact
        const double pa = ext[a] * f;
        x[t][a] = P.dom.lo[a] + pa;
      }
      ok[t] = (p < P.npoints) && inside_exact<D, KIND>(P, x[t]);
      rec[t] = ok[t] ? P.gv.rec[cell_exact<D>(P.gv, x[t])] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      if (!ok[t]) continue;
      my_in += 1u;
      const int j = nearest_exact<D>(P.gv, rec[t], x[t]);
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
  // Two 1024-thread workgroups per CU (32 wavefronts to hide the latency of
  // the record loads), each thread looping over many points: the per-
  // workgroup histogram flush (n atomics) is then paid only 512 times.
  int grid = (int)((P.nblocks + kVolBlock * 4 - 1) / (kVolBlock * 4));
  if (grid > 512) grid = 512;
  if (grid < 1) grid = 1;
  const size_t lds = (P.n <= kHistLdsMax) ? sizeof(unsigned int) * (size_t)P.n : 0;
  const dim3 g(grid), b(kVolBlock);
  if (P.dim == 2) {
    switch (P.dom.kind) {
      case WOS_BALL: hipLaunchKernelGGL((volume_kernel<2, WOS_BALL>), g, b, lds, stream, P); break;
      case WOS_BOX: hipLaunchKernelGGL((volume_kernel<2, WOS_BOX>), g, b, lds, stream, P); break;
      case WOS_POLYGON: hipLaunchKernelGGL((volume_kernel<2, WOS_POLYGON>), g, b, lds, stream, P); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (P.dom.kind) {
      case WOS_BALL: hipLaunchKernelGGL((volume_kernel<3, WOS_BALL>), g, b, lds, stream, P); break;
      case WOS_BOX: hipLaunchKernelGGL((volume_kernel<3, WOS_BOX>), g, b, lds, stream, P); break;
      case WOS_BOX_MINUS_BALL:
        hipLaunchKernelGGL((volume_kernel<3, WOS_BOX_MINUS_BALL>), g, b, lds, stream, P);
        break;
      default: return hipErrorInvalidValue;
    }
  }
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
