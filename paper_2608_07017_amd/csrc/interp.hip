// Evaluation of a solution off the sites (the approximations of u on the
// partition after eq. min_el_discrete): the query point is binned to its
// nearest site through the same grid the walker bins by (the Voronoi cells
// W_i), then u(x) ~ u_i + <grad u_i, x - x_i>, or u_i without the gradient.
// One thread per point; the grid record and the site are read once per
// point, u and grad u are gathered.  Bound by the random loads (a few per
// point), so the launch is sized by points, not by sites.
#include <hip/hip_runtime.h>

#include "wos_device.hpp"
#include "wos_kernels.hpp"

namespace wos {

namespace {

template <typename T, int D>
__global__ __launch_bounds__(256) void interp_kernel(GridDev<T> g, const double* __restrict__ sites64,
                                                     const double* __restrict__ u, const double* __restrict__ gu,
                                                     int n, const double* __restrict__ x, int64_t npts,
                                                     double* __restrict__ out, int* __restrict__ site) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npts; k += stride) {
    double xd[D];
    T q[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      xd[a] = x[k * D + a];
      q[a] = (T)xd[a];
    }
    const int i = grid_nearest<T, D>(g, g.pts, q);
    double v = u[i];
    if (gu) {
      const double* yi = sites64 + (size_t)i * PtStride<D>::value;
#pragma unroll
      for (int a = 0; a < D; ++a) v += gu[(size_t)a * n + i] * (xd[a] - yi[a]);
    }
    out[k] = v;
    if (site) site[k] = i;
  }
}

template <typename T, int D>
hipError_t launch_d(const GridDev<T>& g, const double* sites64, const double* u, const double* gu, int n,
                    const double* x, int64_t npts, double* out, int* site, hipStream_t st) {
  int64_t blocks = (npts + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((interp_kernel<T, D>), dim3((unsigned)blocks), dim3(256), 0, st, g, sites64, u, gu, n, x,
                     npts, out, site);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_interpolate(int dim, const GridDev<T>& g, const double* sites64, const double* u,
                              const double* gu, int n, const double* x, int64_t npts, double* out, int* site,
                              hipStream_t st) {
  if (npts <= 0) return hipSuccess;
  if (dim == 2) return launch_d<T, 2>(g, sites64, u, gu, n, x, npts, out, site, st);
  if (dim == 3) return launch_d<T, 3>(g, sites64, u, gu, n, x, npts, out, site, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_interpolate<float>(int, const GridDev<float>&, const double*, const double*,
                                              const double*, int, const double*, int64_t, double*, int*,
                                              hipStream_t);
template hipError_t launch_interpolate<double>(int, const GridDev<double>&, const double*, const double*,
                                               const double*, int, const double*, int64_t, double*, int*,
                                               hipStream_t);

}  // namespace wos
