// Kernel launchers (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include "wos_types.hpp"

namespace wos {

size_t walker_lds_bytes(int dim, int m, int p, int nseg, bool f64);
size_t walker_window_lds_bytes(int dim, int pc, int pb, int npv, int npb, int nseg);
int walker_block_size(size_t lds);
hipError_t launch_walker_f32(const WalkerParams<float>& P, int dim, int kind, int items,
                             hipStream_t stream);
hipError_t launch_walker_f64(const WalkerParams<double>& P, int dim, int kind, int items,
                             hipStream_t stream);

// X (rows x cols, 4-byte elements, row-major) <- X[:, rank] in place;
// cols <= permute_max_cols().
size_t permute_max_cols();
hipError_t launch_permute_cols(void* X, int rows, int cols, const int* rank, hipStream_t st);

hipError_t launch_volume(const VolumeParams& P, hipStream_t stream);
hipError_t launch_lambda(const unsigned long long* counts, int n, double* lambda,
                         hipStream_t stream);
hipError_t launch_h_from_counts_f32(const uint32_t* hc, size_t count, float inv_N, float* h,
                                    hipStream_t stream);
hipError_t launch_h_from_counts_f64(const uint32_t* hc, size_t count, double inv_N, double* h,
                                    hipStream_t stream);

// u[i] = sum_j M[i,j] x[j] + sum_j N[i,j] y[j] for the rows of `batch`
// independent (M, N) pairs laid out back to back.
hipError_t launch_apply_f32(const float* M, int rows, int cols_m, const double* x, const float* N,
                            int cols_n, const double* y, double* out, int batch, hipStream_t stream);
hipError_t launch_apply_f64(const double* M, int rows, int cols_m, const double* x,
                            const double* N, int cols_n, const double* y, double* out, int batch,
                            hipStream_t stream);

// out[k] = u[i] (+ <gu[:, i], x_k - y_i> when gu is given), i the nearest
// site of x_k by the site grid g; site[k] = i when site is given.
template <typename T>
hipError_t launch_interpolate(int dim, const GridDev<T>& g, const double* sites64, const double* u,
                              const double* gu, int n, const double* x, int64_t npts, double* out, int* site,
                              hipStream_t st);

}  // namespace wos
