// Device side of the solution operators: the pointer batch handed to the
// application kernel and the launchers of operator.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace wos {

constexpr int kOpBatch = 8;  // right-hand sides per application launch

// Device pointers of one launch's right-hand sides (passed by value).
struct OpBatch {
  const double* f[kOpBatch];
  const double* g[kOpBatch];
  double* u[kOpBatch];
  double* gu[kOpBatch];  // NULL: gradient not wanted for that right-hand side
};

// out[b] = U [f[b]; g[b]] for b < nb; U rows x cols (ld), FP32 or FP64;
// rows [0, grad_rows) go to gu[b], the next n rows to u[b]
hipError_t launch_op_apply(bool f32, const void* U, int rows, int cols, int ld, int n, int grad_rows, int nb,
                           const OpBatch& bt, hipStream_t st);
// X[i][j] *= alpha w[j]
hipError_t launch_scale_cols(double* X, int rows, int cols, int ld, const double* w, double alpha, hipStream_t st);
// Y (ld ldy) += X (dense rows x cols, FP64 or FP32)
hipError_t launch_add_block(double* Y, int rows, int cols, int ldy, bool x_f64, const void* X, hipStream_t st);
hipError_t launch_narrow(size_t count, const double* x, float* y, hipStream_t st);

}  // namespace wos
