// Solution operators of linear problems (C ABI wos_operator_*).
//
// For fixed coefficients the Tikhonov solve of eq. linear_q and the
// reconstruction u = A q + H g form a linear map of the data (f, g).  The
// preparation writes that map out as dense matrices, in FP64 on the matrix
// cores, with the same Lambda, Sigma and regularisation as wos_solve:
//
//   R          = W [L | K;H]              weighted rows, (d+1) n x (m + p)
//   [Lambda|S] = L^T R                    m x (m + p)
//   N          = Lambda^T Lambda + reg I, reg = rcond^2 max_j N_jj
//   X          = chol(N)^{-1}             so N^{-1} = X^T X
//   Y          = X^T (X Lambda^T)         = N^{-1} Lambda^T
//   V          = Y [-A^T diag(lambda) | -S]           m x (n + p)
//   U          = [B; A] V + [0 | K; H]    ((d+1) n or n) x (n + p)
//
// with L = [B^(0); ..; B^(d-1); A] and W the per-site coefficient blocks.
// The right-hand side of eq. linear_q is -A^T (lambda o f) - S g, so
// q = V [f; g] and u = A q + H g = U [f; g] (the rows of U past the
// gradient rows); the rows of B give grad u.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "toolbox.hpp"
#include "wos_operator.hpp"
#include "wos_solve_kernels.hpp"

namespace wos {
void set_last_error(const char* msg);  // api.cpp
}

using namespace wos;

struct wos_operator {
  const wos_toolbox* tb = nullptr;
  int n = 0, m = 0, p = 0, d = 0;
  bool grad = false, f32 = false;
  int rows = 0, cols = 0;  // U: rows = (grad ? d + 1 : 1) n, cols = n + p
  int ld = 0;              // row stride of U: cols rounded up to a multiple of 4
  void* U = nullptr;
  double reg = 0.0;
  size_t bytes = 0;
  double prep_ms = 0.0;
};

namespace {

wos_status ofail(wos_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  wos::set_last_error(buf);
  return s;
}

#define OHIP(call)                                                                                    \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return ofail(e_ == hipErrorOutOfMemory ? WOS_ENOMEM : WOS_EDEVICE, "%s: %s (%s:%d)", #call,     \
                   hipGetErrorString(e_), __FILE__, __LINE__);                                        \
  } while (0)

// Temporary device buffers of one preparation, freed on every exit.
struct Temps {
  std::vector<void*> ptrs;
  ~Temps() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <typename T>
  wos_status get(T** out, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess)
      return ofail(WOS_ENOMEM, "operator preparation: hipMalloc(%zu) failed", count * sizeof(T));
    ptrs.push_back(q);
    *out = static_cast<T*>(q);
    return WOS_OK;
  }
};

#define OTRY(x)                   \
  do {                            \
    const wos_status s_ = (x);    \
    if (s_ != WOS_OK) return s_;  \
  } while (0)

// C = alpha op(T) op(Z) + beta C with T a toolbox array (FP32 or FP64)
// on the left, or on the right
hipError_t gemm_tb_left(bool f64, bool ta, int M, int N, int K, double alpha, const void* T, int ldt, const double* Z,
                        int ldz, double beta, double* C, int ldc, hipStream_t st) {
  if (f64)
    return mfma_gemm_f64(ta, false, M, N, K, alpha, static_cast<const double*>(T), ldt, Z, ldz, beta, C, ldc, st);
  return mfma_gemm_f64_a32(ta, false, M, N, K, alpha, static_cast<const float*>(T), ldt, Z, ldz, beta, C, ldc, st);
}
hipError_t gemm_tb_right_t(bool f64, int M, int N, int K, double alpha, const double* Z, int ldz, const void* T,
                           int ldt, double beta, double* C, int ldc, hipStream_t st) {
  if (f64)
    return mfma_gemm_f64(false, true, M, N, K, alpha, Z, ldz, static_cast<const double*>(T), ldt, beta, C, ldc, st);
  return mfma_gemm_f64_b32(false, true, M, N, K, alpha, Z, ldz, static_cast<const float*>(T), ldt, beta, C, ldc, st);
}

wos_status prepare(wos_operator* op, const wos_toolbox* tb, const wos_coeffs* co, hipStream_t st) {
  const int n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const bool f64 = tb->f64;
  const size_t mp = (size_t)m + p, np = (size_t)n + p;
  const double rcond = co->rcond > 0 ? co->rcond : 1e-3;
  Temps t;
  double *R, *LS, *N, *X, *T1, *Y, *V, *work, *regv, *U64;
  int* info;
  OTRY(t.get(&R, (size_t)(d + 1) * n * mp));
  OTRY(t.get(&LS, (size_t)m * mp));
  OTRY(t.get(&N, (size_t)m * m));
  OTRY(t.get(&X, (size_t)m * m));
  OTRY(t.get(&T1, (size_t)m * m));
  OTRY(t.get(&Y, (size_t)m * m));
  OTRY(t.get(&V, (size_t)m * np));
  OTRY(t.get(&work, chol_work_elems(m)));
  OTRY(t.get(&regv, 1));
  OTRY(t.get(&info, 2));
  const size_t ldu = (size_t)op->ld;
  OTRY(t.get(&U64, (size_t)op->rows * ldu));

  hipEvent_t e0 = nullptr, e1 = nullptr;
  OHIP(hipEventCreate(&e0));
  OHIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eg{e0, e1};
  OHIP(hipEventRecord(e0, st));
  OHIP(hipMemsetAsync(info, 0, 2 * sizeof(int), st));
  OHIP(hipMemsetAsync(U64, 0, sizeof(double) * (size_t)op->rows * ldu, st));  // zero row padding

  // [Lambda | S] = L^T W [L | K;H]
  OHIP(launch_weight_rows_any(f64, false, tb->d_A, tb->d_B, tb->d_H, tb->d_K, tb->d_lambda, co->A, co->b, co->c, n, m,
                              p, d, (int)mp, R, st));
  OHIP(gemm_tb_left(f64, true, m, (int)mp, d * n, 1.0, tb->d_B, m, R, (int)mp, 0.0, LS, (int)mp, st));
  OHIP(gemm_tb_left(f64, true, m, (int)mp, n, 1.0, tb->d_A, m, R + (size_t)d * n * mp, (int)mp, 1.0, LS, (int)mp, st));
  // N = Lambda^T Lambda + reg I, its factor and X = factor^{-1}
  OHIP(mfma_gemm_lower_f64(true, false, m, m, m, 1.0, LS, (int)mp, LS, (int)mp, 0.0, N, m, st));
  OHIP(launch_reg_from_diag(true, N, m, m, rcond * rcond, regv, st));
  OHIP(launch_add_diag(true, N, m, m, regv, st));
  OHIP(cholesky_inverse_f64(N, m, m, X, work, info, st));
  // Y = X^T (X Lambda^T)
  OHIP(mfma_gemm_f64(false, true, m, m, m, 1.0, X, m, LS, (int)mp, 0.0, T1, m, st));
  OHIP(mfma_gemm_f64(true, false, m, m, m, 1.0, X, m, T1, m, 0.0, Y, m, st));
  // V = Y [-A^T diag(lambda) | -S]
  OHIP(gemm_tb_right_t(f64, m, n, m, 1.0, Y, m, tb->d_A, m, 0.0, V, (int)np, st));
  OHIP(launch_scale_cols(V, m, n, (int)np, tb->d_lambda, -1.0, st));
  OHIP(mfma_gemm_f64(false, false, m, p, m, -1.0, Y, m, LS + m, (int)mp, 0.0, V + n, (int)np, st));
  // U = [B; A] V + [0 | K; H]: gradient rows first, then the rows of u
  const int grad_rows = op->grad ? d * n : 0;
  if (op->grad) {
    OHIP(gemm_tb_left(f64, false, d * n, (int)np, m, 1.0, tb->d_B, m, V, (int)np, 0.0, U64, (int)ldu, st));
    OHIP(launch_add_block(U64 + n, d * n, p, (int)ldu, f64, tb->d_K, st));
  }
  double* Uu = U64 + (size_t)grad_rows * ldu;
  OHIP(gemm_tb_left(f64, false, n, (int)np, m, 1.0, tb->d_A, m, V, (int)np, 0.0, Uu, (int)ldu, st));
  OHIP(launch_add_block(Uu + n, n, p, (int)ldu, f64, tb->d_H, st));

  const size_t count = (size_t)op->rows * ldu;
  if (op->f32) {
    float* U32 = nullptr;
    OHIP(hipMalloc((void**)&U32, count * sizeof(float)));
    op->U = U32;
    op->bytes = count * sizeof(float);
    OHIP(launch_narrow(count, U64, U32, st));
  } else {
    // keep the FP64 buffer: take it out of the temporaries
    auto it = std::find(t.ptrs.begin(), t.ptrs.end(), static_cast<void*>(U64));
    t.ptrs.erase(it);
    op->U = U64;
    op->bytes = count * sizeof(double);
  }
  OHIP(hipEventRecord(e1, st));
  int hinfo = 0;
  OHIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
  OHIP(hipMemcpyAsync(&op->reg, regv, sizeof(double), hipMemcpyDeviceToHost, st));
  OHIP(hipStreamSynchronize(st));
  float ms = 0.0f;
  OHIP(hipEventElapsedTime(&ms, e0, e1));
  op->prep_ms = ms;
  if (hinfo != 0)
    return ofail(WOS_ENOTCONV, "normal matrix not positive definite at column %d", hinfo - 1);
  return WOS_OK;
}

}  // namespace

extern "C" {

wos_status wos_operator_create(wos_toolbox* tb, const wos_coeffs* co, const wos_operator_opts* opts, void* stream,
                               wos_operator** out) {
  if (!out) return ofail(WOS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tb || !co) return ofail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return ofail(WOS_EINVAL, "toolbox has not been built");
  if (tb->n != tb->m) return ofail(WOS_EINVAL, "operators need V = W (n == m)");
  if (co->kind != WOS_LINEAR) return ofail(WOS_EINVAL, "operators exist for LINEAR problems only");
  if (co->solver != WOS_SOLVER_TIKHONOV)
    return ofail(WOS_ENOTIMPL, "operators are prepared with the Tikhonov solver only");
  if (!(co->rcond >= 0.0)) return ofail(WOS_EINVAL, "rcond must be >= 0");
  const bool grad = opts && opts->want_grad;
  const int storage = opts ? opts->storage : WOS_F64;
  if (storage != WOS_F64 && storage != WOS_F32) return ofail(WOS_EINVAL, "storage must be WOS_F32 or WOS_F64");
  const size_t rows = (size_t)(grad ? tb->dim + 1 : 1) * tb->n;
  if (rows > (size_t)INT32_MAX || (size_t)tb->n + tb->p > (size_t)INT32_MAX / 2)
    return ofail(WOS_EINVAL, "operator too large");
  wos_operator* op = new (std::nothrow) wos_operator();
  if (!op) return ofail(WOS_ENOMEM, "out of host memory");
  op->tb = tb;
  op->n = tb->n;
  op->m = tb->m;
  op->p = tb->p;
  op->d = tb->dim;
  op->grad = grad;
  op->f32 = storage == WOS_F32;
  op->rows = (int)rows;
  op->cols = tb->n + tb->p;
  op->ld = (op->cols + 3) / 4 * 4;
  const wos_status s = prepare(op, tb, co, static_cast<hipStream_t>(stream));
  if (s != WOS_OK) {
    if (op->U) (void)hipFree(op->U);
    delete op;
    return s;
  }
  *out = op;
  return WOS_OK;
}

wos_status wos_operator_apply(const wos_operator* op, int32_t nrhs, const double* const* f, const double* const* g,
                              double* const* u, double* const* grad_u, void* stream) {
  if (!op || !f || !g || !u) return ofail(WOS_EINVAL, "NULL argument");
  if (nrhs < 1 || nrhs > 1024) return ofail(WOS_EINVAL, "nrhs must be in [1, 1024]");
  bool any_grad = false;
  for (int r = 0; r < nrhs; ++r) {
    if (!f[r] || !g[r] || !u[r]) return ofail(WOS_EINVAL, "NULL vector for right-hand side %d", r);
    if (grad_u && grad_u[r]) any_grad = true;
  }
  if (any_grad && !op->grad) return ofail(WOS_EINVAL, "gradient requested from an operator without want_grad");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int np = op->cols;
  const size_t ldu = (size_t)op->ld;
  const int grad_rows = any_grad ? op->d * op->n : 0;
  const size_t skip = (op->grad && !any_grad) ? (size_t)op->d * op->n : 0;  // start of the rows of u
  const void* U = op->f32 ? static_cast<const void*>(static_cast<const float*>(op->U) + skip * ldu)
                          : static_cast<const void*>(static_cast<const double*>(op->U) + skip * ldu);
  const int rows = op->n + grad_rows;
  for (int r0 = 0; r0 < nrhs; r0 += kOpBatch) {
    const int nb = std::min(kOpBatch, nrhs - r0);
    OpBatch bt;
    std::memset(&bt, 0, sizeof bt);
    for (int b = 0; b < nb; ++b) {
      bt.f[b] = f[r0 + b];
      bt.g[b] = g[r0 + b];
      bt.u[b] = u[r0 + b];
      bt.gu[b] = (any_grad && grad_u) ? grad_u[r0 + b] : nullptr;
    }
    OHIP(launch_op_apply(op->f32, U, rows, np, (int)ldu, op->n, grad_rows, nb, bt, st));
  }
  return WOS_OK;
}

wos_status wos_operator_get_info(const wos_operator* op, wos_operator_info* info) {
  if (!op || !info) return ofail(WOS_EINVAL, "NULL argument");
  info->n = op->n;
  info->p = op->p;
  info->dim = op->d;
  info->want_grad = op->grad ? 1 : 0;
  info->storage = op->f32 ? WOS_F32 : WOS_F64;
  info->reg = op->reg;
  info->device_bytes = op->bytes;
  info->prep_ms = op->prep_ms;
  return WOS_OK;
}

void wos_operator_free(wos_operator* op) {
  if (!op) return;
  if (op->U) (void)hipFree(op->U);
  delete op;
}

}  // extern "C"
