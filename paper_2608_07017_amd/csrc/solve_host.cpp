// Solve driver (C ABI wos_solve): reduction of a Dirichlet problem to the
// system for the unknown source and its truncated-SVD solution, plus the
// Newton and Picard outer loops.  Every arithmetic step runs in the kernels
// of solve.hip / apply.hip on the caller's stream; the host only reads back
// scalars (Jacobi convergence, the TSVD threshold, iteration norms).
//
// Linear problem (eq. linearPDE, paper's sign):
//   div(A grad u) + b . grad u - c u = f in D,  u = g on the boundary;
//   Lambda q = -(A^lambda)^T f - Sigma g  (eq. linear_q, with the transpose
//   reading of the A^lambda term), u = A q + H g, grad u_i = B_i q + K_i g.
// Generalised inverse: truncated SVD, singular values <= rcond * sigma_max
// dropped.  Lambda is symmetric when b = 0: its singular values are the
// absolute eigenvalues and the TSVD solution is sum_{|e_j| > tau}
// v_j v_j^T r / e_j.  Otherwise the eigenvectors of Lambda^T Lambda
// (eigenvalues sigma_j^2) give the right singular vectors and the TSVD
// solution is sum_{sigma_j > tau} v_j v_j^T Lambda^T r / sigma_j^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "toolbox.hpp"
#include "wos_kernels.hpp"
#include "wos_solve_kernels.hpp"

using namespace wos;

namespace wos {
void set_last_error(const char* msg);  // api.cpp
}

namespace {

wos_status sfail(wos_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  wos::set_last_error(buf);
  return s;
}

#define SHIP(call)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return sfail(e_ == hipErrorOutOfMemory ? WOS_ENOMEM : WOS_EDEVICE, "%s: %s (%s:%d)", #call, \
                   hipGetErrorString(e_), __FILE__, __LINE__);                              \
  } while (0)

template <typename P>
wos_status walloc(wos_toolbox* tb, P** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count * sizeof(P), 16));
  if (e != hipSuccess) return sfail(WOS_ENOMEM, "solve workspace: hipMalloc(%zu) failed", count * sizeof(P));
  tb->bytes += count * sizeof(P);
  return WOS_OK;
}

wos_status ensure_work(wos_toolbox* tb) {
  SolveWork& w = tb->sw;
  if (w.ready) return WOS_OK;
  const size_t n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  w.M = (int)(m + (m & 1));
  const size_t M = w.M;
  w.vlen = std::max(std::max(n, M), std::max(p, d * n));
  wos_status s;
  if ((s = walloc(tb, &w.R, (d + 1) * n * (m + p))) != WOS_OK) return s;
  if ((s = walloc(tb, &w.Lam, m * m)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.Sig, m * p)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.Lam0, m * m)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.Sig0, m * p)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.Hess, m * m)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.G, M * M)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.V, M * M)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.E, M)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.rot, M)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.pq, M)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.vec, 10 * w.vlen)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.Ac, n * d * d)) != WOS_OK) return s;
  if ((s = walloc(tb, &w.red, 2)) != WOS_OK) return s;
  w.ready = true;
  return WOS_OK;
}

// Lambda (m x m) and Sigma (m x p) for coefficients (Ac, bc, cc) into
// (Lam, Sig); Ac == NULL means A = I.
wos_status assemble(wos_toolbox* tb, const double* Ac, const double* bc, const double* cc, double* Lam,
                    double* Sig, hipStream_t st) {
  SolveWork& w = tb->sw;
  const int n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const bool f64 = tb->f64;
  SHIP(launch_weight_rows(f64, tb->d_A, tb->d_B, tb->d_H, tb->d_K, tb->d_lambda, Ac, bc, cc, n, m, p, d, w.R, st));
  // L = [B^(0); ...; B^(d-1); A]: d contiguous blocks at d_B, then d_A
  SHIP(launch_gemm_tn(f64, tb->d_B, tb->d_A, d + 1, n, m, w.R, m + p, m, Lam, m, 1.0, 0.0, st));
  SHIP(launch_gemm_tn(f64, tb->d_B, tb->d_A, d + 1, n, m, w.R + m, m + p, p, Sig, p, 1.0, 0.0, st));
  return WOS_OK;
}

struct TsvdResult {
  int rank = 0;
  int sweeps = 0;
  double smax = 0, smin_kept = 0;
};

// q (m) = TSVD(Mat) r (m), Mat m x m; `symmetric` selects the eigen route.
wos_status tsvd_solve(wos_toolbox* tb, const double* Mat, bool symmetric, const double* r, double rcond,
                      int max_sweeps, double* q, TsvdResult* res, hipStream_t st) {
  SolveWork& w = tb->sw;
  const int m = tb->m, M = w.M;
  double* rr = w.vec + 6 * w.vlen;  // padded right-hand side (M)
  double* z = w.vec + 7 * w.vlen;   // M
  SHIP(hipMemsetAsync(rr, 0, sizeof(double) * M, st));
  if (symmetric) {
    // G = (Mat + Mat^T) / 2 (symmetric up to rounding already), padded to M x M
    SHIP(launch_pad_copy(Mat, m, m, w.G, M, st));
    SHIP(launch_symmetrize(w.G, M, st));
    SHIP(hipMemcpyAsync(rr, r, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
  } else {
    // G = Mat^T Mat, rr = Mat^T r
    double* Gm = w.Hess;  // m x m scratch
    SHIP(launch_gram64(Mat, m, m, Gm, st));
    SHIP(launch_pad_copy(Gm, m, m, w.G, M, st));
    SHIP(launch_gemv_t(true, Mat, m, m, r, 1.0, 0.0, rr, st));
  }
  SHIP(launch_set_identity(w.V, M, st));
  // Jacobi sweeps until the off-diagonal mass is below (1e-15)^2 of the diagonal's
  double host2[2] = {0, 0};
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    SHIP(launch_offnorm(w.G, M, w.red, st));
    SHIP(hipMemcpyAsync(host2, w.red, sizeof host2, hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (!(host2[0] > 1e-30 * host2[1]) || host2[1] == 0.0) break;
    for (int rd = 0; rd < M - 1; ++rd) SHIP(launch_jacobi_round(w.G, w.V, M, rd, w.rot, w.pq, st));
  }
  SHIP(launch_diag(w.G, M, w.E, st));
  double emax = 0.0;
  SHIP(launch_absmax(M, w.E, w.red, st));
  SHIP(hipMemcpyAsync(&emax, w.red, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  // symmetric: sigma = |e|, keep sigma > rcond sigma_max; Gram: sigma^2 = e
  const double thr = symmetric ? rcond * emax : rcond * rcond * emax;
  unsigned long long rank = 0;
  SHIP(launch_count_above(M, w.E, thr, w.red + 1, st));
  SHIP(hipMemcpyAsync(&rank, w.red + 1, sizeof(rank), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  const double kmin = symmetric ? thr : std::sqrt(thr);  // the threshold on sigma (reported)
  // q = V diag(filter) V^T rr
  SHIP(launch_gemv_t(true, w.V, M, M, rr, 1.0, 0.0, z, st));
  SHIP(launch_tsvd_filter(M, w.E, thr, z, st));
  double* qM = w.vec + 9 * w.vlen;
  SHIP(launch_gemv_n(true, w.V, M, M, z, 1.0, 0.0, qM, st));
  SHIP(hipMemcpyAsync(q, qM, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
  if (res) {
    res->rank = (int)rank;
    res->sweeps = sweeps;
    res->smax = symmetric ? emax : std::sqrt(emax);
    res->smin_kept = kmin;
  }
  return WOS_OK;
}

// u = A q + H g, grad_u = B q + K g
wos_status reconstruct(wos_toolbox* tb, const double* q, const double* g, double* u, double* gu, hipStream_t st) {
  if (tb->f64) {
    SHIP(launch_apply_f64((const double*)tb->d_A, tb->n, tb->m, q, (const double*)tb->d_H, tb->p, g, u, 1, st));
    if (gu)
      SHIP(launch_apply_f64((const double*)tb->d_B, tb->n, tb->m, q, (const double*)tb->d_K, tb->p, g, gu,
                            tb->dim, st));
  } else {
    SHIP(launch_apply_f32((const float*)tb->d_A, tb->n, tb->m, q, (const float*)tb->d_H, tb->p, g, u, 1, st));
    if (gu)
      SHIP(launch_apply_f32((const float*)tb->d_B, tb->n, tb->m, q, (const float*)tb->d_K, tb->p, g, gu,
                            tb->dim, st));
  }
  return WOS_OK;
}

// rhs = -A^T (lambda o fp) - Sigma g   (fp: the paper's right-hand side)
wos_status linear_rhs(wos_toolbox* tb, const double* Sig, const double* fp, const double* g, double* rhs,
                      hipStream_t st) {
  SolveWork& w = tb->sw;
  double* lf = w.vec + 5 * w.vlen;
  SHIP(launch_pointwise(tb->n, tb->d_lambda, nullptr, fp, 0.0, 0.0, 0.0, 0.0, -1.0, lf, st));  // lam * f
  SHIP(launch_gemv_t(tb->f64, tb->d_A, tb->n, tb->m, lf, -1.0, 0.0, rhs, st));
  SHIP(launch_gemv_n(true, Sig, tb->m, tb->p, g, -1.0, 1.0, rhs, st));
  return WOS_OK;
}

// sum_i w_i x_i y_i on the device; the scalar is read back
wos_status dev_dot(wos_toolbox* tb, const double* dx, const double* dy, const double* dw, int n, double* out,
                   hipStream_t st) {
  SHIP(launch_dot(n, dx, dy, dw, tb->sw.red, st));
  SHIP(hipMemcpyAsync(out, tb->sw.red, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  return WOS_OK;
}

}  // namespace

extern "C" wos_status wos_solve(wos_toolbox* tb, const wos_coeffs* co, const double* f, const double* g,
                                double* u, double* grad_u, double* q_out, wos_solve_info* info, void* stream_) {
  if (!tb || !co || !f || !g || !u) return sfail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return sfail(WOS_EINVAL, "toolbox has not been built");
  hipStream_t st = static_cast<hipStream_t>(stream_);
  const double rcond = co->rcond > 0 ? co->rcond : 1e-3;
  if (!(rcond < 1.0)) return sfail(WOS_EINVAL, "rcond must be in (0, 1)");
  const int max_sweeps = co->max_sweeps > 0 ? co->max_sweeps : 40;
  wos_status s = ensure_work(tb);
  if (s != WOS_OK) return s;
  SolveWork& w = tb->sw;
  const int n = tb->n, m = tb->m, d = tb->dim;
  double* rhs = w.vec + 0 * w.vlen;
  double* q = w.vec + 1 * w.vlen;
  double* uu = w.vec + 2 * w.vlen;
  double* t1 = w.vec + 3 * w.vlen;
  double* t2 = w.vec + 4 * w.vlen;
  wos_solve_info inf{};
  TsvdResult tr;

  if (co->kind == WOS_LINEAR) {
    if ((s = assemble(tb, co->A, co->b, co->c, w.Lam, w.Sig, st)) != WOS_OK) return s;
    if ((s = linear_rhs(tb, w.Sig, f, g, rhs, st)) != WOS_OK) return s;
    if ((s = tsvd_solve(tb, w.Lam, co->b == nullptr, rhs, rcond, max_sweeps, q, &tr, st)) != WOS_OK) return s;
    inf.iters = 1;
  } else if (co->kind == WOS_SEMILINEAR_CUBIC) {
    // F = |p|^2/2 + kappa u^4/4 - f u; grad J = A^T(lam (kappa u^3 - f)) + Lam0 h + Sig0 g
    const double kappa = co->kappa;
    const double tol = co->tol > 0 ? co->tol : 1e-8;
    const int max_iter = co->max_iter > 0 ? co->max_iter : 50;
    if ((s = assemble(tb, nullptr, nullptr, nullptr, w.Lam0, w.Sig0, st)) != WOS_OK) return s;
    // h0: the problem without the cubic term, rhs = A^T (lam f) - Sig0 g
    SHIP(launch_pointwise(n, tb->d_lambda, nullptr, f, 0.0, 0.0, 0.0, 0.0, -1.0, t1, st));
    SHIP(launch_gemv_t(tb->f64, tb->d_A, n, m, t1, 1.0, 0.0, rhs, st));
    SHIP(launch_gemv_n(true, w.Sig0, m, tb->p, g, -1.0, 1.0, rhs, st));
    if ((s = tsvd_solve(tb, w.Lam0, true, rhs, rcond, max_sweeps, q, &tr, st)) != WOS_OK) return s;
    double gn0 = -1.0, gn = 0.0;
    int it = 0;
    for (it = 0; it <= max_iter; ++it) {
      if ((s = reconstruct(tb, q, g, uu, nullptr, st)) != WOS_OK) return s;
      // grad = A^T (lam (kappa u^3 - f)) + Lam0 h + Sig0 g
      SHIP(launch_pointwise(n, tb->d_lambda, uu, f, 0.0, 0.0, 0.0, kappa, 1.0, t1, st));
      SHIP(launch_gemv_t(tb->f64, tb->d_A, n, m, t1, 1.0, 0.0, rhs, st));
      SHIP(launch_gemv_n(true, w.Lam0, m, m, q, 1.0, 1.0, rhs, st));
      SHIP(launch_gemv_n(true, w.Sig0, m, tb->p, g, 1.0, 1.0, rhs, st));
      if ((s = dev_dot(tb, rhs, rhs, nullptr, m, &gn, st)) != WOS_OK) return s;
      gn = std::sqrt(gn);
      if (gn0 < 0) gn0 = gn;
      if (gn <= tol * gn0 || it == max_iter) break;
      // Hessian = Lam0 + A^T diag(3 kappa lam u^2) A
      SHIP(hipMemcpyAsync(w.Hess, w.Lam0, sizeof(double) * m * m, hipMemcpyDeviceToDevice, st));
      SHIP(launch_pointwise(n, tb->d_lambda, uu, nullptr, 0.0, 0.0, 3.0 * kappa, 0.0, 0.0, t2, st));
      SHIP(launch_gram(tb->f64, tb->d_A, n, m, t2, w.Hess, st));
      if ((s = tsvd_solve(tb, w.Hess, true, rhs, rcond, max_sweeps, t1, &tr, st)) != WOS_OK) return s;
      SHIP(launch_axpby(m, 1.0, q, -1.0, t1, q, st));
    }
    inf.iters = it;
    inf.grad_norm = gn;
    inf.grad_norm0 = gn0;
  } else if (co->kind == WOS_QUASILINEAR) {
    // -div((1 + u^2) grad u) = f: A(x_i) = (1 + u_i^2) I, b = c = 0, paper f = -f
    const double tol = co->tol > 0 ? co->tol : 1e-10;
    const int max_iter = co->max_iter > 0 ? co->max_iter : 100;
    SHIP(hipMemsetAsync(uu, 0, sizeof(double) * n, st));
    double* fp = t2;  // the paper's right-hand side, -f
    SHIP(launch_axpby(n, -1.0, f, 0.0, nullptr, fp, st));
    int it = 0;
    double du = 0, nu = 0;
    for (it = 1; it <= max_iter; ++it) {
      SHIP(launch_picard_coef(n, d, uu, w.Ac, st));  // A(x_i) = (1 + u_i^2) I
      if ((s = assemble(tb, w.Ac, nullptr, nullptr, w.Lam, w.Sig, st)) != WOS_OK) return s;
      if ((s = linear_rhs(tb, w.Sig, fp, g, rhs, st)) != WOS_OK) return s;
      if ((s = tsvd_solve(tb, w.Lam, true, rhs, rcond, max_sweeps, q, &tr, st)) != WOS_OK) return s;
      if ((s = reconstruct(tb, q, g, t1, nullptr, st)) != WOS_OK) return s;
      // du = |u_new - u|_lam, nu = |u_new|_lam
      SHIP(launch_axpby(n, 1.0, t1, -1.0, uu, rhs, st));
      if ((s = dev_dot(tb, rhs, rhs, tb->d_lambda, n, &du, st)) != WOS_OK) return s;
      if ((s = dev_dot(tb, t1, t1, tb->d_lambda, n, &nu, st)) != WOS_OK) return s;
      SHIP(hipMemcpyAsync(uu, t1, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      if (std::sqrt(du) <= tol * std::sqrt(nu)) break;
    }
    inf.iters = std::min(it, max_iter);
    inf.update_norm = std::sqrt(du);
  } else {
    return sfail(WOS_EINVAL, "unknown problem kind %d", co->kind);
  }
  if ((s = reconstruct(tb, q, g, u, grad_u, st)) != WOS_OK) return s;
  if (q_out) SHIP(hipMemcpyAsync(q_out, q, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
  SHIP(hipStreamSynchronize(st));
  inf.rank = tr.rank;
  inf.sweeps = tr.sweeps;
  inf.sigma_max = tr.smax;
  inf.sigma_threshold = tr.smin_kept;
  if (info) *info = inf;
  return WOS_OK;
}
