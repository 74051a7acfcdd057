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
#include <chrono>
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
wos_status walloc(SolveWork& w, P** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count * sizeof(P), 16));
  if (e != hipSuccess) return sfail(WOS_ENOMEM, "solve workspace: hipMalloc(%zu) failed", count * sizeof(P));
  w.bytes += count * sizeof(P);
  return WOS_OK;
}

// A workspace is sized for one toolbox shape; one that was sized for another
// shape (a server slot that served another toolbox) is emptied first, and
// every buffer is then allocated again on demand.
void fit_work(wos_toolbox* tb, SolveWork& w) {
  if (w.bytes > 0 && (w.n != tb->n || w.m != tb->m || w.p != tb->p || w.d != tb->dim)) free_work(w);
  w.n = tb->n;
  w.m = tb->m;
  w.p = tb->p;
  w.d = tb->dim;
}

// The partial-sum buffer of the transposed products for up to nv vectors
// of max(m, p) columns.  Grown only before a request's first launch that
// needs more (the stream is synchronised first, as queued work may still
// read the old buffer).
wos_status ensure_part(wos_toolbox* tb, SolveWork& w, int nv, hipStream_t st) {
  const size_t need = gemv_part_elems(std::max(tb->m, tb->p), nv);
  if (w.part_cap >= need) return WOS_OK;
  if (w.fixed) return sfail(WOS_ENOMEM, "the fixed workspace holds no room for %zu partial sums", need);
  if (w.part) {
    SHIP(hipStreamSynchronize(st));
    (void)hipFree(w.part);
    w.bytes -= w.part_cap * sizeof(double);
    w.part = nullptr;
    w.part_cap = 0;
  }
  wos_status s = walloc(w, &w.part, need);
  if (s != WOS_OK) return s;
  w.part_cap = need;
  return WOS_OK;
}

wos_status ensure_work(wos_toolbox* tb, SolveWork& w) {
  fit_work(tb, w);
  if (w.ready) return WOS_OK;
  const size_t n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  w.M = (int)(m + (m & 1));
  const size_t M = w.M;
  w.vlen = std::max(std::max(n, M), std::max(p, d * n));
  wos_status s;
  if ((s = walloc(w, &w.R, (d + 1) * n * (m + p))) != WOS_OK) return s;
  if ((s = walloc(w, &w.Lam, m * m)) != WOS_OK) return s;
  if ((s = walloc(w, &w.Sig, m * p)) != WOS_OK) return s;
  if ((s = walloc(w, &w.Lam0, m * m)) != WOS_OK) return s;
  if ((s = walloc(w, &w.Sig0, m * p)) != WOS_OK) return s;
  if ((s = walloc(w, &w.Hess, m * m)) != WOS_OK) return s;
  if ((s = walloc(w, &w.G, M * M)) != WOS_OK) return s;
  if ((s = walloc(w, &w.V, M * M)) != WOS_OK) return s;
  if ((s = walloc(w, &w.E, M)) != WOS_OK) return s;
  if ((s = walloc(w, &w.rot, M)) != WOS_OK) return s;
  if ((s = walloc(w, &w.pq, M)) != WOS_OK) return s;
  if ((s = walloc(w, &w.vec, 10 * w.vlen)) != WOS_OK) return s;
  if ((s = walloc(w, &w.Ac, n * d * d)) != WOS_OK) return s;
  if ((s = walloc(w, &w.red, 2)) != WOS_OK) return s;
  w.ready = true;
  return WOS_OK;
}

// Lambda (m x m) and Sigma (m x p) for coefficients (Ac, bc, cc) into
// (Lam, Sig); Ac == NULL means A = I.
wos_status assemble(wos_toolbox* tb, SolveWork& w, const double* Ac, const double* bc, const double* cc,
                    double* Lam, double* Sig, hipStream_t st) {
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

// Eigen-decomposition of the symmetric M x M matrix in w.G by cyclic Jacobi
// sweeps until the off-diagonal mass is below (1e-15)^2 of the diagonal's:
// eigenvalues to w.E, eigenvectors to the columns of w.V.
wos_status jacobi_eig(SolveWork& w, int max_sweeps, int* sweeps_out, hipStream_t st) {
  const int M = w.M;
  SHIP(launch_set_identity(w.V, M, st));
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
  *sweeps_out = sweeps;
  return WOS_OK;
}

// q (m) = TSVD(Mat) r (m), Mat m x m; `symmetric` selects the eigen route.
wos_status tsvd_solve(wos_toolbox* tb, SolveWork& w, const double* Mat, bool symmetric, const double* r,
                      double rcond, int max_sweeps, double* q, TsvdResult* res, hipStream_t st) {
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
  int sweeps = 0;
  wos_status s;
  if ((s = jacobi_eig(w, max_sweeps, &sweeps, st)) != WOS_OK) return s;
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
wos_status linear_rhs(wos_toolbox* tb, SolveWork& w, const double* Sig, const double* fp, const double* g,
                      double* rhs, hipStream_t st) {
  double* lf = w.vec + 5 * w.vlen;
  SHIP(launch_pointwise(tb->n, tb->d_lambda, nullptr, fp, 0.0, 0.0, 0.0, 0.0, -1.0, lf, st));  // lam * f
  SHIP(launch_gemv_t(tb->f64, tb->d_A, tb->n, tb->m, lf, -1.0, 0.0, rhs, st));
  SHIP(launch_gemv_n(true, Sig, tb->m, tb->p, g, -1.0, 1.0, rhs, st));
  return WOS_OK;
}

// sum_i w_i x_i y_i on the device; the scalar is read back
wos_status dev_dot(SolveWork& w, const double* dx, const double* dy, const double* dw, int n, double* out,
                   hipStream_t st) {
  SHIP(launch_dot(n, dx, dy, dw, w.red, st));
  SHIP(hipMemcpyAsync(out, w.red, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  return WOS_OK;
}


// ------------------------------------------------------------ Tikhonov
// Regularised generalised inverse: q minimises |Lambda q - rhs|^2 + reg |q|^2
// with reg = rcond^2 max_j (Lambda^T Lambda)_jj, i.e. q solves the normal
// equations (Lambda^T Lambda + reg I) q = Lambda^T rhs.
//
// FP64: Lambda and the normal matrix are formed by FP64 MFMA GEMMs and
// factored by Cholesky in FP64.  MIXED (FP32 toolbox): both are formed and
// factored in FP32 on the matrix cores; the solution is then refined with
// residuals of the exact system evaluated matrix-free in FP64
// (Lambda = L^T W L applied as GEMVs over the toolbox rows with FP64
// accumulation), until |r| <= refine_tol |Lambda^T rhs|.  If the FP32
// factorisation meets a non-positive pivot the request is solved in FP64.
wos_status ensure_tik(wos_toolbox* tb, SolveWork& w, bool mixed, bool bf = false) {
  const size_t n = tb->n, m = tb->m, d = tb->dim;
  wos_status s;
  if (bf && !w.RT) {
    if ((s = walloc(w, &w.RT, (d + 1) * n * m)) != WOS_OK) return s;
    if ((s = walloc(w, &w.cg, 3 * m)) != WOS_OK) return s;
  }
  if (mixed && !w.colp) {
    if ((s = walloc(w, &w.colp, (size_t)kColsqChunks * m)) != WOS_OK) return s;
    if ((s = walloc(w, &w.cn, 2 * m)) != WOS_OK) return s;
  }
  if (!w.blk) {
    if ((s = walloc(w, &w.P64, chol_work_elems(m))) != WOS_OK) return s;
    if ((s = walloc(w, &w.blk, 2 * (d + 1) * std::max<size_t>(n, 1))) != WOS_OK) return s;
    if ((s = walloc(w, &w.regv, 2)) != WOS_OK) return s;
    if ((s = walloc(w, &w.info, 2)) != WOS_OK) return s;
  }
  if (mixed && !bf && !w.R32) {
    if ((s = walloc(w, &w.R32, (d + 1) * n * m)) != WOS_OK) return s;
  }
  if (mixed && !w.Lam32) {
    if ((s = walloc(w, &w.Lam32, m * m)) != WOS_OK) return s;
    if ((s = walloc(w, &w.N32, m * m)) != WOS_OK) return s;
    if ((s = walloc(w, &w.v32, m)) != WOS_OK) return s;
    if ((s = walloc(w, &w.L0_32, m * m)) != WOS_OK) return s;
    if ((s = walloc(w, &w.P32, chol_work_elems(m))) != WOS_OK) return s;
  }
  return WOS_OK;
}

// y ((d+1) n) = L x, L = [B; A]
wos_status apply_L(wos_toolbox* tb, const double* x, double* y, hipStream_t st) {
  const int n = tb->n, m = tb->m, d = tb->dim;
  SHIP(launch_gemv_n_ld(tb->f64, tb->d_B, d * n, m, m, x, 1.0, 0.0, y, st));
  SHIP(launch_gemv_n_ld(tb->f64, tb->d_A, n, m, m, x, 1.0, 0.0, y + (size_t)d * n, st));
  return WOS_OK;
}
// x (m) = alpha L^T y + beta x
wos_status apply_Lt(wos_toolbox* tb, SolveWork& w, const double* y, double alpha, double beta, double* x,
                    hipStream_t st) {
  const int n = tb->n, m = tb->m, d = tb->dim;
  SHIP(launch_gemv_t_ld(tb->f64, tb->d_B, d * n, m, m, y, alpha, beta, x, w.part, st));
  SHIP(launch_gemv_t_ld(tb->f64, tb->d_A, n, m, m, y + (size_t)d * n, alpha, 1.0, x, w.part, st));
  return WOS_OK;
}
// out = Lambda x (trans = false) or Lambda^T x, Lambda = L^T W L
wos_status apply_Lambda(wos_toolbox* tb, SolveWork& w, const wos_coeffs* co, const double* x, bool trans,
                        double* out, hipStream_t st) {
  const int n = tb->n, d = tb->dim;
  double* y1 = w.blk;
  double* y2 = w.blk + (size_t)(d + 1) * n;
  wos_status s;
  if ((s = apply_L(tb, x, y1, st)) != WOS_OK) return s;
  SHIP(launch_apply_w(n, d, tb->d_lambda, co->A, co->b, co->c, y1, trans, nullptr, y2, st));
  return apply_Lt(tb, w, y2, 1.0, 0.0, out, st);
}

// The regularisation parameter of the mixed route, rcond^2 max_j
// |Lambda e_j|^2, equal to the FP64 route's (read there from the diagonal of
// its FP64 normal matrix), so that FP64 refinement converges to the same
// regularised system: the column norms of the FP32 Lambda (accumulated in
// FP64) pick the candidates within 1e-5 of the largest (at most 16, largest
// first), and those columns are formed again in FP64, matrix-free.  e and col
// are m-vectors of work.
wos_status mixed_tikhonov_reg(wos_toolbox* tb, SolveWork& w, const wos_coeffs* co, double rcond, double* e,
                              double* col, hipStream_t st) {
  const int m = tb->m;
  SHIP(launch_colsq(false, w.Lam32, m, m, m, nullptr, 1, false, w.colp, w.cn, st));
  std::vector<double> cn(m);
  SHIP(hipMemcpyAsync(cn.data(), w.cn, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  const double mx = *std::max_element(cn.begin(), cn.end());
  std::vector<std::pair<double, int>> cand;
  for (int j = 0; j < m; ++j)
    if (cn[j] >= (1.0 - 1e-5) * mx) cand.push_back({cn[j], j});
  std::sort(cand.begin(), cand.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  });
  if (cand.size() > 16) cand.resize(16);
  double best = 0.0;
  wos_status s;
  for (const auto& c : cand) {
    SHIP(launch_unit_vector(m, c.second, e, st));
    if ((s = apply_Lambda(tb, w, co, e, false, col, st)) != WOS_OK) return s;
    double nn = 0.0;
    if ((s = dev_dot(w, col, col, nullptr, m, &nn, st)) != WOS_OK) return s;
    best = std::max(best, nn);
  }
  SHIP(launch_set_scalar(w.regv, rcond * rcond * best, st));
  return WOS_OK;
}

wos_status tikhonov_linear(wos_toolbox* tb, SolveWork& w, const wos_coeffs* co, double rcond, const double* f,
                           const double* g, double* q, wos_solve_info* inf, hipStream_t st) {
  const int n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const int K = d * n;
  const bool bf = co->precision == WOS_SOLVE_MIXED_BF16;
  bool mixed = (co->precision == WOS_SOLVE_MIXED && !tb->f64) || bf;
  wos_status s;
  if ((s = ensure_tik(tb, w, mixed, bf)) != WOS_OK) return s;
  if (bf && (s = toolbox_bf16_current(tb, st)) != WOS_OK) return s;
  double* rhs = w.vec + 5 * w.vlen;
  double* c = w.vec + 6 * w.vlen;
  double* r = w.vec + 7 * w.vlen;
  double* t = w.vec + 8 * w.vlen;
  double* y1 = w.blk;
  double* y2 = w.blk + (size_t)(d + 1) * n;

  // right-hand side and c = Lambda^T rhs, matrix-free in FP64
  SHIP(launch_gemv_n_ld(tb->f64, tb->d_K, d * n, p, p, g, 1.0, 0.0, y1, st));
  SHIP(launch_gemv_n_ld(tb->f64, tb->d_H, n, p, p, g, 1.0, 0.0, y1 + (size_t)d * n, st));
  SHIP(launch_apply_w(n, d, tb->d_lambda, co->A, co->b, co->c, y1, false, f, y2, st));
  if ((s = apply_Lt(tb, w, y2, -1.0, 0.0, rhs, st)) != WOS_OK) return s;
  if ((s = apply_Lambda(tb, w, co, rhs, true, c, st)) != WOS_OK) return s;
  SHIP(hipMemsetAsync(w.info, 0, 2 * sizeof(int), st));

  if (mixed) {
    // Lambda (FP32) = L^T R, R = W L; N = Lambda^T Lambda + reg I; Cholesky
    if (bf) {
      // from the BF16 shadows on the matrix cores (FP32 accumulation):
      // Lambda[i][j] = sum_k S_V[i][k] RT[j][k]
      const size_t KB = (size_t)(d + 1) * n;
      SHIP(launch_weight_t_bf16(tb->d_SV, n, m, d, tb->d_lambda, co->A, co->b, co->c, w.RT, st));
      SHIP(gemm_nt_bf16(m, m, (int)KB, 1.0f, tb->d_SV, KB, w.RT, KB, 0.0f, w.Lam32, m, st));
    } else {
      SHIP(launch_weight_rows_any(false, true, tb->d_A, tb->d_B, tb->d_H, tb->d_K, tb->d_lambda, co->A, co->b,
                                  co->c, n, m, p, d, m, w.R32, st));
      SHIP(mfma_gemm_f32(true, false, m, m, K, 1.0f, (const float*)tb->d_B, m, w.R32, m, 0.0f, w.Lam32, m, st));
      SHIP(mfma_gemm_f32(true, false, m, m, n, 1.0f, (const float*)tb->d_A, m, w.R32 + (size_t)K * m, m, 1.0f,
                         w.Lam32, m, st));
    }
    SHIP(mfma_gemm_lower_f32(true, false, m, m, m, 1.0f, w.Lam32, m, w.Lam32, m, 0.0f, w.N32, m, st));
    if ((s = mixed_tikhonov_reg(tb, w, co, rcond, r, t, st)) != WOS_OK) return s;
    SHIP(launch_add_diag(false, w.N32, m, m, w.regv, st));
    SHIP(cholesky_inverse_f32(w.N32, m, m, w.Lam32, w.P32, w.info, st));  // X = L^{-1} over Lambda's storage
    int hinfo = 0;
    SHIP(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (hinfo != 0) {
      mixed = false;  // fall back to FP64 for this request
      inf->fallback = 1;
      SHIP(hipMemsetAsync(w.info, 0, 2 * sizeof(int), st));
    }
  }
  if (mixed && bf) {
    // Preconditioned conjugate gradients on (Lambda^T Lambda + reg I) q = c,
    // products in FP64 matrix-free, preconditioner X^T X from the FP32
    // factor of the BF16-assembled normal matrix (symmetric positive
    // definite, so the iteration converges where plain refinement with a
    // preconditioner this rough would not)
    const double tol = co->refine_tol > 0 ? co->refine_tol : 1e-10;
    const int maxit = co->max_refine > 0 ? co->max_refine : 50;
    double* z = w.cg;
    double* pv = w.cg + m;
    double* Ap = w.cg + 2 * (size_t)m;
    double cn = 0.0, rn = 0.0, rz = 0.0, pAp = 0.0;
    auto precond = [&](const double* x, double* y) -> wos_status {
      SHIP(launch_gemv_n_ld(false, w.Lam32, m, m, m, x, 1.0, 0.0, t, st));
      SHIP(launch_gemv_t_ld(false, w.Lam32, m, m, m, t, 1.0, 0.0, y, w.part, st));
      return WOS_OK;
    };
    if ((s = dev_dot(w, c, c, nullptr, m, &cn, st)) != WOS_OK) return s;
    cn = std::sqrt(cn);
    SHIP(hipMemsetAsync(q, 0, sizeof(double) * m, st));
    SHIP(hipMemcpyAsync(r, c, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    if ((s = precond(r, z)) != WOS_OK) return s;
    SHIP(hipMemcpyAsync(pv, z, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    if ((s = dev_dot(w, r, z, nullptr, m, &rz, st)) != WOS_OK) return s;
    rn = cn;
    int it = 0;
    for (it = 1; it <= maxit && rn > tol * cn; ++it) {
      double* y = w.vec + 9 * w.vlen;
      if ((s = apply_Lambda(tb, w, co, pv, false, y, st)) != WOS_OK) return s;
      if ((s = apply_Lambda(tb, w, co, y, true, Ap, st)) != WOS_OK) return s;
      SHIP(launch_axpy_reg(m, Ap, w.regv, 1.0, pv, Ap, st));
      if ((s = dev_dot(w, pv, Ap, nullptr, m, &pAp, st)) != WOS_OK) return s;
      if (!(pAp > 0.0)) break;
      const double alpha = rz / pAp;
      SHIP(launch_axpby(m, 1.0, q, alpha, pv, q, st));
      SHIP(launch_axpby(m, 1.0, r, -alpha, Ap, r, st));
      if ((s = dev_dot(w, r, r, nullptr, m, &rn, st)) != WOS_OK) return s;
      rn = std::sqrt(rn);
      if (rn <= tol * cn) break;
      if ((s = precond(r, z)) != WOS_OK) return s;
      double rz1 = 0.0;
      if ((s = dev_dot(w, r, z, nullptr, m, &rz1, st)) != WOS_OK) return s;
      SHIP(launch_axpby(m, 1.0, z, rz1 / rz, pv, pv, st));
      rz = rz1;
    }
    inf->refine_iters = std::min(it, maxit);
    inf->refine_residual = cn > 0 ? rn / cn : 0.0;
    if (!(rn <= tol * cn)) inf->refine_converged = 0;
  } else if (mixed) {
    const double tol = co->refine_tol > 0 ? co->refine_tol : 1e-10;
    const int maxit = co->max_refine > 0 ? co->max_refine : 10;
    double cn = 0.0, rn = 0.0;
    if ((s = dev_dot(w, c, c, nullptr, m, &cn, st)) != WOS_OK) return s;
    cn = std::sqrt(cn);
    SHIP(hipMemsetAsync(q, 0, sizeof(double) * m, st));
    SHIP(hipMemcpyAsync(r, c, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    int it = 0;
    for (it = 1; it <= maxit; ++it) {
      // q += X^T (X r): the FP32 factor's inverse applied with FP64 accumulation
      SHIP(launch_gemv_n_ld(false, w.Lam32, m, m, m, r, 1.0, 0.0, t, st));
      SHIP(launch_gemv_t_ld(false, w.Lam32, m, m, m, t, 1.0, 1.0, q, w.part, st));
      // r = c - Lambda^T Lambda q - reg q   (FP64)
      if ((s = apply_Lambda(tb, w, co, q, false, t, st)) != WOS_OK) return s;
      if ((s = apply_Lambda(tb, w, co, t, true, r, st)) != WOS_OK) return s;
      SHIP(launch_axpy_reg(m, c, nullptr, -1.0, r, r, st));
      SHIP(launch_axpy_reg(m, r, w.regv, -1.0, q, r, st));
      if ((s = dev_dot(w, r, r, nullptr, m, &rn, st)) != WOS_OK) return s;
      rn = std::sqrt(rn);
      if (rn <= tol * cn) break;
    }
    inf->refine_iters = std::min(it, maxit);
    inf->refine_residual = cn > 0 ? rn / cn : 0.0;
    if (!(rn <= tol * cn)) inf->refine_converged = 0;
  } else {
    // FP64: Lambda = L^T R (R = W L in FP64), N = Lambda^T Lambda + reg I
    SHIP(launch_weight_rows_any(tb->f64, false, tb->d_A, tb->d_B, tb->d_H, tb->d_K, tb->d_lambda, co->A, co->b,
                                co->c, n, m, p, d, m, w.R, st));
    if (tb->f64) {
      SHIP(mfma_gemm_f64(true, false, m, m, K, 1.0, (const double*)tb->d_B, m, w.R, m, 0.0, w.Lam, m, st));
      SHIP(mfma_gemm_f64(true, false, m, m, n, 1.0, (const double*)tb->d_A, m, w.R + (size_t)K * m, m, 1.0, w.Lam,
                         m, st));
    } else {
      SHIP(mfma_gemm_f64_a32(true, false, m, m, K, 1.0, (const float*)tb->d_B, m, w.R, m, 0.0, w.Lam, m, st));
      SHIP(mfma_gemm_f64_a32(true, false, m, m, n, 1.0, (const float*)tb->d_A, m, w.R + (size_t)K * m, m, 1.0,
                             w.Lam, m, st));
    }
    SHIP(mfma_gemm_lower_f64(true, false, m, m, m, 1.0, w.Lam, m, w.Lam, m, 0.0, w.Hess, m, st));
    SHIP(launch_reg_from_diag(true, w.Hess, m, m, rcond * rcond, w.regv, st));
    SHIP(launch_add_diag(true, w.Hess, m, m, w.regv, st));
    SHIP(cholesky_inverse_f64(w.Hess, m, m, w.Lam, w.P64, w.info, st));  // X = L^{-1} over Lambda's storage
    SHIP(launch_gemv_n_ld(true, w.Lam, m, m, m, c, 1.0, 0.0, t, st));
    SHIP(launch_gemv_t_ld(true, w.Lam, m, m, m, t, 1.0, 0.0, q, w.part, st));
    int hinfo = 0;
    SHIP(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (hinfo != 0) return sfail(WOS_ENOTCONV, "normal matrix not positive definite at column %d", hinfo - 1);
  }
  return WOS_OK;
}

// Regularised solve of a symmetric positive semidefinite system H x = rhs:
// x = (H + reg I)^{-1} rhs with reg = rcond max_j H_jj (the analogue, for a
// symmetric matrix, of dropping the eigenvalues below rcond times the
// largest).  H is formed by the caller in FP64 (w.Hess) or, mixed, in FP32
// (w.N32); `applyH(x, out)` applies the exact H in FP64 (matrix-free) for
// the refinement of the mixed route.
template <typename F>
wos_status sym_reg_solve(wos_toolbox* tb, SolveWork& w, bool mixed, double rcond, double tol, int maxit,
                         const double* rhs, double* x, F applyH, const double* diag, wos_solve_info* inf,
                         hipStream_t st) {
  const int m = tb->m;
  double* r = w.vec + 6 * w.vlen;
  double* t = w.vec + 7 * w.vlen;
  SHIP(hipMemsetAsync(w.info, 0, 2 * sizeof(int), st));
  int hinfo = 0;
  if (mixed) {
    // reg from the exact FP64 diagonal of H (as the FP64 route reads it)
    SHIP(launch_reg_from_vec(diag, m, rcond, w.regv, st));
    SHIP(launch_add_diag(false, w.N32, m, m, w.regv, st));
    SHIP(cholesky_inverse_f32(w.N32, m, m, w.Lam32, w.P32, w.info, st));
    SHIP(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (hinfo != 0) return sfail(WOS_ENOTCONV, "FP32 factorisation failed at column %d", hinfo - 1);
    double rn0 = 0.0, rn = 0.0;
    wos_status s;
    if ((s = dev_dot(w, rhs, rhs, nullptr, m, &rn0, st)) != WOS_OK) return s;
    rn0 = std::sqrt(rn0);
    SHIP(hipMemsetAsync(x, 0, sizeof(double) * m, st));
    SHIP(hipMemcpyAsync(r, rhs, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    int it = 0;
    for (it = 1; it <= maxit; ++it) {
      SHIP(launch_gemv_n_ld(false, w.Lam32, m, m, m, r, 1.0, 0.0, t, st));
      SHIP(launch_gemv_t_ld(false, w.Lam32, m, m, m, t, 1.0, 1.0, x, w.part, st));
      if ((s = applyH(x, t)) != WOS_OK) return s;
      SHIP(launch_axpy_reg(m, rhs, nullptr, -1.0, t, r, st));
      SHIP(launch_axpy_reg(m, r, w.regv, -1.0, x, r, st));
      if ((s = dev_dot(w, r, r, nullptr, m, &rn, st)) != WOS_OK) return s;
      rn = std::sqrt(rn);
      if (rn <= tol * rn0) break;
    }
    inf->refine_iters = std::min(it, maxit);
    inf->refine_residual = rn0 > 0 ? rn / rn0 : 0.0;
    if (!(rn <= tol * rn0)) inf->refine_converged = 0;
  } else {
    SHIP(launch_reg_from_diag(true, w.Hess, m, m, rcond, w.regv, st));
    SHIP(launch_add_diag(true, w.Hess, m, m, w.regv, st));
    SHIP(cholesky_inverse_f64(w.Hess, m, m, w.Lam, w.P64, w.info, st));
    SHIP(launch_gemv_n_ld(true, w.Lam, m, m, m, rhs, 1.0, 0.0, t, st));
    SHIP(launch_gemv_t_ld(true, w.Lam, m, m, m, t, 1.0, 0.0, x, w.part, st));
    SHIP(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (hinfo != 0) return sfail(WOS_ENOTCONV, "matrix not positive definite at column %d", hinfo - 1);
  }
  return WOS_OK;
}

// Newton for -Lap u + kappa u^3 = f with regularised steps (solver
// TIKHONOV): the Hessian Lambda_0 + A^T diag(3 kappa lambda u^2) A is formed
// explicitly (FP64, or FP32 in the mixed route) on the matrix cores, the
// gradient and the refinement residuals are evaluated matrix-free in FP64.
wos_status newton_tikhonov(wos_toolbox* tb, SolveWork& w, const wos_coeffs* co, double rcond, const double* f,
                           const double* g, double* q, wos_solve_info* inf, hipStream_t st) {
  const int n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const int K = d * n;
  const bool mixed = co->precision == WOS_SOLVE_MIXED && !tb->f64;
  const double kappa = co->kappa;
  const double tol = co->tol > 0 ? co->tol : 1e-8;
  const int max_iter = co->max_iter > 0 ? co->max_iter : 50;
  const double rtol = co->refine_tol > 0 ? co->refine_tol : 1e-10;
  const int rmax = co->max_refine > 0 ? co->max_refine : 10;
  wos_status s;
  if ((s = ensure_tik(tb, w, mixed)) != WOS_OK) return s;
  double* grad = w.vec + 0 * w.vlen;
  double* uu = w.vec + 2 * w.vlen;
  double* t1 = w.vec + 3 * w.vlen;
  double* wts = w.vec + 4 * w.vlen;
  double* tmp = w.vec + 5 * w.vlen;
  double* sig0g = w.vec + 8 * w.vlen;
  double* dlt = w.vec + 9 * w.vlen;
  double* y1 = w.blk;
  double* y2 = w.blk + (size_t)(d + 1) * n;
  wos_coeffs co0{};  // A = I, b = c = 0: Lambda_0 and Sigma_0
  // Lambda_0 explicit: L^T W0 L (the A rows carry no weight); only its
  // lower triangle, as only the Cholesky of the Hessian reads it
  SHIP(launch_weight_rows_any(tb->f64, mixed, tb->d_A, tb->d_B, tb->d_H, tb->d_K, tb->d_lambda, nullptr, nullptr,
                              nullptr, n, m, p, d, m, mixed ? (void*)w.R32 : (void*)w.R, st));
  if (mixed)
    SHIP(mfma_gemm_lower_f32(true, false, m, m, K, 1.0f, (const float*)tb->d_B, m, w.R32, m, 0.0f, w.L0_32, m, st));
  else if (tb->f64)
    SHIP(mfma_gemm_lower_f64(true, false, m, m, K, 1.0, (const double*)tb->d_B, m, w.R, m, 0.0, w.Lam0, m, st));
  else
    SHIP(mfma_gemm_lower_f64_a32(true, false, m, m, K, 1.0, (const float*)tb->d_B, m, w.R, m, 0.0, w.Lam0, m,
                                 st));
  auto apply_lam0 = [&](const double* x, double* out) { return apply_Lambda(tb, w, &co0, x, false, out, st); };
  // Sigma_0 g = L^T W0 [K; H] g
  SHIP(launch_gemv_n_ld(tb->f64, tb->d_K, d * n, p, p, g, 1.0, 0.0, y1, st));
  SHIP(launch_gemv_n_ld(tb->f64, tb->d_H, n, p, p, g, 1.0, 0.0, y1 + (size_t)d * n, st));
  SHIP(launch_apply_w(n, d, tb->d_lambda, nullptr, nullptr, nullptr, y1, false, nullptr, y2, st));
  if ((s = apply_Lt(tb, w, y2, 1.0, 0.0, sig0g, st)) != WOS_OK) return s;
  auto load_lam0 = [&]() -> wos_status {
    if (mixed)
      SHIP(hipMemcpyAsync(w.N32, w.L0_32, sizeof(float) * m * m, hipMemcpyDeviceToDevice, st));
    else
      SHIP(hipMemcpyAsync(w.Hess, w.Lam0, sizeof(double) * m * m, hipMemcpyDeviceToDevice, st));
    return WOS_OK;
  };
  // h0: the problem without the cubic term, Lambda_0 h = A^T (lambda f) - Sigma_0 g
  SHIP(launch_pointwise(n, tb->d_lambda, nullptr, f, 0.0, 0.0, 0.0, 0.0, -1.0, t1, st));
  SHIP(launch_gemv_t_ld(tb->f64, tb->d_A, n, m, m, t1, 1.0, 0.0, grad, w.part, st));
  SHIP(launch_axpy_reg(m, grad, nullptr, -1.0, sig0g, grad, st));
  if ((s = load_lam0()) != WOS_OK) return s;
  // mixed: the exact FP64 diagonal of Lambda_0, sum_a sum_i lambda_i B^(a)_ij^2
  double* diag0 = mixed ? w.cn : nullptr;
  double* diagH = mixed ? w.cn + m : nullptr;
  if (mixed)
    SHIP(launch_colsq(tb->f64, tb->d_B, d * n, m, m, tb->d_lambda, n, false, w.colp, diag0, st));
  if ((s = sym_reg_solve(tb, w, mixed, rcond, rtol, rmax, grad, q, apply_lam0, diag0, inf, st)) != WOS_OK) return s;
  double gn0 = -1.0, gn = 0.0;
  int it = 0;
  for (it = 0; it <= max_iter; ++it) {
    if ((s = reconstruct(tb, q, g, uu, nullptr, st)) != WOS_OK) return s;
    // grad = A^T (lambda (kappa u^3 - f)) + Lambda_0 h + Sigma_0 g
    SHIP(launch_pointwise(n, tb->d_lambda, uu, f, 0.0, 0.0, 0.0, kappa, 1.0, t1, st));
    if ((s = apply_lam0(q, grad)) != WOS_OK) return s;
    SHIP(launch_gemv_t_ld(tb->f64, tb->d_A, n, m, m, t1, 1.0, 1.0, grad, w.part, st));
    SHIP(launch_axpy_reg(m, grad, nullptr, 1.0, sig0g, grad, st));
    if ((s = dev_dot(w, grad, grad, nullptr, m, &gn, st)) != WOS_OK) return s;
    gn = std::sqrt(gn);
    if (gn0 < 0) gn0 = gn;
    if (gn <= tol * gn0 || it == max_iter) break;
    // Hessian = Lambda_0 + A^T diag(wts) A, wts = 3 kappa lambda u^2
    SHIP(launch_pointwise(n, tb->d_lambda, uu, nullptr, 0.0, 0.0, 3.0 * kappa, 0.0, 0.0, wts, st));
    if ((s = load_lam0()) != WOS_OK) return s;
    SHIP(launch_scale_rows(tb->f64, mixed, tb->d_A, n, m, wts, mixed ? (void*)w.R32 : (void*)w.R, st));
    if (mixed)
      SHIP(mfma_gemm_lower_f32(true, false, m, m, n, 1.0f, (const float*)tb->d_A, m, w.R32, m, 1.0f, w.N32, m, st));
    else if (tb->f64)
      SHIP(mfma_gemm_lower_f64(true, false, m, m, n, 1.0, (const double*)tb->d_A, m, w.R, m, 1.0, w.Hess, m, st));
    else
      SHIP(mfma_gemm_lower_f64_a32(true, false, m, m, n, 1.0, (const float*)tb->d_A, m, w.R, m, 1.0, w.Hess, m, st));
    auto apply_hess = [&](const double* x, double* out) -> wos_status {
      wos_status s2 = apply_lam0(x, out);
      if (s2 != WOS_OK) return s2;
      SHIP(launch_gemv_n_ld(tb->f64, tb->d_A, n, m, m, x, 1.0, 0.0, tmp, st));
      SHIP(launch_pointwise(n, wts, nullptr, tmp, 0.0, 0.0, 0.0, 0.0, -1.0, tmp, st));
      SHIP(launch_gemv_t_ld(tb->f64, tb->d_A, n, m, m, tmp, 1.0, 1.0, out, w.part, st));
      return WOS_OK;
    };
    if (mixed) {
      // the Hessian's exact diagonal: Lambda_0's plus sum_i wts_i A_ij^2
      SHIP(hipMemcpyAsync(diagH, diag0, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
      SHIP(launch_colsq(tb->f64, tb->d_A, n, m, m, wts, n, true, w.colp, diagH, st));
    }
    if ((s = sym_reg_solve(tb, w, mixed, rcond, rtol, rmax, grad, dlt, apply_hess, diagH, inf, st)) != WOS_OK)
      return s;
    SHIP(launch_axpy_reg(m, q, nullptr, -1.0, dlt, q, st));
  }
  inf->iters = it;
  inf->grad_norm = gn;
  inf->grad_norm0 = gn0;
  return WOS_OK;
}

}  // namespace

namespace wos {

void free_work(SolveWork& w) {
  void* ptrs[] = {w.R, w.Lam, w.Sig, w.Lam0, w.Sig0, w.Hess, w.G, w.V, w.E, w.rot, w.pq, w.vec, w.Ac, w.red,
                  w.blk, w.regv, w.colp, w.cn, w.info, w.R32, w.Lam32, w.N32, w.v32, w.P64, w.P32, w.L0_32, w.el, w.hs,
                  w.hs_bad, w.hsb, w.part, w.RT, w.cg, w.aj};
  if (!w.fixed)
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
  if (w.cap) (void)hipStreamDestroy(w.cap);
  w = SolveWork();
}

// One solve on the workspace `w` (the toolbox's own, or a server slot's).
wos_status solve_request(wos_toolbox* tb, SolveWork& w, const wos_coeffs* co, const double* f, const double* g,
                         double* u, double* grad_u, double* q_out, wos_solve_info* info, hipStream_t st) {
  if (!tb || !co || !f || !g || !u) return sfail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return sfail(WOS_EINVAL, "toolbox has not been built");
  fit_work(tb, w);
  if (tb->n != tb->m && co->kind != WOS_LINEAR)
    return sfail(WOS_EINVAL, "only LINEAR solves are supported on a toolbox with a separate V partition");
  const double rcond = co->rcond > 0 ? co->rcond : 1e-3;
  if (!(rcond < 1.0)) return sfail(WOS_EINVAL, "rcond must be in (0, 1)");
  if (co->solver != WOS_SOLVER_TSVD && co->solver != WOS_SOLVER_TIKHONOV)
    return sfail(WOS_EINVAL, "unknown solver %d", co->solver);
  if (co->precision != WOS_SOLVE_F64 && co->precision != WOS_SOLVE_MIXED && co->precision != WOS_SOLVE_MIXED_BF16)
    return sfail(WOS_EINVAL, "unknown solve precision %d", co->precision);
  if (co->precision == WOS_SOLVE_MIXED_BF16 &&
      !(co->solver == WOS_SOLVER_TIKHONOV && (co->kind == WOS_LINEAR || co->kind == WOS_QUASILINEAR)))
    return sfail(WOS_EINVAL, "the BF16 route solves LINEAR and QUASILINEAR problems with the Tikhonov solver");
  const int max_sweeps = co->max_sweeps > 0 ? co->max_sweeps : 40;
  wos_status s = ensure_work(tb, w);
  if (s != WOS_OK) return s;
  if ((s = ensure_part(tb, w, 1, st)) != WOS_OK) return s;
  const int n = tb->n, m = tb->m, d = tb->dim;
  double* rhs = w.vec + 0 * w.vlen;
  double* q = w.vec + 1 * w.vlen;
  double* uu = w.vec + 2 * w.vlen;
  double* t1 = w.vec + 3 * w.vlen;
  double* t2 = w.vec + 4 * w.vlen;
  wos_solve_info inf{};
  inf.refine_converged = 1;
  TsvdResult tr;

  if (co->kind == WOS_LINEAR && co->solver == WOS_SOLVER_TIKHONOV) {
    if ((s = tikhonov_linear(tb, w, co, rcond, f, g, q, &inf, st)) != WOS_OK) return s;
    inf.iters = 1;
  } else if (co->kind == WOS_LINEAR) {
    if ((s = assemble(tb, w, co->A, co->b, co->c, w.Lam, w.Sig, st)) != WOS_OK) return s;
    if ((s = linear_rhs(tb, w, w.Sig, f, g, rhs, st)) != WOS_OK) return s;
    if ((s = tsvd_solve(tb, w, w.Lam, co->b == nullptr, rhs, rcond, max_sweeps, q, &tr, st)) != WOS_OK) return s;
    inf.iters = 1;
  } else if (co->kind == WOS_SEMILINEAR_CUBIC && co->solver == WOS_SOLVER_TIKHONOV) {
    if ((s = newton_tikhonov(tb, w, co, rcond, f, g, q, &inf, st)) != WOS_OK) return s;
  } else if (co->kind == WOS_SEMILINEAR_CUBIC) {
    // F = |p|^2/2 + kappa u^4/4 - f u; grad J = A^T(lam (kappa u^3 - f)) + Lam0 h + Sig0 g
    const double kappa = co->kappa;
    const double tol = co->tol > 0 ? co->tol : 1e-8;
    const int max_iter = co->max_iter > 0 ? co->max_iter : 50;
    if ((s = assemble(tb, w, nullptr, nullptr, nullptr, w.Lam0, w.Sig0, st)) != WOS_OK) return s;
    // h0: the problem without the cubic term, rhs = A^T (lam f) - Sig0 g
    SHIP(launch_pointwise(n, tb->d_lambda, nullptr, f, 0.0, 0.0, 0.0, 0.0, -1.0, t1, st));
    SHIP(launch_gemv_t(tb->f64, tb->d_A, n, m, t1, 1.0, 0.0, rhs, st));
    SHIP(launch_gemv_n(true, w.Sig0, m, tb->p, g, -1.0, 1.0, rhs, st));
    if ((s = tsvd_solve(tb, w, w.Lam0, true, rhs, rcond, max_sweeps, q, &tr, st)) != WOS_OK) return s;
    double gn0 = -1.0, gn = 0.0;
    int it = 0;
    for (it = 0; it <= max_iter; ++it) {
      if ((s = reconstruct(tb, q, g, uu, nullptr, st)) != WOS_OK) return s;
      // grad = A^T (lam (kappa u^3 - f)) + Lam0 h + Sig0 g
      SHIP(launch_pointwise(n, tb->d_lambda, uu, f, 0.0, 0.0, 0.0, kappa, 1.0, t1, st));
      SHIP(launch_gemv_t(tb->f64, tb->d_A, n, m, t1, 1.0, 0.0, rhs, st));
      SHIP(launch_gemv_n(true, w.Lam0, m, m, q, 1.0, 1.0, rhs, st));
      SHIP(launch_gemv_n(true, w.Sig0, m, tb->p, g, 1.0, 1.0, rhs, st));
      if ((s = dev_dot(w, rhs, rhs, nullptr, m, &gn, st)) != WOS_OK) return s;
      gn = std::sqrt(gn);
      if (gn0 < 0) gn0 = gn;
      if (gn <= tol * gn0 || it == max_iter) break;
      // Hessian = Lam0 + A^T diag(3 kappa lam u^2) A
      SHIP(hipMemcpyAsync(w.Hess, w.Lam0, sizeof(double) * m * m, hipMemcpyDeviceToDevice, st));
      SHIP(launch_pointwise(n, tb->d_lambda, uu, nullptr, 0.0, 0.0, 3.0 * kappa, 0.0, 0.0, t2, st));
      SHIP(launch_gram(tb->f64, tb->d_A, n, m, t2, w.Hess, st));
      if ((s = tsvd_solve(tb, w, w.Hess, true, rhs, rcond, max_sweeps, t1, &tr, st)) != WOS_OK) return s;
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
      if (co->solver == WOS_SOLVER_TIKHONOV) {
        wos_coeffs cl = *co;
        cl.kind = WOS_LINEAR;
        cl.A = w.Ac;
        cl.b = nullptr;
        cl.c = nullptr;
        if ((s = tikhonov_linear(tb, w, &cl, rcond, fp, g, q, &inf, st)) != WOS_OK) return s;
      } else {
        if ((s = assemble(tb, w, w.Ac, nullptr, nullptr, w.Lam, w.Sig, st)) != WOS_OK) return s;
        if ((s = linear_rhs(tb, w, w.Sig, fp, g, rhs, st)) != WOS_OK) return s;
        if ((s = tsvd_solve(tb, w, w.Lam, true, rhs, rcond, max_sweeps, q, &tr, st)) != WOS_OK) return s;
      }
      if ((s = reconstruct(tb, q, g, t1, nullptr, st)) != WOS_OK) return s;
      // du = |u_new - u|_lam, nu = |u_new|_lam
      SHIP(launch_axpby(n, 1.0, t1, -1.0, uu, rhs, st));
      if ((s = dev_dot(w, rhs, rhs, tb->d_lambda, n, &du, st)) != WOS_OK) return s;
      if ((s = dev_dot(w, t1, t1, tb->d_lambda, n, &nu, st)) != WOS_OK) return s;
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
  // the regularisation parameter of the last Tikhonov solve, read at the
  // final synchronisation (no copy into `inf` is left pending on a return)
  if (co->solver == WOS_SOLVER_TIKHONOV && w.regv)
    SHIP(hipMemcpyAsync(&inf.reg, w.regv, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  if (co->solver == WOS_SOLVER_TSVD) {
    inf.rank = tr.rank;
    inf.sweeps = tr.sweeps;
    inf.sigma_max = tr.smax;
    inf.sigma_threshold = tr.smin_kept;
  }
  if (info) *info = inf;
  return WOS_OK;
}

// ------------------------------------------------ Euler-Lagrange route
// grad J for one energy, its constant parts formed once (`setup`):
// c = A^T (-lambda o f) when dF/du = -f (else 0), K g, and H g when u
// enters dF/du.  `acc` adds B^T yB(x) (+ A^T yA(x)) onto `out`, which
// holds c; `eval` first sets out = c.
struct ElGrad {
  wos_toolbox* tb = nullptr;
  int kind = 0;
  double P = 2.0;
  bool uterm = false;
  const double* f = nullptr;
  EnergyCoef co;           // kind 3 coefficients
  double* cvec = nullptr;  // m
  double* gB = nullptr;    // d n
  double* yB = nullptr;    // (d + 1) n: the B weights, then yA
  double* yA = nullptr;
  double* kgv = nullptr;   // d n
  double* hg = nullptr;    // n
  double* uA = nullptr;    // n
  double* part = nullptr;  // partial sums of the transposed products
  hipStream_t st = nullptr;

  // carves m + (3d + 3) n doubles from `base`; returns the first one after
  double* carve(double* base) {
    const size_t n = tb->n, m = tb->m, d = tb->dim;
    cvec = base;
    gB = cvec + m;
    yB = gB + d * n;
    yA = yB + d * n;
    kgv = yA + n;
    hg = kgv + d * n;
    uA = hg + n;
    return uA + n;
  }
  wos_status setup(const double* g) {
    const int n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
    if (uterm) {
      SHIP(hipMemsetAsync(cvec, 0, sizeof(double) * m, st));
      if (p > 0)
        SHIP(launch_gemv_n_ld(tb->f64, tb->d_H, n, p, p, g, 1.0, 0.0, hg, st));
      else
        SHIP(hipMemsetAsync(hg, 0, sizeof(double) * n, st));
    } else {
      SHIP(launch_pointwise(n, tb->d_lambda, nullptr, f, 0.0, 0.0, 0.0, 0.0, 1.0, yA, st));  // -lambda f
      SHIP(launch_gemv_t_ld(tb->f64, tb->d_A, n, m, m, yA, 1.0, 0.0, cvec, part, st));
    }
    if (p > 0)
      SHIP(launch_gemv_n_ld(tb->f64, tb->d_K, d * n, p, p, g, 1.0, 0.0, kgv, st));
    else
      SHIP(hipMemsetAsync(kgv, 0, sizeof(double) * (size_t)d * n, st));
    return WOS_OK;
  }
  wos_status acc(const double* x, double* out) {
    const int n = tb->n, m = tb->m, d = tb->dim;
    SHIP(launch_gemv_n_ld(tb->f64, tb->d_B, d * n, m, m, x, 1.0, 0.0, gB, st));
    if (uterm) SHIP(launch_gemv_n_ld(tb->f64, tb->d_A, n, m, m, x, 1.0, 0.0, uA, st));
    SHIP(launch_energy_wb(kind, n, d, P, tb->d_lambda, gB, kgv, yB, uterm ? uA : nullptr, hg, f, yA, co, st));
    SHIP(launch_gemv_t_acc(tb->f64, tb->d_B, d * n, m, m, yB, 1.0, out, part, st));
    if (uterm) SHIP(launch_gemv_t_acc(tb->f64, tb->d_A, n, m, m, yA, 1.0, out, part, st));
    return WOS_OK;
  }
  wos_status eval(const double* x, double* out) {
    SHIP(hipMemcpyAsync(out, cvec, sizeof(double) * tb->m, hipMemcpyDeviceToDevice, st));
    return acc(x, out);
  }
  // whether eval_batch reads the toolbox once for nv points (nv odd in
  // 3..17: the 2k + 1 points of a saddle-search iteration); otherwise it
  // evaluates one point at a time
  static bool batchable(int nv) { return nv >= 3 && nv <= 17 && (nv & 1); }
  // out[t] = grad J(x[t]) for nv points stored one after another (m each);
  // scratch holds nv (2d + 2) n doubles
  wos_status eval_batch(const double* x, double* out, int nv, double* scratch) {
    const int n = tb->n, m = tb->m, d = tb->dim;
    if (!batchable(nv)) {
      for (int t = 0; t < nv; ++t) {
        wos_status s = eval(x + (size_t)t * m, out + (size_t)t * m);
        if (s != WOS_OK) return s;
      }
      return WOS_OK;
    }
    const size_t dn = (size_t)d * n;
    double* GB = scratch;                   // nv d n
    double* UA = GB + (size_t)nv * dn;      // nv n
    double* YB = UA + (size_t)nv * n;       // nv (d + 1) n
    SHIP(launch_gemv_batch(tb->f64, false, tb->d_B, d * n, m, m, x, m, nv, GB, (int)dn, part, st));
    if (uterm) SHIP(launch_gemv_batch(tb->f64, false, tb->d_A, n, m, m, x, m, nv, UA, n, part, st));
    SHIP(launch_energy_wb_batch(kind, n, d, P, tb->d_lambda, GB, kgv, YB, uterm ? UA : nullptr, hg, f, nv, co, st));
    SHIP(launch_hisd_broadcast(m, nv, cvec, out, st));
    SHIP(launch_gemv_batch(tb->f64, true, tb->d_B, d * n, m, m, YB, (int)(dn + n), nv, out, m, part, st));
    if (uterm) SHIP(launch_gemv_batch(tb->f64, true, tb->d_A, n, m, m, YB + dn, (int)(dn + n), nv, out, m, part, st));
    return WOS_OK;
  }
};

wos_status check_energy(int kind, double p_exp) {
  if (kind != WOS_EL_PLAPLACE && kind != WOS_EL_MINIMAL_SURFACE && kind != WOS_EL_SEMILINEAR &&
      kind != WOS_EL_ELLIPTIC)
    return sfail(WOS_EINVAL, "unknown energy %d", kind);
  if (kind == WOS_EL_PLAPLACE && !(p_exp > 1.0)) return sfail(WOS_EINVAL, "p_exp must be > 1");
  return WOS_OK;
}

// Adam on J(fbar) = sum_i lambda_i F(x_i, u_i, grad u_i) (eq. gradJ).  For
// the p-Laplace and minimal surface energies dF/du = -f does not depend on
// u, so grad J = c + B^T yB with the constant c = A^T (-lambda o f) and
// yB = lambda dF/dp(p), p = B fbar + K g (K g fixed too).  An iteration
// therefore streams B twice (B fbar, then B^T yB accumulated onto c) and
// nothing else: four kernels, all on the device.  The semilinear energy's
// dF/du = f - u^2 does depend on u: its iteration also forms u = A fbar +
// H g (H g fixed) and accumulates A^T (lambda o dF/du), so it streams A
// twice as well, c being 0.  u = A fbar + H g and J are formed once at the
// end.
wos_status minimize_request(wos_toolbox* tb, SolveWork& w, const wos_adam_opts* o, const double* f, const double* g,
                            double* fbar, double* u, double* grad_u, wos_adam_info* info, hipStream_t st) {
  if (!o || !f || !g || !fbar || !u) return sfail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return sfail(WOS_EINVAL, "toolbox has not been built");
  fit_work(tb, w);
  const int kind = o->energy;
  wos_status s;
  if ((s = check_energy(kind, o->p_exp)) != WOS_OK) return s;
  const double P = kind == WOS_EL_PLAPLACE ? o->p_exp : 2.0;
  // a negative beta asks for the paper's value; 0 is a valid choice
  const double b1 = o->beta1 < 0 ? 0.9 : o->beta1;
  const double b2 = o->beta2 < 0 ? 0.999 : o->beta2;
  const double eps = o->eps > 0 ? o->eps : 1e-10;
  const int check = o->check_every > 0 ? o->check_every : 50;
  if (!(o->alpha > 0.0)) return sfail(WOS_EINVAL, "alpha must be > 0");
  if (!(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0)) return sfail(WOS_EINVAL, "beta1, beta2 must be in [0, 1)");
  if (o->eps < 0.0 || !(o->tol >= 0.0)) return sfail(WOS_EINVAL, "eps and tol must be >= 0");
  if (o->max_iter <= 0) return sfail(WOS_EINVAL, "max_iter must be > 0");
  const int n = tb->n, m = tb->m, d = tb->dim;
  if (!w.el && (s = walloc(w, &w.el, (size_t)(3 * d + 4) * n + 4 * (size_t)m + 2)) != WOS_OK) return s;
  if ((s = ensure_part(tb, w, 1, st)) != WOS_OK) return s;
  ElGrad eg;
  eg.tb = tb;
  eg.kind = kind;
  eg.P = P;
  eg.uterm = kind == WOS_EL_SEMILINEAR || kind == WOS_EL_ELLIPTIC;  // dF/du depends on u
  eg.f = f;
  eg.part = w.part;
  eg.st = st;
  eg.co.A = o->coef_A;
  eg.co.c = o->coef_c;
  eg.co.w = o->coef_w;
  double* F = eg.carve(w.el);           // n: the energy density at the end
  double* grad = F + n;                 // m
  double* mv = grad + m;                // m
  double* vv = mv + m;                  // m
  double* red = vv + m;                 // 2
  double* gB = eg.gB;                   // at the end: grad u when the caller passes none
  double* yB = eg.yB;                   // at the end: all weights
  double* cvec = eg.cvec;
  SHIP(hipMemsetAsync(mv, 0, sizeof(double) * 2 * (size_t)m, st));
  if ((s = eg.setup(g)) != WOS_OK) return s;
  SHIP(hipMemcpyAsync(grad, cvec, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
  // grad += B^T yB(x) (+ A^T yA(x))  (grad holds c on entry)
  auto gradient = [&](const double* x) -> wos_status { return eg.acc(x, grad); };
  auto weighted = [&](const double* x, const double* z, double* out) -> wos_status {
    SHIP(launch_dot(m, x, z, tb->d_lambda_v, red, st));  // the V cells' measures
    SHIP(hipMemcpyAsync(out, red, sizeof(double), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    return WOS_OK;
  };
  wos_adam_info inf{};
  double gg = 0.0;
  if ((s = gradient(fbar)) != WOS_OK) return s;
  if ((s = weighted(grad, grad, &gg)) != WOS_OK) return s;
  inf.grad_norm0 = std::sqrt(gg);
  const auto t0 = std::chrono::steady_clock::now();
  // the step sizes alpha sqrt(1 - beta2^j) / (1 - beta1^j)
  std::vector<double> ajh(o->max_iter);
  {
    double b1j = 1.0, b2j = 1.0;
    for (int j = 1; j <= o->max_iter; ++j) {
      b1j *= b1;
      b2j *= b2;
      ajh[j - 1] = o->alpha * std::sqrt(1.0 - b2j) / (1.0 - b1j);
    }
  }
  int it = 0;
  bool done = false;
  // blocks of C iterations replayed from one captured graph: the Adam
  // kernel of the block's i-th iteration reads its step size from slot i,
  // which is filled from the table of all step sizes before each replay
  const int C = o->tol > 0.0 ? check : 64;
  if (o->graph && o->max_iter >= C) {
    const size_t need = (size_t)o->max_iter + C;
    if (w.aj_cap < need) {
      if (w.aj) {
        SHIP(hipStreamSynchronize(st));
        SHIP(hipFree(w.aj));
        w.bytes -= w.aj_cap * sizeof(double);
        w.aj = nullptr;
        w.aj_cap = 0;
      }
      if ((s = walloc(w, &w.aj, need)) != WOS_OK) return s;
      w.aj_cap = need;
    }
    double* slot = w.aj + o->max_iter;
    SHIP(hipMemcpyAsync(w.aj, ajh.data(), sizeof(double) * o->max_iter, hipMemcpyHostToDevice, st));
    SHIP(hipStreamSynchronize(st));
    if (!w.cap) SHIP(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SHIP(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal));
    eg.st = w.cap;
    wos_status cs = WOS_OK;
    for (int i = 0; i < C && cs == WOS_OK; ++i) {
      if (launch_adam_dev(m, grad, b1, b2, eps, slot + i, mv, vv, fbar, cvec, w.cap) != hipSuccess)
        cs = sfail(WOS_EDEVICE, "Adam: launch failed during graph capture");
      else
        cs = eg.acc(fbar, grad);
    }
    eg.st = st;
    const hipError_t ce = hipStreamEndCapture(w.cap, &graph);
    if (cs != WOS_OK) {
      if (ce == hipSuccess && graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    SHIP(ce);
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      SHIP(ie);
    }
    hipError_t le = hipSuccess;
    for (int j0 = 0; j0 + C <= o->max_iter && le == hipSuccess; j0 += C) {
      le = hipMemcpyAsync(slot, w.aj + j0, sizeof(double) * C, hipMemcpyDeviceToDevice, st);
      if (le == hipSuccess) le = hipGraphLaunch(exec, st);
      it = j0 + C;
      if (le == hipSuccess && o->tol > 0.0 && it % check == 0) {
        if ((s = weighted(grad, grad, &gg)) != WOS_OK) break;
        if (std::sqrt(gg) <= o->tol) {
          done = true;
          break;
        }
      }
    }
    (void)hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    SHIP(le);
    if (s != WOS_OK) return s;
  }
  for (int j = it + 1; j <= o->max_iter && !done; ++j) {
    SHIP(launch_adam(m, grad, b1, b2, eps, ajh[j - 1], mv, vv, fbar, cvec, st));  // grad <- c afterwards
    it = j;
    if ((s = gradient(fbar)) != WOS_OK) return s;  // at the new fbar: next step and the checks
    if (o->tol > 0.0 && j % check == 0) {
      if ((s = weighted(grad, grad, &gg)) != WOS_OK) return s;
      if (std::sqrt(gg) <= o->tol) break;
    }
  }
  SHIP(hipStreamSynchronize(st));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  inf.iters = it;
  if ((s = weighted(grad, grad, &gg)) != WOS_OK) return s;
  inf.grad_norm = std::sqrt(gg);
  // u, grad u and J = sum_i lambda_i F_i at the result
  if ((s = reconstruct(tb, fbar, g, u, grad_u ? grad_u : gB, st)) != WOS_OK) return s;
  SHIP(launch_energy_weights(kind, n, d, P, tb->d_lambda, u, grad_u ? grad_u : gB, f, yB, F, eg.co, st));
  SHIP(launch_dot(n, F, tb->d_lambda, nullptr, red, st));
  SHIP(hipMemcpyAsync(&inf.J, red, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  if (info) *info = inf;
  return WOS_OK;
}

// ------------------------------------------------ saddle search (p-HiSD)
// The inverse X ~ A^-1 (m x m, FP64) by Newton-Schulz: X_0 = A^T / |A|_F^2
// (so that I - A X_0 has its spectrum in [0, 1)), then X <- X + X D with
// D = I - A X, whose residual squares at each step (I - A X' = D^2).  Stops
// once |D|_F <= 1e-13 sqrt(m), or when it no longer falls (rounding), or
// after 100 steps.
static wos_status ns_inverse(wos_toolbox* tb, double* X, double* Y, double* D, double* red, int* iters,
                             double* resid, hipStream_t st) {
  const int m = tb->m;
  const size_t mm = (size_t)m * m;
  SHIP(launch_transpose_to_f64(tb->f64, tb->d_A, m, X, st));
  double nf2 = 0.0;
  SHIP(launch_dot((int)mm, X, X, nullptr, red, st));
  SHIP(hipMemcpyAsync(&nf2, red, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  if (!(nf2 > 0.0) || !std::isfinite(nf2)) return sfail(WOS_EINVAL, "p-HiSD: A is zero or not finite");
  SHIP(launch_axpby((int)mm, 1.0 / nf2, X, 0.0, nullptr, X, st));
  double prev = INFINITY, r2 = 0.0;
  int it = 0;
  for (; it < 100; ++it) {
    // D = I - A X
    if (tb->f64)
      SHIP(mfma_gemm_f64(false, false, m, m, m, 1.0, static_cast<const double*>(tb->d_A), m, X, m, 0.0, D, m, st));
    else
      SHIP(mfma_gemm_f64_a32(false, false, m, m, m, 1.0, static_cast<const float*>(tb->d_A), m, X, m, 0.0, D, m,
                             st));
    SHIP(launch_identity_minus(m, D, st));
    SHIP(launch_dot((int)mm, D, D, nullptr, red, st));
    SHIP(hipMemcpyAsync(&r2, red, sizeof(double), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (!std::isfinite(r2)) return sfail(WOS_EINVAL, "p-HiSD: the inverse of A diverged");
    if (r2 <= 1e-26 * m || (prev < 1e-6 && r2 > 0.25 * prev)) break;
    prev = r2;
    // X <- X + X D  (into Y, then swapped back by copy)
    SHIP(hipMemcpyAsync(Y, X, sizeof(double) * mm, hipMemcpyDeviceToDevice, st));
    SHIP(mfma_gemm_f64(false, false, m, m, m, 1.0, X, m, D, m, 1.0, Y, m, st));
    SHIP(hipMemcpyAsync(X, Y, sizeof(double) * mm, hipMemcpyDeviceToDevice, st));
  }
  *iters = it;
  *resid = std::sqrt(r2);
  return WOS_OK;
}

wos_status saddle_request(wos_toolbox* tb, SolveWork& w, const wos_hisd_opts* o, const double* f, const double* g,
                          double* fbar, double* V, double* u, double* grad_u, wos_hisd_info* info, hipStream_t st) {
  if (!o || !f || !g || !fbar || !V || !u) return sfail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return sfail(WOS_EINVAL, "toolbox has not been built");
  fit_work(tb, w);
  const int kind = o->energy;
  wos_status s;
  if ((s = check_energy(kind, o->p_exp)) != WOS_OK) return s;
  if (kind == WOS_EL_ELLIPTIC) return sfail(WOS_EINVAL, "p-HiSD: the weighted quadratic energy has no saddle points");
  const int n = tb->n, m = tb->m, d = tb->dim, k = o->k;
  if (k < 1 || k > 8 || k > m) return sfail(WOS_EINVAL, "k must be in 1..min(8, m)");
  if (!(o->eta > 0.0) || !(o->tau > 0.0)) return sfail(WOS_EINVAL, "eta and tau must be > 0");
  if (o->max_iter <= 0) return sfail(WOS_EINVAL, "max_iter must be > 0");
  if (!(o->tol >= 0.0)) return sfail(WOS_EINVAL, "tol must be >= 0");
  if (o->precond != WOS_HISD_PRECOND_IDENTITY && o->precond != WOS_HISD_PRECOND_A)
    return sfail(WOS_EINVAL, "unknown preconditioner %d", o->precond);
  if (o->init != WOS_HISD_INIT_GIVEN && o->init != WOS_HISD_INIT_HESSIAN)
    return sfail(WOS_EINVAL, "unknown initialisation %d", o->init);
  const bool useA = o->precond == WOS_HISD_PRECOND_A;
  if (useA && (n != m || m > 16384)) return sfail(WOS_EINVAL, "the preconditioner A needs n = m <= 16384");
  if (o->init == WOS_HISD_INIT_HESSIAN && kind != WOS_EL_SEMILINEAR)
    return sfail(WOS_EINVAL, "the Hessian initialisation is provided for the semilinear energy only");
  const int check = o->check_every > 0 ? o->check_every : 50;
  const double P = kind == WOS_EL_PLAPLACE ? o->p_exp : 2.0;
  const size_t mm = (size_t)m * m;
  if (!w.el && (s = walloc(w, &w.el, (size_t)(3 * d + 4) * n + 4 * (size_t)m + 2)) != WOS_OK) return s;
  // the three m x m Newton-Schulz matrices only with M = A; the buffer
  // grows when a later call needs more
  const size_t nmat = useA ? 3 * mm : 0;
  const size_t hs_len = nmat + 78 * (size_t)m + 8;
  if (w.hs_cap < hs_len) {
    if (w.hs) {
      SHIP(hipStreamSynchronize(st));
      SHIP(hipFree(w.hs));
      w.bytes -= w.hs_cap * sizeof(double);
      w.hs = nullptr;
      w.hs_cap = 0;
    }
    if ((s = walloc(w, &w.hs, hs_len)) != WOS_OK) return s;
    w.hs_cap = hs_len;
  }
  if (!w.hs_bad && (s = walloc(w, &w.hs_bad, 1)) != WOS_OK) return s;
  if ((s = ensure_part(tb, w, std::min(17, 2 * k + 1), st)) != WOS_OK) return s;
  ElGrad eg;
  eg.tb = tb;
  eg.kind = kind;
  eg.P = P;
  eg.uterm = kind == WOS_EL_SEMILINEAR || kind == WOS_EL_ELLIPTIC;
  eg.f = f;
  eg.part = w.part;
  hipStream_t cs = st;  // the stream the iteration's launches go to (switched while capturing)
  eg.st = st;
  double* F = eg.carve(w.el);  // n
  double* red = F + n;         // 2 (the Adam route's slots are not used here)
  double* Minv = w.hs;         // m^2 (M = A)
  double* Y2 = Minv + mm;      // m^2 (Newton-Schulz)
  double* D = Y2 + mm;         // m^2 (Newton-Schulz)
  double* Vc = w.hs + nmat;    // 8 m: the directions
  double* Vn = Vc + 8 * (size_t)m;   // 8 m
  double* MV = Vn + 8 * (size_t)m;   // 8 m: M V
  double* HV = MV + 8 * (size_t)m;   // 9 m: H v_i, then grad J
  double* Yv = HV + 9 * (size_t)m;   // 9 m: M^-1 of them
  double* Xs = Yv + 9 * (size_t)m;   // 17 m: fbar +- h v_i, then fbar
  double* Gs = Xs + 17 * (size_t)m;  // 17 m: their gradients
  double* gr0 = Gs + 17 * (size_t)m; // m: the gradient at the start
  double* wv = gr0 + m;              // m: M^-1 grad J
  double* hbuf = wv + m;             // 8: the difference step h (device)
  if ((size_t)(hbuf + 8 - w.hs) > hs_len) return sfail(WOS_EINVAL, "p-HiSD: work layout");
  const int nv = 2 * k + 1;  // the points of one iteration's gradients
  if (eg.batchable(nv) && !w.hsb && (s = walloc(w, &w.hsb, 17 * (size_t)(2 * d + 2) * n)) != WOS_OK) return s;
  wos_hisd_info inf{};
  if ((s = eg.setup(g)) != WOS_OK) return s;
  if (useA) {
    if ((s = ns_inverse(tb, Minv, Y2, D, red, &inf.ns_iters, &inf.ns_residual, st)) != WOS_OK) return s;
    // the GPU update uses v^T grad J for v^T M (M^-1 grad J): M^-1 must be
    // an inverse to well below the iteration's own accuracy
    if (!(inf.ns_residual <= 1e-6 * std::sqrt((double)m)))
      return sfail(WOS_ENOTCONV, "p-HiSD: the Newton-Schulz inverse of A reached only |I - A X|_F = %g", inf.ns_residual);
  }
  // y = M^-1 x, and M x, for one vector
  auto minv = [&](const double* x, double* y) -> wos_status {
    if (useA)
      SHIP(launch_gemv_n(true, Minv, m, m, x, 1.0, 0.0, y, cs));
    else
      SHIP(hipMemcpyAsync(y, x, sizeof(double) * m, hipMemcpyDeviceToDevice, cs));
    return WOS_OK;
  };
  // Y[t] = M^-1 X[t] for nv vectors: one pass over M^-1
  auto minv_batch = [&](const double* X, int nvec, double* Y) -> wos_status {
    if (useA)
      SHIP(launch_gemv_batch(true, false, Minv, m, m, m, X, m, nvec, Y, m, w.part, cs));
    else
      SHIP(hipMemcpyAsync(Y, X, sizeof(double) * nvec * (size_t)m, hipMemcpyDeviceToDevice, cs));
    return WOS_OK;
  };
  auto mult = [&](const double* x, double* y) -> wos_status {
    if (useA)
      SHIP(launch_gemv_n_ld(tb->f64, tb->d_A, m, m, m, x, 1.0, 0.0, y, cs));
    else
      SHIP(hipMemcpyAsync(y, x, sizeof(double) * m, hipMemcpyDeviceToDevice, cs));
    return WOS_OK;
  };
  // the Gram-Schmidt flag is sticky: cleared once, read (with a
  // synchronisation) after the first pass, at the norm checks and at the end
  auto orthonormalise = [&](double* Vx) -> wos_status {
    if (useA && k >= 2) {  // M V in one pass over A
      SHIP(launch_gemv_batch(tb->f64, false, tb->d_A, m, m, m, Vx, m, k, MV, m, w.part, cs));
    } else {
      for (int i = 0; i < k; ++i)
        if ((s = mult(Vx + (size_t)i * m, MV + (size_t)i * m)) != WOS_OK) return s;
    }
    SHIP(launch_hisd_gs(m, k, Vx, MV, w.hs_bad, cs));
    return WOS_OK;
  };
  auto check_bad = [&]() -> wos_status {
    int bad = 0;
    SHIP(hipMemcpyAsync(&bad, w.hs_bad, sizeof(int), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (bad) return sfail(WOS_EINVAL, "p-HiSD: the directions are not M-independent");
    return WOS_OK;
  };
  SHIP(hipMemsetAsync(w.hs_bad, 0, sizeof(int), st));
  auto weighted_norm = [&](const double* x, double* out) -> wos_status {
    SHIP(launch_dot(m, x, x, tb->d_lambda_v, red, st));
    SHIP(hipMemcpyAsync(out, red, sizeof(double), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    *out = std::sqrt(*out);
    return WOS_OK;
  };
  // the initial directions
  if (o->init == WOS_HISD_INIT_HESSIAN) {
    // H = Lambda_0 + A^T diag(lambda (-2 u)) A at fbar, u = A fbar + H g;
    // its k lowest eigenvectors
    if ((s = ensure_work(tb, w)) != WOS_OK) return s;
    if ((s = assemble(tb, w, nullptr, nullptr, nullptr, w.Lam0, w.Sig0, st)) != WOS_OK) return s;
    double* uu = w.vec;                 // n
    double* t2 = w.vec + w.vlen;        // n
    if ((s = reconstruct(tb, fbar, g, uu, nullptr, st)) != WOS_OK) return s;
    SHIP(launch_pointwise(n, tb->d_lambda, uu, nullptr, 0.0, -2.0, 0.0, 0.0, 0.0, t2, st));  // -2 lambda u
    SHIP(hipMemcpyAsync(w.Hess, w.Lam0, sizeof(double) * mm, hipMemcpyDeviceToDevice, st));
    SHIP(launch_gram(tb->f64, tb->d_A, n, m, t2, w.Hess, st));
    SHIP(launch_pad_copy(w.Hess, m, m, w.G, w.M, st));
    SHIP(launch_symmetrize(w.G, w.M, st));
    int sweeps = 0;
    if ((s = jacobi_eig(w, 60, &sweeps, st)) != WOS_OK) return s;
    SHIP(launch_hisd_select(w.M, m, k, w.E, w.V, Vc, st));
  } else {
    SHIP(hipMemcpyAsync(Vc, V, sizeof(double) * k * (size_t)m, hipMemcpyDeviceToDevice, st));
  }
  if ((s = orthonormalise(Vc)) != WOS_OK) return s;
  if ((s = check_bad()) != WOS_OK) return s;
  double gn = 0.0;
  const double* gr = gr0;  // grad J at the current fbar
  const double* wcur = wv;  // M^-1 of it
  if ((s = eg.eval(fbar, gr0)) != WOS_OK) return s;
  if ((s = minv(gr0, wv)) != WOS_OK) return s;
  if ((s = weighted_norm(gr, &inf.grad_norm0)) != WOS_OK) return s;
  const auto t0 = std::chrono::steady_clock::now();
  int it = 0;
  // one iteration, launched on cs
  auto iteration = [&]() -> wos_status {
    // fbar_j = fbar_{j-1} - eta R M^-1 grad J(fbar_{j-1})  (gr holds the
    // gradient, wcur its product with M^-1)
    SHIP(launch_hisd_fbar(m, k, Vc, gr, wcur, o->eta, fbar, hbuf, cs));
    // the 2k + 1 gradients at fbar_j +- h v_i and fbar_j (one pass over the
    // toolbox when batchable): H(fbar_j) v_i by central differences, and
    // grad J(fbar_j) for the next step and the checks
    SHIP(launch_hisd_shift(m, k, fbar, Vc, hbuf, Xs, cs));
    eg.st = cs;
    wos_status es = eg.eval_batch(Xs, Gs, nv, w.hsb);
    eg.st = st;
    if (es != WOS_OK) return es;
    gr = Gs + 2 * (size_t)k * m;
    // H v_i and grad J(fbar_j), then M^-1 of all k + 1 in one pass: y_i for
    // the directions, and the next step's M^-1 grad J
    SHIP(launch_hisd_hv(m, k, Gs, hbuf, HV, cs));
    if ((es = minv_batch(HV, k + 1, Yv)) != WOS_OK) return es;
    wcur = Yv + (size_t)k * m;
    SHIP(launch_hisd_v(m, k, Vc, HV, Yv, o->tau, Vn, cs));
    if ((es = orthonormalise(Vn)) != WOS_OK) return es;
    std::swap(Vc, Vn);
    return WOS_OK;
  };
  // Blocks of C iterations replayed from one captured graph, after a first
  // block launch by launch (the first iteration reads the starting
  // gradient's buffers; afterwards every pointer an iteration uses recurs
  // after two iterations, so a graph of an even number of them returns the
  // buffers to where it found them).
  const int C = o->tol > 0.0 ? check : 64;
  const bool use_graph = o->graph != 0 && C % 2 == 0 && o->max_iter >= 2 * C;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool stop = false;
  for (int j = 1; j <= o->max_iter && !stop;) {
    if (use_graph && j > C && j + C - 1 <= o->max_iter) {
      if (!exec) {
        if (!w.cap) SHIP(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
        SHIP(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal));
        cs = w.cap;
        const double* gr_s = gr;
        const double* wc_s = wcur;
        double* vc_s = Vc;
        double* vn_s = Vn;
        wos_status es = WOS_OK;
        for (int i = 0; i < C && es == WOS_OK; ++i) es = iteration();
        cs = st;
        const hipError_t ce = hipStreamEndCapture(w.cap, &graph);
        // the capture ran nothing: the state is the one before it
        gr = gr_s;
        wcur = wc_s;
        Vc = vc_s;
        Vn = vn_s;
        if (es != WOS_OK) {
          if (ce == hipSuccess && graph) (void)hipGraphDestroy(graph);
          return es;
        }
        SHIP(ce);
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
          (void)hipGraphDestroy(graph);
          SHIP(ie);
        }
      }
      const hipError_t le = hipGraphLaunch(exec, st);
      if (le != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        SHIP(le);
      }
      // the same pointers as after C launch-by-launch iterations
      gr = Gs + 2 * (size_t)k * m;
      wcur = Yv + (size_t)k * m;
      j += C;
    } else {
      if ((s = iteration()) != WOS_OK) return s;
      ++j;
    }
    it = j - 1;
    if (o->tol > 0.0 && it % check == 0) {
      if ((s = check_bad()) != WOS_OK) break;
      if ((s = weighted_norm(gr, &gn)) != WOS_OK) break;
      if (gn <= o->tol) stop = true;
    }
  }
  if (exec) {
    (void)hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
  }
  if (s != WOS_OK) return s;
  SHIP(hipStreamSynchronize(st));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  inf.iters = it;
  if ((s = check_bad()) != WOS_OK) return s;
  if ((s = weighted_norm(gr, &inf.grad_norm)) != WOS_OK) return s;
  SHIP(hipMemcpyAsync(V, Vc, sizeof(double) * k * (size_t)m, hipMemcpyDeviceToDevice, st));
  // u, grad u and J at the result
  if ((s = reconstruct(tb, fbar, g, u, grad_u ? grad_u : eg.gB, st)) != WOS_OK) return s;
  SHIP(launch_energy_weights(kind, n, d, P, tb->d_lambda, u, grad_u ? grad_u : eg.gB, f, eg.yB, F, eg.co, st));
  SHIP(launch_dot(n, F, tb->d_lambda, nullptr, red, st));
  SHIP(hipMemcpyAsync(&inf.J, red, sizeof(double), hipMemcpyDeviceToHost, st));
  SHIP(hipStreamSynchronize(st));
  if (info) *info = inf;
  return WOS_OK;
}

}  // namespace wos

extern "C" wos_status wos_saddle(wos_toolbox* tb, const wos_hisd_opts* opts, const double* f, const double* g,
                                 double* fbar, double* V, double* u, double* grad_u, wos_hisd_info* info,
                                 void* stream) {
  if (!tb) return sfail(WOS_EINVAL, "NULL argument");
  return wos::saddle_request(tb, tb->sw, opts, f, g, fbar, V, u, grad_u, info, static_cast<hipStream_t>(stream));
}

extern "C" wos_status wos_minimize(wos_toolbox* tb, const wos_adam_opts* opts, const double* f, const double* g,
                                   double* fbar, double* u, double* grad_u, wos_adam_info* info, void* stream) {
  if (!tb) return sfail(WOS_EINVAL, "NULL argument");
  return wos::minimize_request(tb, tb->sw, opts, f, g, fbar, u, grad_u, info, static_cast<hipStream_t>(stream));
}

extern "C" wos_status wos_solve(wos_toolbox* tb, const wos_coeffs* co, const double* f, const double* g,
                                double* u, double* grad_u, double* q_out, wos_solve_info* info, void* stream) {
  if (!tb) return sfail(WOS_EINVAL, "NULL argument");
  return wos::solve_request(tb, tb->sw, co, f, g, u, grad_u, q_out, info, static_cast<hipStream_t>(stream));
}
