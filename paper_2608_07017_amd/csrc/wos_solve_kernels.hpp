// Launchers of the solve-path kernels (solve.hip).  All FP64 unless noted;
// `f64` selects the toolbox storage precision of toolbox operands.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace wos {

hipError_t launch_weight_rows(bool f64, const void* A, const void* B, const void* H, const void* K,
                              const double* lam, const double* Ac, const double* bc, const double* cc, int n,
                              int m, int p, int d, double* R, hipStream_t st);
// C (M x N) = alpha L^T X + beta C, L = (nblk) row blocks of n x M: blocks
// 0..nblk-2 contiguous at Lb, the last at La.
hipError_t launch_gemm_tn(bool f64, const void* Lb, const void* La, int nblk, int n, int M, const double* X,
                          int ldx, int N, double* C, int ldc, double alpha, double beta, hipStream_t st);
hipError_t launch_gemv_t(bool f64, const void* X, int rows, int cols, const double* v, double alpha, double beta,
                         double* y, hipStream_t st);
hipError_t launch_gemv_n(bool f64, const void* X, int rows, int cols, const double* v, double alpha, double beta,
                         double* y, hipStream_t st);
hipError_t launch_axpby(int n, double a, const double* x, double b, const double* y, double* z, hipStream_t st);
hipError_t launch_pointwise(int n, const double* lam, const double* u, const double* f, double c0, double c1,
                            double c2, double c3, double cf, double* out, hipStream_t st);
// C (cols x cols) += X^T diag(w) X
hipError_t launch_gram(bool f64, const void* X, int rows, int cols, const double* w, double* C, hipStream_t st);
// C = X^T X (FP64 X)
hipError_t launch_gram64(const double* X, int rows, int cols, double* C, hipStream_t st);
hipError_t launch_jacobi_round(double* G, double* V, int M, int r, double* rot, int* pq, hipStream_t st);
hipError_t launch_offnorm(const double* G, int M, double* out2, hipStream_t st);
hipError_t launch_set_identity(double* V, int M, hipStream_t st);
hipError_t launch_pad_copy(const double* src, int m, int lds, double* dst, int M, hipStream_t st);
hipError_t launch_diag(const double* G, int M, double* e, hipStream_t st);
hipError_t launch_tsvd_filter(int M, const double* e, double thr, double* z, hipStream_t st);
hipError_t launch_symmetrize(double* G, int M, hipStream_t st);
hipError_t launch_dot(int n, const double* x, const double* y, const double* w, double* out, hipStream_t st);
// Euler-Lagrange route, energy kind 0 p-Laplace, 1 minimal surface,
// 2 semilinear, 3 weighted quadratic (coefficients `co`): all site weights
// y = [lambda dF/dp; lambda dF/du] and the energy density F at a result; the weights inside the iteration (yB from
// p = gB + kg, and with uA non-NULL yA from u = uA + hg); one Adam step
// per-site coefficients of energy kind 3 (device, each NULL for 1, I, 0):
// w (n), A (n x d x d), c (n)
struct EnergyCoef {
  const double* A = nullptr;
  const double* c = nullptr;
  const double* w = nullptr;
};
hipError_t launch_energy_weights(int kind, int n, int d, double P, const double* lam, const double* u,
                                 const double* gu, const double* f, double* y, double* F, const EnergyCoef& co,
                                 hipStream_t st);
hipError_t launch_energy_wb(int kind, int n, int d, double P, const double* lam, const double* gB, const double* kg,
                            double* yB, const double* uA, const double* hg, const double* f, double* yA,
                            const EnergyCoef& co, hipStream_t st);
// the weights at nv points: point t reads GB + t d n (and UA + t n) and
// writes YB + t (d + 1) n (the B weights, then the A weights)
hipError_t launch_energy_wb_batch(int kind, int n, int d, double P, const double* lam, const double* GB,
                                  const double* kg, double* YB, const double* UA, const double* hg, const double* f,
                                  int nv, const EnergyCoef& co, hipStream_t st);
// FP32 X with 16-byte rows, nv odd in 3..17 (else hipErrorInvalidValue):
// Y[t] = X V[t] and Y[t] += X^T V[t], X read once for all nv vectors
hipError_t launch_gemv_n4_batch(const float* X, int rows, int cols, int ld, const double* V, int vs, int nv,
                                double* Y, int ys, hipStream_t st);
hipError_t launch_gemv_t4_batch(const float* X, int rows, int cols, int ld, const double* V, int vs, int nv,
                                double* Y, int ys, double* part, hipStream_t st);
// the same for any storage (FP32 rows of 16 bytes take the 4-wide kernels
// above): Y[t] = X V[t] (trans false; nv in 1..17) or Y[t] += X^T V[t]
// (trans true; nv odd in 3..17)
hipError_t launch_gemv_batch(bool f64, bool trans, const void* X, int rows, int cols, int ld, const double* V, int vs,
                             int nv, double* Y, int ys, double* part, hipStream_t st);
// The transposed products (X^T v) sum over row blocks deterministically:
// every block writes its column sums to `part`, a buffer of
// gemv_part_elems(cols, nv) doubles, and a second kernel adds the blocks in
// order.  At most kMaxRowBlocks row blocks.
constexpr int kMaxRowBlocks = 128;
size_t gemv_part_elems(int cols, int nv);
hipError_t launch_adam(int m, double* g, double b1, double b2, double eps, double aj, double* mv, double* vv,
                       double* fbar, const double* reset, hipStream_t st);
// the same with the step size read from device memory (for captured graphs)
hipError_t launch_adam_dev(int m, double* g, double b1, double b2, double eps, const double* aj, double* mv,
                           double* vv, double* fbar, const double* reset, hipStream_t st);
hipError_t launch_picard_coef(int n, int d, const double* u, double* Ac, hipStream_t st);
// out (one double slot) = max |e_i|;  count of |e_i| > thr (as an integer in the slot)
hipError_t launch_absmax(int n, const double* e, double* out, hipStream_t st);
hipError_t launch_count_above(int n, const double* e, double thr, double* out, hipStream_t st);


// ---- MFMA GEMM (mfma_gemm.hip): C = alpha op(A) op(B) + beta C, row-major
hipError_t mfma_gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                         const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st);
hipError_t mfma_gemm_f32(bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda,
                         const float* B, int ldb, float beta, float* C, int ldc, hipStream_t st);
hipError_t mfma_gemm_f64_a32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
                             const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st);
hipError_t mfma_gemm_f64_b32(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                             const float* B, int ldb, double beta, double* C, int ldc, hipStream_t st);
// the same for a square C whose upper triangle is never read (symmetric
// products): only the tiles that reach the diagonal or below are computed,
// the rest of C is left as it was
hipError_t mfma_gemm_lower_f64(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                               const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st);
hipError_t mfma_gemm_lower_f32(bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda,
                               const float* B, int ldb, float beta, float* C, int ldc, hipStream_t st);
hipError_t mfma_gemm_lower_f64_a32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
                                   const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st);

// ---- Cholesky (chol.hip): A (n x n, lda, row-major, lower part read) is
// overwritten by its factor L (lower); X (n x n, ld n) receives L^{-1}
// (zeros above the diagonal); info = first bad pivot + 1; work holds
// chol_work_elems(n) elements
size_t chol_work_elems(int n);
hipError_t cholesky_inverse_f64(double* A, int n, int lda, double* X, double* work, int* info, hipStream_t st);
hipError_t cholesky_inverse_f32(float* A, int n, int lda, float* X, float* work, int* info, hipStream_t st);

// ---- regularised solve and matrix-free operator (tikhonov.hip)
hipError_t launch_weight_rows_any(bool f64_in, bool f32_out, const void* A, const void* B, const void* H,
                                  const void* K, const double* lam, const double* Ac, const double* bc,
                                  const double* cc, int n, int m, int p, int d, int cols, void* R, hipStream_t st);
hipError_t launch_apply_w(int n, int d, const double* lam, const double* Ac, const double* bc, const double* cc,
                          const double* y, bool trans, const double* f, double* z, hipStream_t st);
// y += alpha X^T v (no scaling of y first)
hipError_t launch_gemv_t_acc(bool f64, const void* X, int rows, int cols, int ld, const double* v, double alpha,
                             double* y, double* part, hipStream_t st);
hipError_t launch_gemv_t_ld(bool f64, const void* X, int rows, int cols, int ld, const double* v, double alpha,
                            double beta, double* y, double* part, hipStream_t st);
hipError_t launch_gemv_n_ld(bool f64, const void* X, int rows, int cols, int ld, const double* v, double alpha,
                            double beta, double* y, hipStream_t st);
// Weighted column sums of squares with FP64 accumulation, deterministic:
// out[j] (+)= sum_i w[i mod wn] X[i][j]^2 (w NULL: 1); part holds
// kColsqChunks x cols doubles.
constexpr int kColsqChunks = 64;
int colsq_chunks(int rows);
hipError_t launch_colsq(bool f64, const void* X, int rows, int cols, int ld, const double* w, int wn, bool accumulate,
                        double* part, double* out, hipStream_t st);
// out = coef * max_j v[j]
hipError_t launch_reg_from_vec(const double* v, int m, double coef, double* out, hipStream_t st);
hipError_t launch_set_scalar(double* out, double v, hipStream_t st);
// x = e_j (m entries)
hipError_t launch_unit_vector(int m, int j, double* x, hipStream_t st);
// out = coef * max_i N[i][i]
hipError_t launch_reg_from_diag(bool f64, const void* N, int m, int ld, double coef, double* out, hipStream_t st);
// Y = diag(w) X (rows x cols)
hipError_t launch_scale_rows(bool f64_in, bool f32_out, const void* X, int rows, int cols, const double* w, void* Y,
                             hipStream_t st);
hipError_t launch_add_diag(bool f64, void* N, int m, int ld, const double* reg, hipStream_t st);
hipError_t launch_axpy_reg(int n, const double* x, const double* reg, double sign, const double* z, double* y,
                           hipStream_t st);
hipError_t launch_to_f32(int n, const double* x, float* y, hipStream_t st);
// ---- p-HiSD (phisd.hip): k <= 8 directions stored as V[i m + j]
hipError_t launch_hisd_fbar(int m, int k, const double* V, const double* gr, const double* w, double eta, double* fbar,
                            double* h, hipStream_t st);
hipError_t launch_hisd_shift(int m, int k, const double* fbar, const double* V, const double* h, double* X,
                             hipStream_t st);
// HV (k + 1 vectors): the k central differences, then G[2k] copied
hipError_t launch_hisd_hv(int m, int k, const double* G, const double* h, double* HV, hipStream_t st);
hipError_t launch_hisd_v(int m, int k, const double* V, const double* HV, const double* Y, double tau, double* Vn,
                         hipStream_t st);
hipError_t launch_hisd_gs(int m, int k, double* V, double* MV, int* bad, hipStream_t st);
hipError_t launch_hisd_select(int Mp, int m, int k, const double* e, const double* Evec, double* Vout,
                              hipStream_t st);
hipError_t launch_transpose_to_f64(bool f64, const void* A, int m, double* X, hipStream_t st);
hipError_t launch_identity_minus(int m, double* D, hipStream_t st);
// Y[t] = c for t < nv (m-vectors, stride m)
hipError_t launch_hisd_broadcast(int m, int nv, const double* c, double* Y, hipStream_t st);
hipError_t launch_add_f32(int n, const float* dlt, double* q, hipStream_t st);

// ---- BF16 shadows and products (bf16.hip)
// S[c][off + r] = bf16(X[r][c]), X rows x cols row-major, S leading dimension lds
hipError_t launch_shadow_t(bool f64, const void* X, int rows, int cols, uint16_t* S, size_t lds, int off,
                           hipStream_t st);
// RT = (W L)^T in BF16 from the shadow S = L^T (m x (d+1) n)
hipError_t launch_weight_t_bf16(const uint16_t* S, int n, int m, int d, const double* lam, const double* Ac,
                                const double* bc, const double* cc, uint16_t* RT, hipStream_t st);
// C (M x N, FP32) = alpha X Y^T + beta C, X (M x K), Y (N x K) BF16, k-contiguous
hipError_t gemm_nt_bf16(int M, int N, int K, float alpha, const uint16_t* X, size_t ldx, const uint16_t* Y,
                        size_t ldy, float beta, float* C, size_t ldc, hipStream_t st);
size_t gemv_t_bf16_part_elems(int K);
// y (K) = alpha S^T v + beta y, S (rows x K) BF16, deterministic order
hipError_t launch_gemv_t_bf16(const uint16_t* S, int rows, int K, size_t ld, const double* v, double alpha,
                              double beta, double* y, double* part, hipStream_t st);
hipError_t launch_split_apply(int n, int d, const double* y, double* u, double* grad_u, hipStream_t st);

}  // namespace wos
