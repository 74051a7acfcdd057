/*
 * wos.h -- C ABI of libwos, the MI355X (gfx950) Walk-on-Spheres operator
 * toolbox.
 *
 * The library builds, on one GPU, the "Laplacian Operator Toolbox" of
 * Cimpean, Grecu & Zarnescu, "Extended Walk-on-Spheres Algorithm for Linear
 * and Nonlinear Elliptic Problems of Divergence-type" (eq. LOT): for interior
 * sites x_1..x_n (the W- and V-centres, n = m) and boundary nodes
 * z_1..z_p (the Gamma-centres) of a domain D in R^d (d = 2, 3),
 *
 *   A   (n x m)     estimates U = (-Lap/2)^{-1} binned over the Voronoi
 *                   cells of the sites          (eq. Estimator_A),
 *   B   (d x n x m) estimates grad U            (eq. Estimator_B),
 *   H   (n x p)     estimates the harmonic extension binned over the
 *                   Voronoi cells of the nodes   (eq. Estimator_H),
 *   K   (d x n x p) estimates grad H            (eq. Estimator_K),
 *
 * by the one-pass walk of Alg. "WoS-LOT" in the refined form of Rem.
 * "MC_no_singular", and reduces Dirichlet problems to the system for the
 * unknown source q with u = A q + H g (eq. linear_q and the boxed
 * reconstruction of Sec. "Second order linear elliptic PDEs").
 *
 * Conventions shared by every entry point:
 *   - Every function returns a wos_status; a message for the last error of
 *     the calling thread is returned by wos_last_error().  No C++ exception
 *     crosses this interface.
 *   - Arrays are row-major and dense.  "host" pointers are read during the
 *     call only; "device" pointers must be GPU memory of the current device
 *     and stay valid until the work queued on `stream` has completed.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Functions that
 *     take a stream only queue work on it and return; the caller
 *     synchronises.  Device-side faults surface as WOS_EDEVICE from the next
 *     call that synchronises.
 *   - The caller owns every buffer it passes; a wos_toolbox owns its own
 *     device memory until wos_toolbox_free().
 */
#ifndef WOS_H
#define WOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WOS_OK = 0,
  WOS_EINVAL = -1,    /* null pointer, bad size, NaN, unsupported option      */
  WOS_EDOMAIN = -2,   /* a site outside D or at zero distance from the boundary */
  WOS_ENOMEM = -3,    /* device or host allocation failed                     */
  WOS_EDEVICE = -4,   /* a HIP call or kernel failed                          */
  WOS_ENOTCONV = -5,  /* an iteration stopped at its cap before its tolerance  */
  WOS_EBUSY = -6,
  WOS_ENOTIMPL = -7
} wos_status;

/* Domains (the distance to the boundary r(x) of eq. r and an inside test). */
typedef enum {
  WOS_BALL = 1,           /* disk (dim 2) or ball (dim 3): center, radius     */
  WOS_BOX = 2,            /* [lo, hi]                                          */
  WOS_POLYGON = 3,        /* dim 2, simple polygon, counter-clockwise vertices */
  WOS_BOX_MINUS_BALL = 4  /* dim 3: [lo, hi] minus the closed ball (center, radius) */
} wos_domain_kind;

typedef struct {
  int32_t kind;          /* wos_domain_kind                          */
  int32_t dim;           /* 2 or 3                                   */
  double center[3];
  double radius;
  double lo[3];
  double hi[3];
  int32_t nvert;         /* polygon: number of vertices, 3 .. 64     */
  const double* verts;   /* polygon: host, nvert x 2                 */
} wos_domain;

typedef enum { WOS_F32 = 0, WOS_F64 = 1 } wos_precision;

typedef struct {
  int64_t walks_per_site;   /* N >= 1 (eqs. Estimator_A..K)                      */
  double eps;               /* stop at the first k >= 1 with r(X_k) < eps; > 0
                               unless fixed_M > 0                                 */
  int32_t max_steps;        /* cap on chain tallies per walk; 0 -> 10000          */
  int32_t fixed_M;          /* > 0: the paper's rule, exactly M chain steps,
                               eps ignored                                        */
  uint64_t seed;            /* Philox4x32-10 key                                  */
  int32_t precision;        /* wos_precision of the walk arithmetic and tallies   */
  int64_t volume_samples;   /* candidate points for lambda_i; 0 -> 2^24           */
  int32_t walks_per_item;   /* walks one workgroup takes per site; 0 -> automatic */
  int32_t regen_threshold;  /* free slots of a wavefront's pool of prepared walks
                               that trigger a refill; 0 -> 48 (1 .. 64)           */
  int32_t autotune;         /* 1: the first build times the walker at each supported
                               workgroup size (256, 448, 512, 1024) on its own
                               inputs (the first 4096 work items of the launch),
                               keeps the fastest for later builds, and synchronises
                               the stream once; 0: the size is chosen by occupancy.
                               With fixed-point LDS sums the results do not depend
                               on it (with FP32 or FP64 sums, to rounding only).  */
  int32_t tally_mode;       /* where the walker sums a site's tallies (wos_tally_mode):
                               AUTO (0): LDS_ROWS when a site's rows fit in LDS
                               (about 8 (1 + dim) m + 12 dim p bytes <= 160 KiB),
                               else WINDOW for an FP32 toolbox with m, p <= 40960,
                               else HBM.
                               LDS_ROWS (1): the whole rows of A, B, H, K in LDS,
                               written to the toolbox once per work item.
                               WINDOW (2, FP32): the V cells and the boundary
                               cells are numbered along a Morton curve in pages
                               of 64; each site keeps the pages that receive
                               most of its tallies (window_pages V pages ranked
                               by an estimate of their share, window_bpages
                               nearest boundary pages) in LDS as
                               64-bit fixed-point sums (its items hold few
                               enough walks that the bound of
                               wos_build_plan.fixed_bound stays below 1/2) and
                               adds the tallies that fall elsewhere straight
                               into the toolbox (device atomics); the columns
                               are put back in the caller's order at the end of
                               the build.  AUTO takes it only when items of at
                               least 256 walks satisfy the bound.
                               HBM (3): every tally straight into the toolbox by
                               device atomics, pre-scaled by 1/N.
                               Outside LDS_ROWS the sums are in the toolbox
                               precision and their order of addition is not
                               fixed, so results agree with LDS_ROWS to rounding
                               only; in WINDOW mode ties between equidistant
                               centres go to the lower Morton rank instead of
                               the lower index.                                 */
  int32_t sampler;          /* radial law of Y (the ball-Green density, eq. density
                               Green), d = 2: WOS_SAMPLER_MEDIAN3 (0) R the median
                               of three uniforms (Beta(2,2)) with the weight
                               omega(R) = -(2/3) ln R / (1 - R) (Prop. "removing
                               singularities" (i.1), the representation the paper
                               uses); WOS_SAMPLER_LAMBERT (1) the exact law,
                               R = exp((1 + W_{-1}(-U/e)) / 2) with the lower
                               branch of the Lambert W function and weight 1 (the
                               same proposition), U the first of the same three
                               uniforms.  d = 3 supports only 0.                  */
  int32_t walker_block;     /* walker workgroup size: 0 automatic (occupancy, or the
                               autotuned size), or 256, 448, 512, 1024           */
  int32_t tally_acc;        /* LDS_ROWS accumulators of an FP32 toolbox: 0 automatic
                               (64-bit fixed point in 2^-32 units, exact integer
                               sums; a negative tally above -1 is kept to 2^-25
                               absolute, like one FP32 add near 1; unless the
                               bound of wos_build_plan.fixed_bound reaches 1/2,
                               then FP64), 1 fixed point (WOS_EINVAL when the bound
                               reaches 1/2), 2 FP64.  FP64 toolboxes always
                               accumulate in FP64; WINDOW always in fixed point
                               (2 is refused there).                             */
  int32_t window_pages;     /* WINDOW: pages of V cells per site in LDS (0: as many
                               as fit 159 KiB with the boundary pages, i.e. one
                               workgroup of 1024 lanes per compute unit)         */
  int32_t window_bpages;    /* WINDOW: pages of boundary cells per site in LDS
                               (0: min(8, all))                                  */
  const double* test_phi;   /* host, m values or NULL: a test function phi on the
                               V cells; with test_psi, switches on the per-site
                               moments (WOS_EXPORT_MOMENTS)                       */
  const double* test_psi;   /* host, p values or NULL: a test function psi on the
                               boundary cells.  When either is given, every walk
                               of site i yields the four functionals of the
                               pointwise estimators (Sec. "Monte Carlo
                               estimators": eqs. u MC, gradu U MC, H MC, dh MC)
                               with the binned data phi, psi:
                                 c_A = omega r0^2/d phi(j_0) + sum_k t_k phi(j_k)
                                 c_B = r0 (sum_{l<d} S^l) Zs phi(j_ball)
                                       + w sum_{k>=1} t_k phi(j_k)
                                 c_H = psi(j_T),   c_K = w psi(j_T)
                               (so that the means are A phi, B phi, H psi, K psi)
                               and the build sums c and c^2 per site (a NULL
                               function counts as zero).  Median-of-three
                               sampler only.                                     */
} wos_build_opts;

enum { WOS_TALLY_AUTO = 0, WOS_TALLY_LDS_ROWS = 1, WOS_TALLY_WINDOW = 2, WOS_TALLY_HBM = 3 };
enum { WOS_ACC_AUTO = 0, WOS_ACC_FIXED = 1, WOS_ACC_F64 = 2 };

/* The decisions wos_toolbox_create takes for given inputs, computed on the
 * host only (no device call), for callers that size or check a build before
 * making it.  Arguments as for wos_toolbox_create_wv (vcentres NULL: V = W).
 * fixed_bound is the largest per-item sum of |tally| that any fixed-point
 * word can receive, as a fraction of the fixed-point range 2^31: the K sums
 * are bounded by N_item d / r0 (|w| = d / r0 per walk), the B sums by
 * 4 N_item (d / r0) R^2 / d and the A sums by 4 N_item omega_max R^2 / d
 * (R the half diagonal of the bounding box, R^2 / d a bound on the mean
 * exit time, 4 a margin for its fluctuation over the item's walks,
 * omega_max = 12 the largest d = 2 weight with 24-bit uniforms, 1 in 3-D),
 * r0 the smallest distance of a site to the boundary.  In the WINDOW mode
 * each site is split by its own bound (its own r0), so sites far from the
 * boundary keep larger items than sites near it; walks_per_item is then the
 * smallest item of any site, items_per_site the most items of any site,
 * and fixed_bound the largest over the sites.                                */
typedef struct {
  int32_t tally_mode;       /* the mode used (never AUTO)                         */
  int32_t tally_acc;        /* LDS_ROWS: WOS_ACC_FIXED or WOS_ACC_F64; WINDOW:
                               WOS_ACC_FIXED                                      */
  int32_t walks_per_item;   /* walks one workgroup takes per site (WINDOW: the
                               smallest over the sites)                          */
  int32_t items_per_site;   /* (WINDOW: the most over the sites)                 */
  int32_t window_pages;     /* WINDOW: V pages per site held in LDS              */
  int32_t window_bpages;    /* WINDOW: boundary pages per site held in LDS       */
  int64_t lds_bytes;        /* LDS of one walker workgroup                        */
  double fixed_bound;       /* see above; fixed point is used only below 1/2      */
} wos_build_plan;

wos_status wos_toolbox_plan(const wos_domain* dom, const double* sites, int32_t n, const double* vcentres,
                            int32_t m, const double* bnodes, int32_t p, const wos_build_opts* opts,
                            wos_build_plan* out);

enum { WOS_SAMPLER_MEDIAN3 = 0, WOS_SAMPLER_LAMBERT = 1 };

typedef struct wos_toolbox wos_toolbox;

/* Creates a toolbox: validates the inputs, builds the nearest-centre grids
 * for the sites and the boundary nodes, and allocates the device storage.
 * Queues no walk.
 *   dom     host; sites host n x dim (double); bnodes host p x dim (double).
 *   Every site must be inside D with r(x) > 0 (else WOS_EDOMAIN).
 *   opts    host; copied.
 *   out     receives the toolbox (NULL on error).                              */
wos_status wos_toolbox_create(const wos_domain* dom, const double* sites, int32_t n,
                              const double* bnodes, int32_t p, const wos_build_opts* opts,
                              wos_toolbox** out);

/* Queues one complete toolbox build on `stream`: the cell weights lambda_i,
 * the walks of Alg. "WoS-LOT" for all (site, walk) pairs, and the
 * normalisation by N.  `seed` replaces opts.seed for this call.  Previous
 * contents are overwritten.  Asynchronous.                                      */
wos_status wos_toolbox_build(wos_toolbox* tb, uint64_t seed, void* stream);

/* create + build + synchronise: the one-call form
 * build_toolbox(domain, sites, bnodes, walks, eps, seed).                       */
wos_status wos_build_toolbox(const wos_domain* dom, const double* sites, int32_t n,
                             const double* bnodes, int32_t p, const wos_build_opts* opts,
                             void* stream, wos_toolbox** out);

typedef struct {
  int32_t dim, n, m, p, precision;
  int64_t walks_per_site;
  /* statistics of the last completed build (valid after the stream that ran
     it has been synchronised) */
  uint64_t walk_steps;      /* k = 0 tallies plus chain tallies, all walks */
  uint64_t walks;           /* walks simulated                             */
  uint64_t capped_walks;    /* walks stopped by max_steps                  */
  uint64_t max_walk_steps;  /* longest walk                                */
  uint64_t volume_inside;   /* volume points inside D                      */
  size_t device_bytes;      /* device memory held by the toolbox           */
} wos_toolbox_info;

/* As wos_toolbox_create, with a V partition of its own (the remark after
 * the definition of the partitions in Sec. "Matrix estimators": W_n and V_m
 * may be chosen independently, W discretising the image of the smoothing
 * operators and V their domain).  The walks start at the n W centres
 * `sites` (and lambda_i = |W_i| / |D| is over their cells); the tally
 * points are binned to the m V centres `vcentres` (host, m x d, inside D),
 * so A is n x m and B d x n x m; |V_j| / |D| is computed with lambda
 * (WOS_EXPORT_LAMBDA_V).  With vcentres NULL (m ignored) this is
 * wos_toolbox_create.  Supported on a toolbox with n != m: builds, apply,
 * export, take, interpolate, LINEAR solves and wos_minimize; the nonlinear
 * solve kinds and the operators return WOS_EINVAL.                          */
wos_status wos_toolbox_create_wv(const wos_domain* dom, const double* sites, int32_t n, const double* vcentres,
                                 int32_t m, const double* bnodes, int32_t p, const wos_build_opts* opts,
                                 wos_toolbox** out);

/* Fills *info.  Synchronises the toolbox's last build stream.                  */
wos_status wos_toolbox_get_info(const wos_toolbox* tb, wos_toolbox_info* info);

typedef enum {
  WOS_EXPORT_A = 0,       /* n x m,      toolbox precision             */
  WOS_EXPORT_B = 1,       /* d x n x m,  toolbox precision             */
  WOS_EXPORT_H = 2,       /* n x p,      toolbox precision (counts / N)  */
  WOS_EXPORT_K = 3,       /* d x n x p,  toolbox precision             */
  WOS_EXPORT_HCOUNT = 4,  /* n x p,      uint32 exit counts            */
  WOS_EXPORT_LAMBDA = 5,  /* n,          double lambda_i               */
  WOS_EXPORT_VCOUNT = 6,  /* n,          uint64 volume-point counts    */
  WOS_EXPORT_LAMBDA_V = 7, /* m,         double |V_j| / |D| (= lambda when V = W) */
  WOS_EXPORT_SITE_STEPS = 8, /* n,       uint64 walk-steps of each site's walks of the
                               last build (k = 0 tallies plus chain tallies)      */
  WOS_EXPORT_MOMENTS = 9,   /* n x (4 + 4d) double, with the test functions of the
                               build options: per site sum c_A, sum c_A^2,
                               sum c_B (d), sum c_B^2 (d), sum c_H, sum c_H^2,
                               sum c_K (d), sum c_K^2 (d) over its N walks; the
                               standard error of a mean is
                               sqrt((sum c^2 / N - (sum c / N)^2) / (N - 1))    */
  WOS_EXPORT_SHADOW_V = 10, /* uint16 BF16 bits, m x (d+1) n: the shadow of [B; A]
                               transposed, S_V[j][a n + i] = B^(a)_ij (a < d),
                               S_V[j][d n + i] = A_ij (rounded to nearest even)   */
  WOS_EXPORT_SHADOW_G = 11  /* uint16 BF16 bits, p x (d+1) n: the same for [K; H] */
} wos_export_what;

/* Copies one toolbox array into dst (device if dst_is_device, else host),
 * ordered on `stream`.  `bytes` must equal the array's size.  A host copy
 * synchronises the stream.                                                     */
wos_status wos_toolbox_export(const wos_toolbox* tb, int32_t what, void* dst, size_t bytes,
                              int32_t dst_is_device, void* stream);

/* Per-estimator (M, N) (Sec. "Laplacian Operator Toolbox: Pseudocode
 * algorithms": the WoS steps M and the samples N may differ between the
 * estimators A, B, H and K).  Build a second toolbox `src` on the same
 * domain, sites and boundary nodes, with its own walks, fixed_M, eps and
 * seed, then copy the estimators named in `mask` from it into `dst`:
 *   WOS_TAKE_A = 1, WOS_TAKE_B = 2, WOS_TAKE_H = 4 (with the exit counts),
 *   WOS_TAKE_K = 8.
 * Each estimator of dst is then the one of the toolbox it came from
 * (B^(j) and K^(j) move with all their components j).  Both toolboxes must
 * be built, with the same precision, dimension, domain, sites and nodes
 * (compared exactly).  Device-to-device copies ordered on `stream`.
 * Errors: WOS_EINVAL for a NULL argument, an unbuilt toolbox, a mismatch,
 * or mask outside 1..15.                                                      */
enum { WOS_TAKE_A = 1, WOS_TAKE_B = 2, WOS_TAKE_H = 4, WOS_TAKE_K = 8 };
wos_status wos_toolbox_take(wos_toolbox* dst, const wos_toolbox* src, uint32_t mask, void* stream);

/* Direct application with a known source (Sec. "Matrix estimators" and the
 * boxed reconstruction):  u = A fbar + H g,  grad_u = B fbar + K g,
 * i.e. the solution of -(1/2) Lap u = f, u = g with fbar_j = f(y_j).
 *   fbar device double (m); g device double (p); u device double (n);
 *   grad_u device double (d x n) or NULL.  Asynchronous.                        */
wos_status wos_apply(const wos_toolbox* tb, const double* fbar, const double* g, double* u,
                     double* grad_u, void* stream);

/* BF16 shadows of the built toolbox (low-precision copies kept resident for
 * the matrix cores and for bandwidth-bound applies):
 * S_V = [B; A]^T and S_G = [K; H]^T, rounded to nearest even, about
 * 2 (d+1) n (m + p) bytes on the device, made on `stream` and remade by the
 * next BF16 call after a build, load or take.  Asynchronous.                   */
wos_status wos_toolbox_make_bf16(wos_toolbox* tb, void* stream);

/* wos_apply from the BF16 shadows (made first if needed): the products read
 * BF16 operands and accumulate in FP64 in a fixed order, so the result
 * differs from wos_apply by the rounding of the toolbox to BF16 (relative
 * about 2^-9 per entry).  Uses work buffers of the toolbox: calls on one
 * toolbox must not overlap.  Asynchronous.                                      */
wos_status wos_apply_bf16(wos_toolbox* tb, const double* fbar, const double* g, double* u, double* grad_u,
                          void* stream);

/* The matrix-core product behind the BF16 route, for callers that assemble
 * their own systems from the shadows: C = alpha X Y^T + beta C with X (M x K,
 * leading dimension ldx) and Y (N x K, ldy) BF16 (uint16 bits), both
 * row-major with K contiguous, C (M x N, ldc) FP32 row-major, FP32
 * accumulation (v_mfma_f32_16x16x32_bf16).  All device pointers.  16-byte
 * loads when X, Y are 16-byte aligned and ldx, ldy are multiples of 8, else
 * element loads.  Errors: WOS_EINVAL for a NULL pointer, negative sizes or
 * leading dimensions below K (or N for C).  Asynchronous.                      */
wos_status wos_gemm_bf16_nt(int32_t M, int32_t N, int32_t K, float alpha, const uint16_t* X, int64_t ldx,
                            const uint16_t* Y, int64_t ldy, float beta, float* C, int64_t ldc, void* stream);

/* ------------------------------------------------------------- solves */
typedef enum {
  WOS_LINEAR = 0,            /* div(A grad u) + b . grad u - c u = f, u = g (eq. linearPDE) */
  WOS_SEMILINEAR_CUBIC = 1,  /* -Lap u + kappa u^3 = f, u = g: Newton on grad J = 0 for
                                F = |p|^2/2 + kappa u^4/4 - f u (eq. gradJ)             */
  WOS_QUASILINEAR = 2        /* -div((1 + u^2) grad u) = f, u = g: Picard, each iterate
                                the linear problem with A = (1 + u_k^2) I              */
} wos_problem_kind;

/* Generalised inverse of the assembled system (Sec. "Second order linear
 * elliptic PDEs" allows any, possibly regularised, generalised inverse). */
typedef enum {
  WOS_SOLVER_TSVD = 0,     /* truncated SVD: singular values <= rcond sigma_max dropped  */
  WOS_SOLVER_TIKHONOV = 1  /* Tikhonov: minimise |Lambda q - rhs|^2 + reg |q|^2 with
                              reg = rcond^2 max_j (Lambda^T Lambda)_jj, solved through
                              the Cholesky factor of the normal matrix (LINEAR only)  */
} wos_solver;

typedef enum {
  WOS_SOLVE_F64 = 0,   /* every step in FP64                                          */
  WOS_SOLVE_MIXED = 1, /* Tikhonov on an FP32 toolbox: Lambda and the normal matrix
                          formed and factored in FP32 on the matrix cores, then
                          iterative refinement with FP64 residuals of the exact
                          system (matrix-free) to refine_tol; falls back to FP64 when
                          the FP32 factorisation fails.  The regularisation
                          parameter is the FP64 route's (from exact FP64 columns
                          of Lambda, or the exact FP64 diagonal of the Newton
                          Hessian), so both routes solve the same system.       */
  WOS_SOLVE_MIXED_BF16 = 2  /* Tikhonov (LINEAR, QUASILINEAR) from the toolbox's BF16
                          shadows (made or remade as wos_toolbox_make_bf16 does):
                          Lambda assembled on the matrix cores from BF16 operands
                          (v_mfma_f32_16x16x32_bf16, FP32 accumulation), the
                          normal matrix and its Cholesky factor in FP32, then
                          preconditioned conjugate gradients on the normal
                          equations with FP64 matrix-free products of the exact
                          toolbox to refine_tol (max_refine 0 -> 50 iterations);
                          the regularisation parameter is the FP64 route's.    */
} wos_solve_precision;

typedef struct {
  int32_t kind;          /* wos_problem_kind                                        */
  const double* A;       /* LINEAR: device, n x d x d symmetric A(x_i), or NULL (= I) */
  const double* b;       /* LINEAR: device, n x d b(x_i), or NULL (= 0)               */
  const double* c;       /* LINEAR: device, n c(x_i) >= 0, or NULL (= 0)             */
  double kappa;          /* SEMILINEAR_CUBIC coefficient                            */
  double rcond;          /* truncated SVD: singular values <= rcond * sigma_max are
                            dropped; 0 -> 1e-3                                      */
  double tol;            /* Newton: |grad J| <= tol |grad J(h_0)| (0 -> 1e-8);
                            Picard: |u_{k+1} - u_k|_lambda <= tol |u_{k+1}|_lambda
                            (0 -> 1e-10)                                              */
  int32_t max_iter;      /* outer iterations; 0 -> 50 (Newton), 100 (Picard)        */
  int32_t max_sweeps;    /* Jacobi sweeps of each eigen-decomposition; 0 -> 40      */
  int32_t solver;        /* wos_solver (0: TSVD)                                    */
  int32_t precision;     /* wos_solve_precision (0: FP64)                           */
  int32_t max_refine;    /* MIXED: refinement steps at most; 0 -> 10                */
  double refine_tol;     /* MIXED: stop at |r| <= refine_tol |Lambda^T rhs|; 0 -> 1e-10 */
} wos_coeffs;

typedef struct {
  int32_t iters;          /* outer iterations taken (1 for LINEAR)               */
  int32_t rank;           /* singular values kept in the last truncated solve    */
  int32_t sweeps;         /* Jacobi sweeps of the last eigen-decomposition       */
  double sigma_max;       /* largest singular value of the last system          */
  double sigma_threshold; /* rcond * sigma_max: the truncation threshold        */
  double grad_norm;       /* Newton: final |grad J|                              */
  double grad_norm0;      /* Newton: |grad J(h_0)|                               */
  double update_norm;     /* Picard: final |u_{k+1} - u_k|_lambda                */
  double reg;             /* Tikhonov: the regularisation parameter used         */
  int32_t refine_iters;   /* MIXED: refinement steps taken                       */
  int32_t fallback;       /* MIXED: 1 when the request was solved in FP64        */
  double refine_residual; /* MIXED: final |r| / |Lambda^T rhs|                    */
  int32_t refine_converged; /* MIXED: 1 when every refinement reached refine_tol
                             (else it stopped at max_refine; the result is the
                             last iterate); 1 for FP64 solves                    */
} wos_solve_info;

/* Solves a Dirichlet problem on the toolbox's domain (Sec. "Second order
 * linear elliptic PDEs" and Sec. "Euler-Lagrange boundary value problems"):
 * assembles Lambda, Sigma and the right-hand side of eq. linear_q from the
 * toolbox and the coefficients sampled at the sites, solves it with the
 * chosen generalised inverse (coeffs->solver), and reconstructs
 * u = A q + H g, grad u = B q + K g.
 *   f       device double (n): f(x_i) in the convention of `kind`
 *   g       device double (p): g(z_j)
 *   u       device double (n) output; grad_u device (d x n) or NULL;
 *   q       device double (m) output (the unknown source) or NULL;
 *   info    host, optional.
 * Runs on `stream` and synchronises it before returning (the eigensolver
 * and the outer loops read convergence scalars on the host).  The toolbox
 * must have been built; its solve workspace (about (d+1) n (m+p) + 4 m^2
 * doubles) is allocated on the first call and kept.  Not thread-safe for
 * one toolbox.                                                               */
wos_status wos_solve(wos_toolbox* tb, const wos_coeffs* coeffs, const double* f, const double* g,
                     double* u, double* grad_u, double* q, wos_solve_info* info, void* stream);

/* wos_solve for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve, for kind LINEAR with solver TIKHONOV in FP64 only, with every work
 * buffer taken from one fixed device array of 64 MiB that the library holds
 * on each GPU it runs on until the process ends (instead of the toolbox's
 * workspace).  Arguments, results and synchronisation as for wos_solve; the
 * results are the same bits.  Calls no hipMalloc or hipFree.  The array is
 * shared by every call on one GPU and keeps the last call's contents (each
 * call writes what it reads): calls that overlap on one GPU race.  Work
 * needed: about 8 ((d+1) n m + 2 m^2 + 128 max(m, p) + 10 max(n, m, p, d n))
 * bytes plus the Cholesky work, i.e. m up to about 1100 sites in 2-D.
 * Errors: WOS_EINVAL for another kind, solver or precision (or as wos_solve);
 * WOS_ENOMEM when the work exceeds the array (nothing is launched).          */
wos_status wos_solve_noalloc(wos_toolbox* tb, const wos_coeffs* coeffs, const double* f, const double* g, double* u,
                             double* grad_u, double* q, wos_solve_info* info, void* stream);

/* Evaluation off the sites (the approximations of u on the partition after
 * eq. min_el_discrete in Sec. "Euler-Lagrange boundary value problems"):
 * each point x_k is binned to its nearest site x_i (the Voronoi cell W_i,
 * through the same grid the walks are binned by, in the toolbox
 * precision) and
 *   out[k] = u_i + <grad u_i, x_k - x_i>   with grad_u (gradient-enhanced),
 *   out[k] = u_i                            with grad_u NULL (piecewise constant).
 *   u       device double (n); grad_u device double (d x n) or NULL
 *   x       device double (npts x d), points of D; the nearest site is exact
 *           on the domain's bounding box (outside it a point is binned by
 *           the nearest grid cell)
 *   out     device double (npts); site device int32 (npts) or NULL: i
 * Asynchronous on `stream`.  Errors: WOS_EINVAL for NULL arguments or
 * npts < 0.                                                                  */
wos_status wos_interpolate(const wos_toolbox* tb, const double* u, const double* grad_u, const double* x,
                           int64_t npts, double* out, int32_t* site, void* stream);

/* ------------------------------------------ Euler-Lagrange route (Adam)
 * Minimises the discrete functional of Sec. "Euler-Lagrange boundary
 * value problems" (eq. gradJ) over the unknown source fbar,
 *   J(fbar) = sum_i lambda_i F(x_i, u_i, grad u_i),
 *   u = A fbar + H g,  grad u_i = B_i fbar + K_i g,
 * by Adam as the paper states it in its appendix on the optimisation of J
 * (m_j, v_j, the bias-corrected step alpha sqrt(1 - beta2^j) / (1 - beta1^j)),
 * with the boxed gradient
 *   grad J = A^T (lambda o dF/du) + sum_a B^(a)^T (lambda o dF/dp_a).
 * Energies:
 *   WOS_EL_PLAPLACE         F = |p|^P / P - f u (eq. plaplace), the weak
 *                           form of -div(|grad u|^(P-2) grad u) = f, u = g;
 *   WOS_EL_MINIMAL_SURFACE  F = sqrt(1 + |p|^2) - f u (the minimal surface
 *                           example, f = 0 there): the graph of least area
 *                           over D with boundary values g;
 *   WOS_EL_SEMILINEAR       F = |p|^2 / 2 - u^3 / 3 + f u (the semilinear
 *                           example): Lap u + u^2 = f, u = g.  Its dF/du
 *                           depends on u, so an iteration streams A as well
 *                           as B (twice each), and J is unbounded below:
 *                           Adam finds a local minimiser, if any, near the
 *                           start.
 *   WOS_EL_ELLIPTIC         F = w (p.A p / 2 + c u^2 / 2 - f u) (the example
 *                           "elliptic div min", w = exp(-phi)): the weak
 *                           form of -div(A grad u) + (A grad phi).grad u
 *                           + c u = f, u = g, with per-site coefficient
 *                           fields w, A, c (wos_adam_opts); an iteration
 *                           streams A and B.
 * p_exp is read for WOS_EL_PLAPLACE only.                                  */
typedef enum {
  WOS_EL_PLAPLACE = 0,
  WOS_EL_MINIMAL_SURFACE = 1,
  WOS_EL_SEMILINEAR = 2,
  WOS_EL_ELLIPTIC = 3
} wos_energy;

typedef struct {
  int32_t energy;       /* wos_energy                                         */
  double p_exp;         /* the exponent P > 1 (WOS_EL_PLAPLACE)               */
  double alpha;         /* Adam step size, > 0                                */
  double beta1;         /* in [0, 1); negative -> 0.9 (the paper's)           */
  double beta2;         /* in [0, 1); negative -> 0.999 (the paper's)         */
  double eps;           /* > 0; 0 -> 1e-10 (the paper's)                      */
  int32_t max_iter;     /* iterations at most, > 0                            */
  double tol;           /* stop once |grad J|_lambda <= tol; 0: run max_iter   */
  int32_t check_every;  /* with tol > 0, the norm is evaluated after every
                           check_every-th iteration; 0 -> 50                  */
  /* WOS_EL_ELLIPTIC: device, per site, each NULL for its default         */
  const double* coef_A; /* n x d x d, row-major (NULL: the identity)          */
  const double* coef_c; /* n (NULL: 0)                                        */
  const double* coef_w; /* n (NULL: 1)                                        */
  int32_t graph;        /* 1: the iterations between norm checks (check_every of
                           them with tol > 0, else 64) are captured once in a
                           HIP graph and replayed (one launch per block of
                           iterations instead of one per kernel); the step size
                           of each iteration is read from device memory.  The
                           results are the same bits as with 0.               */
} wos_adam_opts;

typedef struct {
  int32_t iters;        /* iterations taken                                   */
  double J;             /* J at the result                                    */
  double grad_norm;     /* |grad J|_V = (sum_j |V_j| / |D| [grad J]_j^2)^(1/2)
                           at the result                                      */
  double grad_norm0;    /* the same at the start                              */
  double seconds;       /* wall time of the iterations                        */
} wos_adam_info;

/* Runs Adam from the source in `fbar` and leaves the result there.
 *   f       device double (n): f(x_i)
 *   g       device double (p): g(z_j)
 *   fbar    device double (m): the start on entry, the result on return
 *   u       device double (n) output; grad_u device (d x n) or NULL
 *   info    host, optional.
 * Every step runs on the device (the toolbox GEMVs in FP64 accumulation,
 * the site weights and the Adam update); the host reads one scalar per
 * norm check.  Where dF/du = -f does not depend on u (p-Laplace, minimal
 * surface), A^T (lambda o f) and K g are formed once and an iteration
 * streams only B (forward and transposed); for the semilinear and elliptic
 * energies it streams A too, with H g formed once.  u and J are formed at the end.
 * Runs on `stream` and synchronises it before returning.
 * Errors: WOS_EINVAL for a NULL pointer, an unbuilt toolbox, an unknown
 * energy, P <= 1 (WOS_EL_PLAPLACE), alpha <= 0, beta >= 1, eps < 0 or
 * max_iter <= 0.  The work vectors ((3d + 4) n + 4 m doubles) are allocated
 * on the first call and kept with the toolbox.  Not thread-safe for one
 * toolbox.                                                                   */
wos_status wos_minimize(wos_toolbox* tb, const wos_adam_opts* opts, const double* f, const double* g,
                        double* fbar, double* u, double* grad_u, wos_adam_info* info, void* stream);

/* --------------------------------------------- saddle search (p-HiSD)
 * Critical points of J other than minima (the semilinear example's
 * several solutions) by preconditioned high-index saddle dynamics, as the
 * paper states it in its appendix on the optimisation of J: with k
 * directions v_1..v_k,
 *   fbar <- fbar - eta R M^-1 grad J(fbar),   R = I - 2 sum_i v_i v_i^T M,
 *   v_i  <- v_i - tau P_i M^-1 H(fbar) v_i,
 *           P_i = I - v_i v_i^T M - 2 sum_{l<i} v_l v_l^T M,
 * then V is M-orthonormalised (Gram-Schmidt in x^T M y, in the order
 * v_1..v_k).  H(fbar) v is the central difference of grad J with step
 * h = 1e-6 max(1, |fbar|_2).  M is the identity or, as the paper takes it
 * for the semilinear example, the toolbox matrix A (then n = m); its
 * inverse is formed once by the Newton-Schulz iteration X <- X + X (I - A X)
 * from X_0 = A^T / |A|_F^2 on the FP64 matrix cores.                       */
typedef enum { WOS_HISD_PRECOND_IDENTITY = 0, WOS_HISD_PRECOND_A = 1 } wos_hisd_precond;
typedef enum { WOS_HISD_INIT_GIVEN = 0, WOS_HISD_INIT_HESSIAN = 1 } wos_hisd_init;

typedef struct {
  int32_t energy;       /* wos_energy                                          */
  double p_exp;         /* P (WOS_EL_PLAPLACE)                                 */
  int32_t k;            /* the index searched for, 1..8                        */
  double eta;           /* step of fbar, > 0                                   */
  double tau;           /* step of the directions, > 0                         */
  int32_t max_iter;     /* iterations at most, > 0                             */
  double tol;           /* stop once |grad J|_V <= tol; 0: run max_iter        */
  int32_t check_every;  /* with tol > 0; 0 -> 50                               */
  int32_t precond;      /* wos_hisd_precond                                    */
  int32_t init;         /* wos_hisd_init: the caller's directions, or the
                           eigenvectors of the k smallest eigenvalues of the
                           Hessian of J at the start (the paper's choice; the
                           semilinear energy only)                            */
  int32_t graph;        /* 1: after the first block, every block of C
                           iterations (C = check_every with tol > 0, else 64;
                           C must be even, else 0 is used) is replayed from
                           one captured HIP graph; the same bits as 0         */
} wos_hisd_opts;

typedef struct {
  int32_t iters;        /* iterations taken                                    */
  double J;             /* J at the result                                     */
  double grad_norm;     /* |grad J|_V at the result                            */
  double grad_norm0;    /* the same at the start                               */
  double seconds;       /* wall time of the iterations                         */
  int32_t ns_iters;     /* Newton-Schulz iterations (WOS_HISD_PRECOND_A)       */
  double ns_residual;   /* |I - A X|_F of the inverse used                     */
} wos_hisd_info;

/* Runs p-HiSD from the source in `fbar` and leaves the result there.
 *   f, g    device double (n), (p): the data, as for wos_minimize
 *   fbar    device double (m): the start on entry, the result on return
 *   V       device double (k x m, direction i at V + i m): with
 *           WOS_HISD_INIT_GIVEN the initial directions on entry (any
 *           linearly independent set); the final directions on return
 *   u       device double (n) output; grad_u device (d x n) or NULL
 *   info    host, optional.
 * An iteration evaluates grad J at 2k + 1 points in one batched pass over
 * B (and A when dF/du depends on u), forward and transposed, and applies
 * M^-1 to k + 1 vectors in one pass over it (FP64).
 * Runs on `stream` and synchronises it before returning.
 * Errors: WOS_EINVAL for a NULL pointer, an unbuilt toolbox, an unknown
 * energy or option, WOS_EL_ELLIPTIC (a convex energy: no saddle points),
 * k outside 1..8 or above m, eta or tau <= 0, max_iter <= 0,
 * WOS_HISD_PRECOND_A with n != m or m > 16384, WOS_HISD_INIT_HESSIAN with
 * another energy than WOS_EL_SEMILINEAR, and directions that are not
 * M-independent (x^T M x not positive, or below 1e-24 of its value before
 * the Gram-Schmidt projections); WOS_ENOTCONV when the Newton-Schulz
 * inverse of A stops above |I - A X|_F = 1e-6 sqrt(m) (A too
 * ill-conditioned).  Work memory (78 m doubles, 3 m^2 more with
 * WOS_HISD_PRECOND_A, plus the solver's work for WOS_HISD_INIT_HESSIAN) is
 * kept with the toolbox and grows when a call needs more.  Not thread-safe
 * for one toolbox.                                                          */
wos_status wos_saddle(wos_toolbox* tb, const wos_hisd_opts* opts, const double* f, const double* g, double* fbar,
                      double* V, double* u, double* grad_u, wos_hisd_info* info, void* stream);

/* ---------------------------------------------------- solution operators
 * For a LINEAR problem the map from the data (f, g) to the solution is
 * linear (Sec. "Second order linear elliptic PDEs": q solves eq. linear_q,
 * whose right-hand side is -A^T (lambda o f) - Sigma g, and u = A q + H g).
 * An operator holds that map for one toolbox and one set of coefficients
 * as dense matrices,
 *   u      = U_f f + U_g g,           U = A Y [-A^T diag(lambda) | -Sigma] + [0 | H],
 *   grad u = G_f f + G_g g (optional), with B and K in place of A and H,
 * where Y = (Lambda^T Lambda + reg I)^{-1} Lambda^T is the Tikhonov inverse
 * of wos_solve (solver TIKHONOV, same rcond and reg), formed once in FP64 on
 * the matrix cores.  Each solve is then one pass over U (n x (n + p) values),
 * and a batch of solves reads U once for all of them.                        */
typedef struct wos_operator wos_operator;

typedef struct {
  int32_t want_grad;  /* 1: also hold G (d n x (n + p)) for grad u                 */
  int32_t storage;    /* wos_precision of the stored matrices: WOS_F64, or WOS_F32
                         (half the bytes per solve; products accumulate in FP64,
                         relative change of u about 1e-7)                           */
} wos_operator_opts;

typedef struct {
  int32_t n, p, dim, want_grad, storage;
  double reg;          /* Tikhonov parameter used                               */
  size_t device_bytes; /* held by the operator                                  */
  double prep_ms;      /* device time of the preparation                        */
} wos_operator_info;

/* Prepares the operator of `coeffs` (kind LINEAR, solver TIKHONOV; the
 * precision field is ignored: the preparation runs in FP64) on `stream` and
 * synchronises it.  Temporary device memory of about
 * 8 ((d+1) n (m+p) + 4 m (m+p)) bytes is allocated and freed.  The
 * coefficient arrays are read during the call only; the toolbox must stay
 * built and unchanged while the operator is used.
 *   WOS_EINVAL: NULL argument, kind not LINEAR, toolbox not built;
 *   WOS_ENOTIMPL: solver TSVD; WOS_ENOTCONV: normal matrix not positive
 *   definite; WOS_ENOMEM: device memory.                                     */
wos_status wos_operator_create(wos_toolbox* tb, const wos_coeffs* coeffs, const wos_operator_opts* opts,
                               void* stream, wos_operator** out);

/* Solves `nrhs` problems at once: for r < nrhs,
 *   u[r] = U_f f[r] + U_g g[r],  grad_u[r] = G_f f[r] + G_g g[r].
 *   f, g, u, grad_u: host arrays of nrhs device pointers to double vectors of
 *   n, p, n and d x n values (grad_u may be NULL, or hold NULL entries; it
 *   needs an operator with want_grad).  Outputs must not overlap inputs.
 * Asynchronous on `stream`; nrhs in 1 .. 1024.                               */
wos_status wos_operator_apply(const wos_operator* op, int32_t nrhs, const double* const* f,
                              const double* const* g, double* const* u, double* const* grad_u, void* stream);

wos_status wos_operator_get_info(const wos_operator* op, wos_operator_info* info);

void wos_operator_free(wos_operator* op);

/* ------------------------------------------------------------ serving
 * A request server over resident toolboxes.  Solves are queued in arrival
 * order; `slots` workers (each a host thread with its own HIP stream and
 * solve workspaces) take the next request as soon as they are free, so the
 * solves of up to `slots` requests overlap on the device (continuous
 * admission: a request that arrives while others run starts as soon as a
 * slot is free).  A request is admitted only when its workspace fits
 * `mem_budget`; workers release cached workspaces for waiting requests.
 * The result of a request does not depend on what runs beside it.
 * Toolboxes must stay built and unchanged while they have requests queued. */
typedef struct wos_server wos_server;

typedef struct {
  int32_t slots;      /* concurrent requests, 1 .. 16; 0 -> 4                  */
  size_t mem_budget;  /* device bytes for solve workspaces; 0 -> no limit     */
  int32_t max_batch;  /* operator requests solved together, 1 .. 1024; 0 -> 64 */
} wos_server_opts;

wos_status wos_server_create(const wos_server_opts* opts, wos_server** out);

/* Queues one solve (arguments as for wos_solve; device buffers must stay
 * valid until the request is polled as finished).  The coefficients struct
 * is copied.  Returns at once with a ticket.  A WOS_SOLVE_MIXED_BF16 request
 * needs the toolbox's BF16 shadows of its last build made beforehand
 * (wos_toolbox_make_bf16 and a synchronised stream), else WOS_EINVAL.        */
wos_status wos_server_submit(wos_server* sv, wos_toolbox* tb, const wos_coeffs* coeffs, const double* f,
                             const double* g, double* u, double* grad_u, uint64_t* ticket);

/* Queues one solve with a prepared operator.  Requests on the same operator
 * that are queued together are solved as one batch (one pass over the
 * operator for up to `max_batch` of them).  Buffers as for
 * wos_server_submit; the operator must outlive its requests.                */
wos_status wos_server_submit_op(wos_server* sv, const wos_operator* op, const double* f, const double* g,
                                double* u, double* grad_u, uint64_t* ticket);

/* Result of a request: WOS_EBUSY while it runs (block = 0), else its status
 * after it finished (block = 1 waits).  On completion fills *info and, if
 * times != NULL, times[0..2] = submit, start and end times in seconds (one
 * steady clock), and forgets the ticket.                                     */
wos_status wos_server_poll(wos_server* sv, uint64_t ticket, int32_t block, wos_solve_info* info,
                           double* times);

/* Requests waiting for a slot and requests not yet finished.                 */
wos_status wos_server_pending(wos_server* sv, int64_t* queued, int64_t* unfinished);

/* Finishes every queued request, then stops the workers and frees them.     */
void wos_server_destroy(wos_server* sv);

/* Kernel timing.  When enabled, wos_toolbox_build records HIP events on its
 * stream around the volume kernel, the walker kernel and the normalisation;
 * wos_toolbox_get_timings synchronises and returns their durations in
 * milliseconds for the last build (walker first).  Timing adds four event
 * records per build and is off by default.                                     */
wos_status wos_toolbox_set_timing(wos_toolbox* tb, int32_t enable);
wos_status wos_toolbox_get_timings(const wos_toolbox* tb, double* ms_walker, double* ms_volume,
                                   double* ms_finalize);

/* Storing a built toolbox for later use (the toolbox of eq. LOT is
 * precomputed once and reused with any coefficients and data).
 * wos_toolbox_save writes the toolbox's inputs (domain, centres, nodes,
 * build options), its statistics and its arrays (A, B, H, K, the exit
 * counts, lambda and the volume counts, and the V partition's volumes) to
 * `path` in a versioned binary format (little endian, tagged sections; see
 * csrc/persist.cpp); it synchronises the last build's stream.
 * wos_toolbox_load reads such a file: it creates the toolbox from the stored
 * inputs (the grids are rebuilt) and copies the stored arrays into its device
 * memory, so every export, apply and solve of the loaded toolbox gives the
 * same bits as the saved one.  Host memory for staging: 64 MiB.
 * Errors: WOS_EINVAL for NULL arguments, an unbuilt toolbox, an unreadable
 * or unwritable file, a wrong magic or version or malformed sections
 * (checked before any device allocation where the header is at fault);
 * WOS_ENOMEM, WOS_EDEVICE.                                                    */
wos_status wos_toolbox_save(const wos_toolbox* tb, const char* path);
wos_status wos_toolbox_load(const char* path, void* stream, wos_toolbox** out);

void wos_toolbox_free(wos_toolbox* tb);

/* Issue-rate probe of the vector ALU (the peak of the walker's roofline, which
 * is bound by plain lane arithmetic): every lane of 32 workgroups of 256
 * threads per compute unit runs eight independent chains of `iters`
 * instructions of one kind, timed with HIP events on `stream` (synchronised):
 *   WOS_PROBE_FMA_F32       v_fma_f32 (non-packed FP32 fused multiply-add)
 *   WOS_PROBE_ADD_U32       32-bit integer add
 *   WOS_PROBE_SIN_F32       the hardware sine (a transcendental)
 *   WOS_PROBE_MUL_U32       32-bit integer multiply (low half)
 *   WOS_PROBE_MUL_WIDE_U32  32 x 32 -> 64 multiply, both halves (as in Philox)
 * *lane_ops_per_s receives instructions x lanes per second.  Allocates and
 * frees a small device buffer.  Errors: WOS_EINVAL for an unknown op,
 * iters < 1 or NULL; WOS_EDEVICE, WOS_ENOMEM.                                  */
enum { WOS_PROBE_FMA_F32 = 0, WOS_PROBE_ADD_U32 = 1, WOS_PROBE_SIN_F32 = 2, WOS_PROBE_MUL_U32 = 3,
       WOS_PROBE_MUL_WIDE_U32 = 4 };
wos_status wos_probe_valu(int32_t op, int32_t iters, double* lane_ops_per_s, void* stream);

/* Message for the last failing call of this thread ("" if none).             */
const char* wos_last_error(void);

/* Library version string. */
const char* wos_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WOS_H */
