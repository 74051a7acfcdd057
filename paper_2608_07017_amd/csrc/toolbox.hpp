// Host-side state of a toolbox (shared by the C ABI and the solve driver).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "wos.h"

namespace wos {

// Domain description kept on the host (FP64).
struct HostDomain {
  int kind = 0, dim = 0;
  double c[3] = {0, 0, 0}, rad = 0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  std::vector<double> verts;
};

struct DevGrid {
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, h[3] = {1, 1, 1};
  int4* rec = nullptr;
  int* list = nullptr;
  float* ovf32 = nullptr;   // overflow entries (4 values each) in FP32 (index as the int's bits)
  double* ovf64 = nullptr;  // and in FP64
  size_t ncell = 0, nlist = 0;
  double frac_single = 1, mean_multi = 1;
  int max_cand = 1;
};


// Workspace of the solve path, allocated on first use and kept with the
// toolbox (sizes depend only on n, m, p, d).
struct SolveWork {
  bool ready = false;
  int n = 0, m = 0, p = 0, d = 0;  // the toolbox shape the buffers were sized for
  int M = 0;  // m rounded up to even (Jacobi pairs)
  double* R = nullptr;      // (d+1) n x (m+p) weighted rows
  double* Lam = nullptr;    // m x m
  double* Sig = nullptr;    // m x p
  double* Lam0 = nullptr;   // m x m   (Newton: A = I, b = c = 0)
  double* Sig0 = nullptr;   // m x p
  double* Hess = nullptr;   // m x m
  double* G = nullptr;      // M x M Jacobi work
  double* V = nullptr;      // M x M eigenvectors
  double* E = nullptr;      // M eigenvalues
  double* rot = nullptr;    // M
  int* pq = nullptr;        // M
  double* vec = nullptr;    // scratch vectors, 8 x max(n, M, p)
  double* Ac = nullptr;     // n x d x d (Picard coefficients)
  double* red = nullptr;    // 2 reduction slots
  size_t vlen = 0;
  // regularised solve
  double* blk = nullptr;    // 2 block vectors of (d+1) n
  double* regv = nullptr;   // the regularisation parameter (device)
  double* colp = nullptr;   // column sums of squares: kColsqChunks x m partial sums
  double* cn = nullptr;     // 2 m: exact FP64 column sums of squares (diagonals)
  int* info = nullptr;      // Cholesky status (device)
  float* R32 = nullptr;     // (d+1) n x m weighted rows, FP32
  float* Lam32 = nullptr;   // m x m
  float* N32 = nullptr;     // m x m normal matrix / its factor
  float* v32 = nullptr;     // m
  double* P64 = nullptr;    // Cholesky work (chol_work_elems(m))
  float* P32 = nullptr;
  float* L0_32 = nullptr;   // Lambda_0 (A = I), FP32, for the mixed Newton route
  uint16_t* RT = nullptr;   // BF16 route: the weighted rows W L, transposed, m x (d+1) n
  double* aj = nullptr;     // captured Adam iterations: every step size, then a block's
  size_t aj_cap = 0;        // doubles held at aj
  hipStream_t cap = nullptr;  // the stream graphs are captured on (never run on)
  double* cg = nullptr;     // BF16 route: 3 m conjugate-gradient vectors
  double* el = nullptr;     // Euler-Lagrange route: (3d + 4) n + 4 m + 2 work doubles
  double* hs = nullptr;     // p-HiSD: 78 m + 8 work doubles (+ 3 m^2 with M = A)
  size_t hs_cap = 0;        // doubles held at hs
  int* hs_bad = nullptr;    // p-HiSD: Gram-Schmidt status (device)
  double* hsb = nullptr;    // p-HiSD, batched gradients: 17 (2d + 2) n doubles
  double* part = nullptr;   // partial sums of the transposed products (gemv_part_elems)
  size_t part_cap = 0;      // doubles held at part
  bool fixed = false;       // every buffer is provided by the caller: allocate nothing
  size_t bytes = 0;         // device memory held
};

// One solve on workspace `w` (C ABI wos_solve uses the toolbox's own).
// Makes (or remakes, after a build) the toolbox's BF16 shadows on `st`.
wos_status toolbox_bf16_current(wos_toolbox* tb, hipStream_t st);

wos_status solve_request(wos_toolbox* tb, SolveWork& w, const wos_coeffs* co, const double* f, const double* g,
                         double* u, double* grad_u, double* q_out, wos_solve_info* info, hipStream_t st);
// Adam on the discrete functional J (C ABI wos_minimize).
wos_status minimize_request(wos_toolbox* tb, SolveWork& w, const wos_adam_opts* o, const double* f, const double* g,
                            double* fbar, double* u, double* grad_u, wos_adam_info* info, hipStream_t st);
// p-HiSD saddle search on J (C ABI wos_saddle).
wos_status saddle_request(wos_toolbox* tb, SolveWork& w, const wos_hisd_opts* o, const double* f, const double* g,
                          double* fbar, double* V, double* u, double* grad_u, wos_hisd_info* info, hipStream_t st);
void free_work(SolveWork& w);

}  // namespace wos

struct wos_toolbox {
  uint64_t uid = 0;  // unique per toolbox object of the process (workspace caches key on it)
  wos::SolveWork sw;
  wos::HostDomain dom;
  wos_build_opts opts{};
  int dim = 0, n = 0, m = 0, p = 0;
  bool f64 = false;
  int items_per_site = 1, walks_per_item = 1, regen_T = 48;
  int walker_block = 0;  // walker workgroup size (0: by occupancy, or tuned at the first build)
  bool autotune = false;
  int acc_fixed = 1;
  int tally_mode = WOS_TALLY_LDS_ROWS;  // wos_tally_mode in use (never AUTO)
  bool global_tally = false;  // HBM or WINDOW: tallies reach the toolbox by device atomics
  int* d_item_order = nullptr;
  // windowed mode: the items in launch order, {site, first walk, end walk,
  // 1 if the site's only item}
  int n_items = 0;
  int4* d_items = nullptr;
  // windowed tally mode: V centres and boundary nodes ranked along a Morton
  // curve (the walker's columns are ranks until the final permutation)
  int win_pc = 0, win_pb = 0;    // pages of V cells / boundary cells per site in LDS
  wos::DevGrid gv_r, gg_r;       // grids over the ranked V centres / boundary nodes
  void* d_vsites_r = nullptr;    // ranked V centres, FP32, padded
  void* d_bnodes_r = nullptr;    // ranked boundary nodes, FP32, padded
  int* d_vrank = nullptr;        // caller column j -> rank
  int* d_brank = nullptr;        // caller boundary node j -> rank
  uint16_t* d_win = nullptr;     // n x (win_pc + win_pb) page lists
  // per-site moments of the test functionals (build options test_phi, test_psi)
  bool moments = false;
  std::vector<double> test_phi, test_psi;  // host copies (m, p)
  void* d_mom_phi = nullptr;     // toolbox precision, in the walker's column numbering
  void* d_mom_psi = nullptr;
  double* d_mom = nullptr;       // n x (4 + 4 d)
  std::vector<double> sites, vsites, bnodes;  // W centres (n), V centres (m), boundary nodes (p)
  bool wv = false;  // separate V partition (else V = W and the V arrays alias the W ones)
  // device
  wos::DevGrid gv, gg;           // nearest V centre (the walker's tallies), nearest boundary node
  wos::DevGrid gw;               // nearest W centre (cell weights, evaluation off the sites)
  void* d_sites_f32 = nullptr;   // padded W centres
  void* d_sites_f64 = nullptr;
  void* d_vsites_f32 = nullptr;  // padded V centres
  void* d_vsites_f64 = nullptr;
  void* d_bnodes = nullptr;      // toolbox precision, padded
  void* d_segs = nullptr;        // toolbox precision, 5 per edge
  double* d_verts = nullptr;
  void* d_A = nullptr;
  void* d_B = nullptr;
  void* d_K = nullptr;
  void* d_H = nullptr;
  uint32_t* d_Hc = nullptr;
  unsigned long long* d_vcount = nullptr;
  unsigned long long* d_stats = nullptr;  // [0..3] walker, [4] volume inside
  unsigned long long* d_site_steps = nullptr;  // n: walk-steps of each site's walks
  double* d_lambda = nullptr;          // lambda_i = |W_i| / |D| (n)
  double* d_lambda_v = nullptr;        // |V_j| / |D| (m)
  unsigned long long* d_vcount_v = nullptr;
  size_t bytes = 0;
  hipStream_t last_stream = nullptr;
  bool built = false;
  uint64_t gen = 0;       // builds (and loads, takes) so far: what the BF16 shadows are checked against
  // BF16 shadows (bf16.hip): S_V m x (d+1) n of [B; A] and S_G p x (d+1) n of
  // [K; H], transposed (the sites' index contiguous), and their apply work
  uint16_t* d_SV = nullptr;
  uint16_t* d_SG = nullptr;
  double* d_bfy = nullptr;     // (d+1) n
  double* d_bfpart = nullptr;  // gemv_t_bf16_part_elems((d+1) n)
  uint64_t bf16_gen = 0;       // gen the shadows were made from (0: none)
  bool timing = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

