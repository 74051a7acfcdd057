// Plain structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "wos.h"

namespace wos {

constexpr int kMaxPolyVerts = 64;
constexpr int kStepBlock0 = 4;      // first Philox block of the per-step draws
constexpr uint32_t kTagWalk = 0;
constexpr uint32_t kTagVolume = 1;
constexpr int kDefaultMaxSteps = 10000;

template <int D>
struct PtStride {
  static constexpr int value = (D == 2) ? 2 : 4;  // 3-D centres padded to 16 B
};

template <typename T>
struct DomainDev {
  int kind;
  int dim;
  T c[3];
  T rad;
  T lo[3];
  T hi[3];
};

template <typename T>
struct GridDev {
  int n[3];
  T lo[3];
  T inv_h[3];
  T top[3];         // n[a] - 1
  const int4* rec;  // n0*n1*n2 cell records, x slowest
  const int* list;  // overflow lists [count, indices...]
  const T* ovf;     // overflow entries, 4 values each: the centre (padded to
                    // three coordinates) and its index (FP32: the int's bits)
  const T* pts;     // centres, PtStride<D> values each
};

template <typename T>
struct WalkerParams {
  DomainDev<T> dom;
  const T* segs;   // polygon edges, 5 values each
  int nseg;
  const T* sites;  // n centres, padded stride
  GridDev<T> gv;   // nearest site
  GridDev<T> gg;   // nearest boundary node
  int n, m, p;
  int64_t walks;
  int walks_per_item;
  int items_per_site;
  T eps;
  int max_steps;
  int fixed_M;
  uint32_t k0, k1;
  T inv_N;
  int regen_T;     // refill a wavefront's pool of prepared walks when this many slots are free
  int block_override;  // workgroup size chosen by the caller (0: by occupancy)
  int global_tally;    // tallies by atomics to the toolbox in HBM (rows too large for LDS)
  int exact_radius;    // d = 2: R from the exact radial law (Lambert W), weight 1
  const int* item_order;  // blockIdx -> item (longest expected work first)
  // windowed mode: blockIdx -> {site, first walk, end walk, 1 if the site's
  // only item} (each site split by its own fixed-point bound); NULL: items
  // of items_per_site x walks_per_item through item_order
  const int4* items;
  int direct_store;
  int acc_fixed;   // tally accumulators: 0 FP64, 1 64-bit fixed point
  int window;      // windowed tallies: columns are Morton ranks, pages listed per site
  const uint16_t* win;  // n x (win_pc + win_pb): a site's V pages, then its boundary pages
  int win_pc, win_pb;   // pages held in LDS per site
  int npv, npb;         // pages of the ranked V centres / boundary nodes
  T* A;
  T* B;
  uint32_t* Hc;
  T* K;
  unsigned long long* stats;  // [0] walk-steps, [1] walks, [2] capped, [3] max walk-steps
  unsigned long long* site_steps;  // n: walk-steps of each site's walks
  const T* mom_phi;  // moments: the test function on the V cells (walker's column numbering), or NULL
  const T* mom_psi;  // moments: the test function on the boundary cells (walker's numbering)
  double* mom;       // moments: n x (4 + 4 d) sums, NULL when off
};

struct VolumeParams {
  DomainDev<double> dom;  // lo/hi hold the bounding box the points are drawn in
  const double* verts;  // polygon vertices, 2 per vertex
  int nvert;
  GridDev<double> gv;
  int n;
  int dim;
  int64_t npoints;      // candidate points: per_tile * tiles^dim
  int64_t nblocks;      // Philox blocks
  int tile_shift;       // log2(tiles per axis of the bounding box)
  int point_shift;      // log2(points per tile)
  double inv_tiles;     // 1 / tiles
  uint32_t k0, k1;
  unsigned long long* counts;  // n
  unsigned long long* inside;  // 1
};

}  // namespace wos
