// The toolbox walker: Alg. "WoS-LOT" in the refined form of Rem.
// "MC_no_singular", one pass per walk building A, B, H, K at once.
//
// Launch shape: one workgroup per (site, walk-chunk) item.  The site's rows
// of A, B (d x m) and K (d x p) live in LDS as 8-byte accumulators, H's exit
// counts as 32-bit integers, so every tally is an LDS atomic; the rows are
// written to HBM once, at the end, scaled by 1/N (plain stores when one item
// covers a whole site).  The accumulators are either FP64 or 64-bit fixed
// point (2^-32 units, exact integer adds, so the sums do not depend on the
// order of the atomics): on gfx950 both are several times faster than FP32
// LDS atomics, which the tally rate would otherwise be bound by.  The
// workgroup size (256 / 448 / 512 / 1024) is chosen by occupancy, or timed
// on the first build.  When a site's rows do not fit in LDS, the windowed
// mode (`kAccWindow`) keeps the pages of cells nearest to the site (cells
// numbered along a Morton curve) in LDS, again as 64-bit fixed-point sums
// (FP32 LDS atomics are the slow kind), in one workgroup of 1024
// lanes per compute unit, and adds the tallies that fall outside them,
// pre-scaled by 1/N, straight into the toolbox with device atomics; or
// (`kAccGlobal`) every tally goes there.  The walks are the same in every
// mode.
//
// Lanes run walks back to back, so the long tail of walk lengths does not
// idle a wavefront.  The loop advances in supersteps of four chain steps.
// Walks start only at superstep boundaries, which makes the Philox block of
// the next four step draws and the word each step takes the same for every
// walking lane: the block is generated once per superstep on all walking
// lanes, and the four steps are unrolled.  Each wavefront keeps a compact
// pool of prepared walks (per-walk draws made, ball-term and k = 0 tallies
// done), one per lane slot; lanes whose walk stopped bin its terminal point
// into H and K and take walks from the top of the pool at the next
// superstep, and the pool is refilled in one pass over its free slots when
// at least `regen_T` are free.  A walk's path does not depend on where its
// tallies land, so a superstep first moves every walking lane through its
// four steps (arithmetic only), then loads the four tally points' grid
// records together (four loads in flight per lane instead of one), then
// resolves the nearest centres and adds the tallies.
//
// Workgroups take items in the order `item_order` gives (longest expected
// work first, or sites along a Morton curve per accelerator die in the
// windowed mode).
//
// This header holds the kernel template and its launch machinery; the
// instantiations are split over walker_f32_2d.hip, walker_f32_3d.hip,
// walker_f64_2d.hip and walker_f64_3d.hip so that they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "wos_device.hpp"
#include "wos_kernels.hpp"

namespace wos {

namespace {

constexpr size_t kPtsLdsMax = 32 * 1024;
constexpr size_t kLdsMax = 160 * 1024;

// Tally accumulators: FP64 or fixed point in LDS, or (rows too large for
// LDS) atomics straight to the toolbox in HBM, pre-scaled by 1/N, or the
// windowed mode: fixed-point LDS sums for the pages of cells listed for the
// site, device atomics (pre-scaled) for the cells outside them.
enum { kAccF64 = 0, kAccFixed = 1, kAccGlobal = 2, kAccWindow = 3 };
constexpr int kPageCells = 64;     // cells per page (consecutive Morton ranks)
constexpr unsigned char kNoSlot = 0xFF;

template <int ACC>
struct Acc;

template <>
struct Acc<kAccF64> {
  using word = double;
  template <typename T>
  __device__ __forceinline__ static void add(word* p, T v) {
    atomicAdd(p, (double)v);
  }
  __device__ __forceinline__ static double value(word w) { return w; }
};

// Two's-complement 64-bit fixed point, 2^-32 units: v = hi + frac with
// hi = floor(v) in the high word and floor(frac * 2^32) in the low word.
// For v >= 0 the split is exact and the word is v truncated to 2^-32.  For a
// negative v with |v| < 1, frac = 1 + v is rounded to FP32 (to 2^-24 near
// 1): the error of one FP32 add of v to a sum near 1, unbiased.  Converting
// from the float's bits instead (exact to 2^-32) costs 6 to 25 % of the
// walker's time.  The integer sums themselves are exact.  Every tally here
// is far below 2^31 in magnitude and the sums of a site's walks stay below
// 2^31 too.
template <>
struct Acc<kAccFixed> {
  using word = unsigned long long;
  __device__ __forceinline__ static word encode(float v) {
    const float fl = floorf(v);
    const float fr = v - fl;  // in [0, 1]; exact for v >= 0
    const unsigned int lo = (unsigned int)(fr * 4294967296.0f);
    const unsigned int hi = (unsigned int)(int)fl;
    return ((word)hi << 32) | lo;
  }
  __device__ __forceinline__ static word encode(double v) {
    const double fl = floor(v);
    const double fr = v - fl;
    const unsigned int lo = (unsigned int)(fr * 4294967296.0);
    const unsigned int hi = (unsigned int)(int)fl;
    return ((word)hi << 32) | lo;
  }
  template <typename T>
  __device__ __forceinline__ static void add(word* p, T v) {
    atomicAdd(p, encode(v));
  }
  __device__ __forceinline__ static double value(word w) {
    return (double)(long long)w * (1.0 / 4294967296.0);
  }
};

template <typename T, int D, int KIND>
__device__ __forceinline__ T step_distance(const WalkerParams<T>& P, const T* X, const T* seg) {
  const T r = boundary_distance<T, D, KIND>(P.dom, X, seg, P.nseg);
  return P.fixed_M > 0 ? fmax(r, T(0)) : r;
}

template <typename T, int D>
__device__ __forceinline__ int4 load_record(const GridDev<T>& g, const T* q) {
  return g.rec[(unsigned int)grid_cell<T, D>(g, q)];
}

template <>
struct Acc<kAccGlobal> {};
template <>
struct Acc<kAccWindow> {};

template <int ACC, typename T>
struct AccWord {
  using type = typename Acc<ACC>::word;
};
template <typename T>
struct AccWord<kAccGlobal, T> {
  using type = T;
};
template <typename T>
struct AccWord<kAccWindow, T> {
  using type = typename Acc<kAccFixed>::word;
};

// KIND carries the domain kind in its low four bits, in bit 4
// (kExactRadius) the d = 2 exact radial sampler and in bit 5 (kMoments) the
// per-site moments of the test functionals, so that the default kernels hold
// none of that code.
constexpr int kExactRadius = 16;
constexpr int kMoments = 32;

template <typename T, int D, int KIND, bool PTS_LDS, int kBlock, int ACC>
__global__ __launch_bounds__(kBlock) void walker_kernel(WalkerParams<T> P) {
  constexpr int GEO = KIND & 15;
  constexpr bool EXACT = D == 2 && (KIND & kExactRadius) != 0;
  constexpr bool GLOBAL = ACC == kAccGlobal;
  constexpr bool WINDOW = ACC == kAccWindow;
  constexpr bool MOM = (KIND & kMoments) != 0;
  constexpr int NMOM = 4 + 4 * D;  // sums and sums of squares of c_A, c_B (d), c_H, c_K (d)
  using AW = typename AccWord<ACC, T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned int s_next;
  __shared__ unsigned long long s_steps, s_walks, s_capped;
  __shared__ unsigned int s_maxk;

  int site;
  int64_t l_begin, l_end;
  bool sole_item;  // the site's only item: its window cells are this workgroup's alone
  if (P.items) {
    const int4 it = P.items[blockIdx.x];
    site = it.x;
    l_begin = it.y;
    l_end = it.z;
    sole_item = it.w != 0;
  } else {
    const int item = P.item_order[blockIdx.x];
    site = item / P.items_per_site;
    const int chunk = item - site * P.items_per_site;
    l_begin = (int64_t)chunk * P.walks_per_item;
    l_end = min(P.walks, l_begin + (int64_t)P.walks_per_item);
    sole_item = P.items_per_site == 1;
  }
  const int m = P.m, p = P.p;
  constexpr int PS = PtStride<D>::value;

  // LDS: the site's rows of A, B, K, the polygon edges, the site centres
  // (when they fit) and the exit counts of H.  In the global mode the rows
  // are the site's rows of the toolbox itself (row a of B, K at stride
  // n m, n p) and only the edges and centres are in LDS.  In the windowed
  // mode LDS holds the listed pages of the rows (slot (s, c) for cell
  // 64 page_s + c), the page lists and the page -> slot tables; the rows in
  // the toolbox receive the rest.
  const size_t n_sites = (size_t)P.n;
  AW *sA, *sB, *sK;
  unsigned int* sH;
  T *sSeg, *sPts;
  size_t bstride, kstride;
  // windowed mode only
  T *gA = nullptr, *gB = nullptr, *gK = nullptr;
  unsigned int* gH = nullptr;
  unsigned short* wl = nullptr;   // the site's page list (V pages, then boundary pages)
  unsigned char *tV = nullptr, *tG = nullptr;
  const int pc = P.win_pc, pb = P.win_pb;
  if constexpr (WINDOW) {
    const size_t vs = (size_t)pc * kPageCells, gs = (size_t)pb * kPageCells;
    sA = reinterpret_cast<AW*>(smem);  // 64-bit fixed-point words
    sB = sA + vs;
    sK = sB + (size_t)D * vs;
    sH = reinterpret_cast<unsigned int*>(sK + (size_t)D * gs);
    sSeg = reinterpret_cast<T*>(sH + gs);
    sPts = sSeg + 5 * P.nseg;
    wl = reinterpret_cast<unsigned short*>(sPts + (PTS_LDS ? (size_t)PS * m : 0));
    tV = reinterpret_cast<unsigned char*>(wl + pc + pb);
    tG = tV + P.npv;
    bstride = vs;
    kstride = gs;
    gA = P.A + (size_t)site * m;
    gB = P.B + (size_t)site * m;
    gK = P.K + (size_t)site * p;
    gH = P.Hc + (size_t)site * p;
  } else if constexpr (GLOBAL) {
    sA = P.A + (size_t)site * m;
    sB = P.B + (size_t)site * m;
    sK = P.K + (size_t)site * p;
    sH = P.Hc + (size_t)site * p;
    bstride = n_sites * m;
    kstride = n_sites * p;
    sSeg = reinterpret_cast<T*>(smem);
    sPts = sSeg + 5 * P.nseg;
  } else {
    sA = reinterpret_cast<AW*>(smem);
    sB = sA + m;
    sK = sB + (size_t)D * m;
    sSeg = reinterpret_cast<T*>(sK + (size_t)D * p);
    sPts = sSeg + 5 * P.nseg;
    sH = reinterpret_cast<unsigned int*>(sPts + (PTS_LDS ? (size_t)PS * m : 0));
    bstride = m;
    kstride = p;
  }
  auto add_tally = [&](AW* at, T v) {
    if constexpr (GLOBAL)
      atomicAdd(at, v * P.inv_N);
    else if constexpr (!WINDOW)
      Acc<ACC>::add(at, v);
  };
  // Tallies by cell: j a V cell (A, B) or a boundary cell (H, K).
  const size_t gbs = n_sites * m, gks = n_sites * p;  // toolbox strides of B, K rows
  auto tally_A = [&](int j, T v) {
    if constexpr (WINDOW) {
      const unsigned int sl = tV[j >> 6];
      if (sl != kNoSlot)
        lds_atomic_add(&sA[(sl << 6) | (j & 63)], Acc<kAccFixed>::encode(v));
      else
        dev_atomic_add(&gA[j], v * P.inv_N);
    } else {
      add_tally(&sA[j], v);
    }
  };
  auto tally_B = [&](int j, const T* v) {
    if constexpr (WINDOW) {
      const unsigned int sl = tV[j >> 6];
      if (sl != kNoSlot) {
        const int c = (sl << 6) | (j & 63);
#pragma unroll
        for (int a = 0; a < D; ++a) lds_atomic_add(&sB[a * bstride + c], Acc<kAccFixed>::encode(v[a]));
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) dev_atomic_add(&gB[a * gbs + j], v[a] * P.inv_N);
      }
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) add_tally(&sB[a * bstride + j], v[a]);
    }
  };
  auto tally_AB = [&](int j, T t, const T* wv) {
    if constexpr (WINDOW) {
      const unsigned int sl = tV[j >> 6];
      if (sl != kNoSlot) {
        const int c = (sl << 6) | (j & 63);
        lds_atomic_add(&sA[c], Acc<kAccFixed>::encode(t));
#pragma unroll
        for (int a = 0; a < D; ++a) lds_atomic_add(&sB[a * bstride + c], Acc<kAccFixed>::encode(t * wv[a]));
      } else {
        const T ts = t * P.inv_N;
        dev_atomic_add(&gA[j], ts);
#pragma unroll
        for (int a = 0; a < D; ++a) dev_atomic_add(&gB[a * gbs + j], ts * wv[a]);
      }
    } else {
      add_tally(&sA[j], t);
#pragma unroll
      for (int a = 0; a < D; ++a) add_tally(&sB[a * bstride + j], t * wv[a]);
    }
  };
  auto tally_HK = [&](int j, const T* wv) {
    if constexpr (WINDOW) {
      const unsigned int sl = tG[j >> 6];
      if (sl != kNoSlot) {
        const int c = (sl << 6) | (j & 63);
        lds_atomic_add(&sH[c], 1u);
#pragma unroll
        for (int a = 0; a < D; ++a) lds_atomic_add(&sK[a * kstride + c], Acc<kAccFixed>::encode(wv[a]));
      } else {
        dev_atomic_add(&gH[j], 1u);
#pragma unroll
        for (int a = 0; a < D; ++a) dev_atomic_add(&gK[a * gks + j], wv[a] * P.inv_N);
      }
    } else {
      atomicAdd(&sH[j], 1u);
#pragma unroll
      for (int a = 0; a < D; ++a) add_tally(&sK[a * kstride + j], wv[a]);
    }
  };

  const int tid = threadIdx.x;
  if constexpr (WINDOW) {
    const int cells = (pc + pb) * kPageCells;
    for (int j = tid; j < (1 + D) * pc * kPageCells + D * pb * kPageCells; j += kBlock) sA[j] = AW(0);
    for (int j = tid; j < pb * kPageCells; j += kBlock) sH[j] = 0u;
    (void)cells;
    const unsigned short* lst = P.win + (size_t)site * (pc + pb);
    for (int j = tid; j < pc + pb; j += kBlock) wl[j] = lst[j];
    for (int j = tid; j < P.npv + P.npb; j += kBlock) tV[j] = kNoSlot;
    __syncthreads();
    for (int j = tid; j < pc; j += kBlock) tV[wl[j]] = (unsigned char)j;
    for (int j = tid; j < pb; j += kBlock) tG[wl[pc + j]] = (unsigned char)j;
  } else if constexpr (!GLOBAL) {
    for (int j = tid; j < (1 + D) * m + D * p; j += kBlock) sA[j] = AW(0);
    for (int j = tid; j < p; j += kBlock) sH[j] = 0u;
  }
  for (int j = tid; j < 5 * P.nseg; j += kBlock) sSeg[j] = P.segs[j];
  if constexpr (PTS_LDS)
    for (int j = tid; j < PS * m; j += kBlock) sPts[j] = P.gv.pts[j];
  if (tid == 0) {
    s_next = 0u;
    s_steps = 0ull;
    s_walks = 0ull;
    s_capped = 0ull;
    s_maxk = 0u;
  }
  __syncthreads();
  const T* vpts = PTS_LDS ? sPts : P.gv.pts;

  T x[D];
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = P.sites[(size_t)site * PS + a];
  const T r0 = boundary_distance<T, D, GEO>(P.dom, x, sSeg, P.nseg);
  const T d_over_r0 = T(D) / r0;
  const T r0sq = r0 * r0;

  // Supersteps.  Walks start only at superstep boundaries, so at the start
  // of a superstep every walking lane is at chain step k = 1 + SS * j: the
  // Philox block of its next SS step draws and the word each step uses are
  // the same for the whole wavefront, the block is generated for all
  // walking lanes at once, and the steps of the superstep are unrolled with
  // compile-time word indices.
  constexpr int QB = (D == 2) ? 4 : 2;  // steps per Philox block
  constexpr int SS = 4;                 // steps per superstep
  constexpr int NB = SS / QB;           // blocks per superstep
  constexpr int kWave = 64;

  const int lane = (int)__lane_id();
  const unsigned long long lt_mask = __lanemask_lt();

  // Walking state of the lane: r and q are the distance at X and the tally
  // point X + r Y of the next step.
  bool active = false, done = false;
  T X[D], Y[D], w[D], q[D];
  T omd = T(0), r = T(0);
  int k = 0;
  uint32_t l = 0;
  // The wavefront's pool of prepared walks (per-walk draws made, ball-term
  // and k = 0 tallies done): slots 0 .. V-1, one per lane, consumed from the
  // top by any lane that needs a walk, refilled in one pass over the free
  // slots when at least regen_T of them are free (or a lane would starve).
  uint32_t pl = 0;
  T pU1[D], pY[D];
  T pomd = T(0);
  int V = 0;
  bool exhausted = false;
#pragma unroll
  for (int a = 0; a < D; ++a) X[a] = Y[a] = w[a] = q[a] = pU1[a] = pY[a] = T(0);
  // Moments (MOM only): per walk the test functionals' parts so far, the
  // k = 0 term phi-weighted (m0), the ball term (mb) and the chain sum
  // S = sum_{k >= 1} t_k phi(j_k); pool copies of the first two; per lane
  // the sums of c and c^2 over its finished walks.
  T pm0 = T(0), m0 = T(0), mS = T(0);
  T pmb[D], mb[D];
  double macc[NMOM];  // FP64, so that the sums do not depend on which lane ran which walk
#pragma unroll
  for (int a = 0; a < D; ++a) pmb[a] = mb[a] = T(0);
#pragma unroll
  for (int e = 0; e < NMOM; ++e) macc[e] = 0.0;
  unsigned long long n_walks = 0;  // wave-uniform
  unsigned int lane_steps = 0, lane_capped = 0, lane_maxk = 0;

  while (true) {
    const unsigned long long idle = __ballot(!active);
    const int c = __popcll(idle);

    // ---- prepare walks into the free pool slots V .. 63
    if (!exhausted && (kWave - V >= P.regen_T || c > V)) {
      const int want = kWave - V;
      unsigned int base = 0u;
      if (lane == 0) base = atomicAdd(&s_next, (unsigned int)want);
      base = __builtin_amdgcn_readfirstlane(base);
      const int64_t first = l_begin + (int64_t)base;
      const int avail = (int)max((int64_t)0, min((int64_t)want, l_end - first));
      if (avail < want) exhausted = true;
      if (lane >= V && lane < V + avail) {
        pl = (uint32_t)(first + (lane - V));
        // per-walk draws (counter blocks 0, 1 [, 2])
        const uint4 b0 = philox(pl, (uint32_t)site, 0u, kTagWalk, P.k0, P.k1);
        const uint4 b1 = philox(pl, (uint32_t)site, 1u, kTagWalk, P.k0, P.k1);
        const T u1 = u01<T>(b0.x), u2 = u01<T>(b0.y), u3 = u01<T>(b0.z);
        // median of three (Beta(2,2), reweighted by omega), or in d = 2 the
        // exact radial law from the first uniform
        T R;
        if constexpr (EXACT)
          R = radius_exact2<T>(u1);
        else
          R = fmax(fmin(u1, u2), fmin(fmax(u1, u2), u3));
        const T S = T(1) - dsqrt(u01<T>(b0.w));
        T Z[D], Zs[D];
        T om;
        if constexpr (D == 2) {
          dir2(u01<T>(b1.x), Z);
          dir2(u01<T>(b1.y), Zs);
          dir2(u01<T>(b1.z), pU1);
          if constexpr (EXACT)
            om = T(1);
          else
            om = omega2<T>(R);
        } else {
          const uint4 b2 = philox(pl, (uint32_t)site, 2u, kTagWalk, P.k0, P.k1);
          dir3(u01<T>(b1.x), u01<T>(b1.y), Z);
          dir3(u01<T>(b1.z), u01<T>(b1.w), Zs);
          dir3(u01<T>(b2.x), u01<T>(b2.y), pU1);
          om = T(1);
        }
        pomd = om / T(D);
#pragma unroll
        for (int a = 0; a < D; ++a) pY[a] = R * Z[a];
        // ball term of B: r0 * sum_{k<d} S^k * Zs at the cell of x + r0 S Zs,
        // and the k = 0 term of A: omega r0^2 / d at the cell of x + r0 Y
        T qb[D], q0[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          qb[a] = x[a] + r0 * S * Zs[a];
          q0[a] = x[a] + r0 * pY[a];
        }
        const int4 rb = load_record<T, D>(P.gv, qb);
        const int4 r0c = load_record<T, D>(P.gv, q0);
        T poly = T(1) + S;
        if constexpr (D == 3) poly += S * S;
        const T bw = r0 * poly;
        const int jb = grid_resolve<T, D>(P.gv, vpts, rb, qb);
        T bt[D];
#pragma unroll
        for (int a = 0; a < D; ++a) bt[a] = bw * Zs[a];
        tally_B(jb, bt);
        const int j0 = grid_resolve<T, D>(P.gv, vpts, r0c, q0);
        tally_A(j0, pomd * r0sq);
        if constexpr (MOM) {
          const T phb = P.mom_phi[jb];
#pragma unroll
          for (int a = 0; a < D; ++a) pmb[a] = bt[a] * phb;
          pm0 = pomd * r0sq * P.mom_phi[j0];
        }
      }
      V += avail;
      n_walks += (unsigned long long)avail;
    }

    // ---- terminal tallies of the walks that stopped (eqs. Estimator_H, _K)
    if (done) {
      const int j = grid_nearest<T, D>(P.gg, P.gg.pts, X);
      tally_HK(j, w);
      if constexpr (MOM) {
        // the walk's values of the four test functionals (eqs. u MC,
        // gradu U MC, H MC, dh MC with the binned data phi and psi)
        const double ps = (double)P.mom_psi[j];
        const double cA = (double)(m0 + mS);
        macc[0] += cA;
        macc[1] += cA * cA;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double cB = (double)(mb[a] + w[a] * mS);
          macc[2 + a] += cB;
          macc[2 + D + a] += cB * cB;
          const double cK = (double)w[a] * ps;
          macc[4 + 2 * D + a] += cK;
          macc[4 + 3 * D + a] += cK * cK;
        }
        macc[2 + 2 * D] += ps;
        macc[3 + 2 * D] += ps * ps;
      }
      done = false;
    }

    // ---- lanes without a walk take prepared walks from the top of the pool
    const int take_n = min(c, V);
    if (take_n > 0) {
      const int rk = __popcll(idle & lt_mask);
      const bool take = !active && rk < V;
      const int src = take ? (V - 1 - rk) : lane;
      const uint32_t tl = (uint32_t)__shfl((int)pl, src);
      T tU1[D], tY[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        tU1[a] = __shfl(pU1[a], src);
        tY[a] = __shfl(pY[a], src);
      }
      const T tomd = __shfl(pomd, src);
      T tm0 = T(0), tmb[D];
#pragma unroll
      for (int a = 0; a < D; ++a) tmb[a] = T(0);
      if constexpr (MOM) {
        tm0 = __shfl(pm0, src);
#pragma unroll
        for (int a = 0; a < D; ++a) tmb[a] = __shfl(pmb[a], src);
      }
      if (take) {
        if constexpr (MOM) {
          m0 = tm0;
          mS = T(0);
#pragma unroll
          for (int a = 0; a < D; ++a) mb[a] = tmb[a];
        }
        // first step X_1 = x + r0 U1; w = (d / r0) U1
#pragma unroll
        for (int a = 0; a < D; ++a) {
          X[a] = x[a] + r0 * tU1[a];
          w[a] = d_over_r0 * tU1[a];
          Y[a] = tY[a];
        }
        omd = tomd;
        l = tl;
        k = 1;
        active = true;
        r = step_distance<T, D, GEO>(P, X, sSeg);
#pragma unroll
        for (int a = 0; a < D; ++a) q[a] = X[a] + r * Y[a];
      }
      V -= take_n;
    }
    if (__ballot(active) == 0ull) break;  // pool used up and every walk binned

    // ---- the superstep's Philox blocks, for every walking lane at once
    uint4 cur[NB];
    if (active) {
      const uint32_t blk = (uint32_t)(kStepBlock0 + ((k - 1) / QB));
#pragma unroll
      for (int b = 0; b < NB; ++b) cur[b] = philox(l, (uint32_t)site, blk + (uint32_t)b, kTagWalk, P.k0, P.k1);
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) cur[b] = make_uint4(0u, 0u, 0u, 0u);
    }

    // the step cap can only be reached in this superstep by a lane already
    // within SS - 1 steps of it; otherwise the stopping test is r < eps alone
    const bool fixed = P.fixed_M > 0;
    const bool cap_near = !fixed && __ballot(active && k + (SS - 1) > P.max_steps) != 0ull;

    // Phase 1, arithmetic only: the superstep's SS moves.  A walk's path
    // does not depend on its tallies, so the tally points of all SS steps
    // (q = X_k + r_k Y), their distances and whether each is tallied are
    // known before any lookup.
    T qs[SS][D], rs[SS];
    bool ts[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) {
      bool stop;
      if (fixed) {
        stop = k > P.fixed_M;
      } else if (cap_near) {
        const bool near = r < P.eps;
        const bool over = k > P.max_steps;
        if (active && over && !near) lane_capped += 1u;
        stop = near || over;
      } else {
        stop = r < P.eps;
      }
      const bool tally = active && !stop;
      if (active && stop) {
        active = false;
        done = true;
        lane_maxk = max(lane_maxk, (unsigned int)k);
        lane_steps += (unsigned int)k;  // the k = 0 tally and k - 1 chain tallies
      }
#pragma unroll
      for (int a = 0; a < D; ++a) qs[s][a] = q[a];
      rs[s] = r;
      ts[s] = tally;
      // draw of this step: word s mod QB of block s / QB
      T U[D];
      const uint4 cb = cur[s / QB];
      if constexpr (D == 2) {
        const uint32_t word = (s % QB == 0) ? cb.x : (s % QB == 1) ? cb.y : (s % QB == 2) ? cb.z : cb.w;
        dir2(u01<T>(word), U);
      } else {
        const uint32_t wa = (s % QB == 0) ? cb.x : cb.z;
        const uint32_t wb = (s % QB == 0) ? cb.y : cb.w;
        dir3(u01<T>(wa), u01<T>(wb), U);
      }
      // X_{k+1} = X_k + r U_k, its distance and tally point
      T Xn[D];
#pragma unroll
      for (int a = 0; a < D; ++a) Xn[a] = X[a] + r * U[a];
      const T rn = step_distance<T, D, GEO>(P, Xn, sSeg);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        X[a] = tally ? Xn[a] : X[a];
        q[a] = Xn[a] + rn * Y[a];
      }
      k += tally ? 1 : 0;
      r = rn;
    }
    // Phase 2: the grid records of the SS tally points, all in flight at
    // once (every lane loads; an idle lane's cell index is clamped into the
    // grid, so the load stays in bounds).
    int4 recs[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) recs[s] = load_record<T, D>(P.gv, qs[s]);
    // Phase 3: nearest centres and tallies, A += t, B += t w at the cell of
    // X_k + r Y with t = omega r^2 / d.
#pragma unroll
    for (int s = 0; s < SS; ++s) {
      if (ts[s]) {
        const int j = grid_resolve<T, D>(P.gv, vpts, recs[s], qs[s]);
        const T t = omd * rs[s] * rs[s];
        tally_AB(j, t, w);
        if constexpr (MOM) mS += t * P.mom_phi[j];
      }
    }
  }

  if constexpr (MOM) {
    // the lanes' sums, added over the wavefront, then into the site's row
    double* mrow = P.mom + (size_t)site * NMOM;
#pragma unroll
    for (int e = 0; e < NMOM; ++e) {
      double v = macc[e];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0 && v != 0.0) atomicAdd(&mrow[e], v);
    }
  }
  if (lane == 0) atomicAdd(&s_walks, n_walks);
  atomicAdd(&s_steps, (unsigned long long)lane_steps);
  if (lane_capped) atomicAdd(&s_capped, (unsigned long long)lane_capped);
  atomicMax(&s_maxk, lane_maxk);
  __syncthreads();

  if constexpr (GLOBAL || WINDOW) {
    if constexpr (WINDOW) {
      // the window's sums, scaled by 1/N, onto the toolbox rows: plain
      // stores when this is the site's only item (no other workgroup writes
      // the window's cells of this row, and the device atomics of this one
      // go to other cells), else device atomics
      const double inv_N = (double)P.inv_N;
      for (int c = tid; c < pc * kPageCells; c += kBlock) {
        const int j = ((int)wl[c >> 6] << 6) | (c & 63);
        if (j < m) {
          const AW va = sA[c];
          const T ta = (T)(Acc<kAccFixed>::value(va) * inv_N);
          if (sole_item)
            gA[j] = ta;
          else if (va != AW(0))
            dev_atomic_add(&gA[j], ta);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const AW vb = sB[a * bstride + c];
            const T tb = (T)(Acc<kAccFixed>::value(vb) * inv_N);
            if (sole_item)
              gB[a * gbs + j] = tb;
            else if (vb != AW(0))
              dev_atomic_add(&gB[a * gbs + j], tb);
          }
        }
      }
      for (int c = tid; c < pb * kPageCells; c += kBlock) {
        const int j = ((int)wl[pc + (c >> 6)] << 6) | (c & 63);
        if (j < p) {
          const unsigned int h = sH[c];
          if (sole_item)
            gH[j] = h;
          else if (h)
            dev_atomic_add(&gH[j], h);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const AW vk = sK[a * kstride + c];
            const T tk = (T)(Acc<kAccFixed>::value(vk) * inv_N);
            if (sole_item)
              gK[a * gks + j] = tk;
            else if (vk != AW(0))
              dev_atomic_add(&gK[a * gks + j], tk);
          }
        }
      }
    }
    if (tid == 0) {
      atomicAdd(&P.stats[0], s_steps);
      atomicAdd(&P.stats[1], s_walks);
      atomicAdd(&P.stats[2], s_capped);
      atomicMax(&P.stats[3], (unsigned long long)s_maxk);
      atomicAdd(&P.site_steps[site], s_steps);
    }
    return;
  } else {
  // ---- flush the site's rows, scaled by 1/N
  const double inv_N = (double)P.inv_N;
  const size_t n = (size_t)P.n;
  T* gA = P.A + (size_t)site * m;
  unsigned int* gH = P.Hc + (size_t)site * p;
  if (P.direct_store) {
    for (int j = tid; j < m; j += kBlock) gA[j] = (T)(Acc<ACC>::value(sA[j]) * inv_N);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T* gB = P.B + (size_t)a * n * m + (size_t)site * m;
      for (int j = tid; j < m; j += kBlock) gB[j] = (T)(Acc<ACC>::value(sB[a * m + j]) * inv_N);
      T* gK = P.K + (size_t)a * n * p + (size_t)site * p;
      for (int j = tid; j < p; j += kBlock) gK[j] = (T)(Acc<ACC>::value(sK[a * p + j]) * inv_N);
    }
    for (int j = tid; j < p; j += kBlock) gH[j] = sH[j];
  } else {
    for (int j = tid; j < m; j += kBlock) {
      const double v = Acc<ACC>::value(sA[j]);
      if (v != 0.0) atomicAdd(&gA[j], (T)(v * inv_N));
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T* gB = P.B + (size_t)a * n * m + (size_t)site * m;
      for (int j = tid; j < m; j += kBlock) {
        const double v = Acc<ACC>::value(sB[a * m + j]);
        if (v != 0.0) atomicAdd(&gB[j], (T)(v * inv_N));
      }
      T* gK = P.K + (size_t)a * n * p + (size_t)site * p;
      for (int j = tid; j < p; j += kBlock) {
        const double v = Acc<ACC>::value(sK[a * p + j]);
        if (v != 0.0) atomicAdd(&gK[j], (T)(v * inv_N));
      }
    }
    for (int j = tid; j < p; j += kBlock) {
      const unsigned int v = sH[j];
      if (v) atomicAdd(&gH[j], v);
    }
  }
  if (tid == 0) {
    atomicAdd(&P.stats[0], s_steps);
    atomicAdd(&P.stats[1], s_walks);
    atomicAdd(&P.stats[2], s_capped);
    atomicMax(&P.stats[3], (unsigned long long)s_maxk);
    atomicAdd(&P.site_steps[site], s_steps);
  }
  }
}

template <typename T, int D, int KIND, bool PTS_LDS, int BS, int ACC>
hipError_t launch_variant(const WalkerParams<T>& P, size_t lds, int items, hipStream_t stream) {
  auto kern = walker_kernel<T, D, KIND, PTS_LDS, BS, ACC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(items), dim3(BS), lds, stream, P);
  return hipGetLastError();
}

// The workgroup size that keeps the most waves resident per CU given the
// kernel's registers and the LDS one workgroup takes (the smallest on ties),
// from the runtime's occupancy calculator; cached per kernel and LDS size.
template <typename K>
int resident_waves(K kern, int bs, size_t lds) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(kern), bs, lds) !=
      hipSuccess)
    return 0;
  return blocks * (bs / 64);
}

template <typename T, int D, int KIND, bool PTS_LDS, int ACC>
int pick_block_for(size_t lds) {
  static std::mutex mu;
  static std::map<size_t, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(lds);
  if (it != cache.end()) return it->second;
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(walker_kernel<T, D, KIND, PTS_LDS, 256, ACC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(walker_kernel<T, D, KIND, PTS_LDS, 448, ACC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(walker_kernel<T, D, KIND, PTS_LDS, 512, ACC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(walker_kernel<T, D, KIND, PTS_LDS, 1024, ACC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  const int w256 = resident_waves(walker_kernel<T, D, KIND, PTS_LDS, 256, ACC>, 256, lds);
  const int w448 = resident_waves(walker_kernel<T, D, KIND, PTS_LDS, 448, ACC>, 448, lds);
  const int w512 = resident_waves(walker_kernel<T, D, KIND, PTS_LDS, 512, ACC>, 512, lds);
  const int w1024 = resident_waves(walker_kernel<T, D, KIND, PTS_LDS, 1024, ACC>, 1024, lds);
  int bs = 256, best = w256;
  if (w448 > best) bs = 448, best = w448;
  if (w512 > best) bs = 512, best = w512;
  if (w1024 > best) bs = 1024, best = w1024;
  cache[lds] = bs;
  return bs;
}

template <typename T, int D, int KIND, bool PTS_LDS, int ACC>
hipError_t launch_bs(const WalkerParams<T>& P, size_t lds, int items, hipStream_t stream) {
  int bs = P.block_override;
  if (bs != 256 && bs != 448 && bs != 512 && bs != 1024) bs = pick_block_for<T, D, KIND, PTS_LDS, ACC>(lds);
  switch (bs) {
    case 256: return launch_variant<T, D, KIND, PTS_LDS, 256, ACC>(P, lds, items, stream);
    case 448: return launch_variant<T, D, KIND, PTS_LDS, 448, ACC>(P, lds, items, stream);
    case 512: return launch_variant<T, D, KIND, PTS_LDS, 512, ACC>(P, lds, items, stream);
    default: return launch_variant<T, D, KIND, PTS_LDS, 1024, ACC>(P, lds, items, stream);
  }
}

// Site centres are copied to LDS when they fit beside the rows.
template <typename T, int D, int KIND>
hipError_t launch_typed(const WalkerParams<T>& P, size_t lds, int items, hipStream_t stream) {
  const size_t pts = sizeof(T) * PtStride<D>::value * (size_t)P.m;
  if constexpr (std::is_same<T, float>::value) {
    if (P.window) {
      const size_t lds_w = walker_window_lds_bytes(D, P.win_pc, P.win_pb, P.npv, P.npb, P.nseg);
      if (pts <= kPtsLdsMax && lds_w + pts <= kLdsMax)
        return launch_bs<T, D, KIND, true, kAccWindow>(P, lds_w + pts, items, stream);
      return launch_bs<T, D, KIND, false, kAccWindow>(P, lds_w, items, stream);
    }
  }
  if (P.global_tally) {
    const size_t lds_g = sizeof(T) * 5 * (size_t)P.nseg;
    if (pts <= kPtsLdsMax) return launch_bs<T, D, KIND, true, kAccGlobal>(P, lds_g + pts, items, stream);
    return launch_bs<T, D, KIND, false, kAccGlobal>(P, lds_g, items, stream);
  }
  const bool pts_lds = pts <= kPtsLdsMax && lds + pts <= kLdsMax;
  if constexpr (std::is_same<T, float>::value) {
    if (P.acc_fixed) {
      if (pts_lds) return launch_bs<T, D, KIND, true, kAccFixed>(P, lds + pts, items, stream);
      return launch_bs<T, D, KIND, false, kAccFixed>(P, lds, items, stream);
    }
  }
  if (pts_lds) return launch_bs<T, D, KIND, true, kAccF64>(P, lds + pts, items, stream);
  return launch_bs<T, D, KIND, false, kAccF64>(P, lds, items, stream);
}

}  // namespace

}  // namespace wos
