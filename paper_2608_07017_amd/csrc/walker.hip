// The toolbox walker: Alg. "WoS-LOT" in the refined form of Rem.
// "MC_no_singular", one pass per walk building A, B, H, K at once.
//
// Launch shape: one workgroup per (site, walk-chunk) item.  The site's rows
// of A, B (d x m) and K (d x p) live in LDS as 8-byte accumulators, H's exit
// counts as 32-bit integers, so every tally is an LDS atomic; the rows are
// written to HBM once, at the end, scaled by 1/N (plain stores when one item
// covers a whole site).  The accumulators are either FP64 or exact 64-bit
// fixed point (2^-32 units, integer adds, so the sums do not depend on the
// order of the atomics): on gfx950 both are several times faster than FP32
// LDS atomics, which the tally rate would otherwise be bound by.  The
// workgroup size (256 / 512 / 1024) is the smallest that fills a CU with
// waves given the LDS each site's rows take.
//
// Lanes regenerate walks, so the long tail of walk lengths does not idle a
// wavefront.  Each lane holds its current walk and one prepared walk (draws
// made, ball-term and k = 0 tallies done).  Walks are prepared in batches,
// when at least `regen_T` lanes of the wavefront lack one (or no lane is
// walking), taking walk indices from the workgroup's counter; a lane whose
// walk stops waits, with its terminal point, for a service pass (at least
// `serve_T` such lanes) that bins the terminal points into H and K and
// starts the prepared walks.  The expensive per-walk work therefore runs on
// nearly full wavefronts and lanes rarely wait for work.
//
// Workgroups take items in the order `item_order` gives (longest expected
// work first), so the short items fill the end of the launch.
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

// Tally accumulators in LDS.
enum { kAccF64 = 0, kAccFixed = 1 };

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
// Every tally here is far below 2^31 in magnitude and the sums of a site's
// walks stay below 2^31 too.
template <>
struct Acc<kAccFixed> {
  using word = unsigned long long;
  __device__ __forceinline__ static word encode(float v) {
    const float fl = floorf(v);
    const float fr = v - fl;  // exact, in [0, 1)
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

template <typename T, int D, int KIND, bool PTS_LDS, int kBlock, int ACC>
__global__ __launch_bounds__(kBlock) void walker_kernel(WalkerParams<T> P) {
  using AW = typename Acc<ACC>::word;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned int s_next;
  __shared__ unsigned long long s_steps, s_walks, s_capped;
  __shared__ unsigned int s_maxk;

  const int item = P.item_order[blockIdx.x];
  const int site = item / P.items_per_site;
  const int chunk = item - site * P.items_per_site;
  const int64_t l_begin = (int64_t)chunk * P.walks_per_item;
  const int64_t l_end = min(P.walks, l_begin + (int64_t)P.walks_per_item);
  const int m = P.m, p = P.p;
  constexpr int PS = PtStride<D>::value;

  // LDS: the site's rows of A, B, K, the polygon edges, the site centres
  // (when they fit) and the exit counts of H.
  AW* sA = reinterpret_cast<AW*>(smem);
  AW* sB = sA + m;
  AW* sK = sB + (size_t)D * m;
  T* sSeg = reinterpret_cast<T*>(sK + (size_t)D * p);
  T* sPts = sSeg + 5 * P.nseg;
  unsigned int* sH = reinterpret_cast<unsigned int*>(sPts + (PTS_LDS ? (size_t)PS * m : 0));

  const int tid = threadIdx.x;
  for (int j = tid; j < (1 + D) * m + D * p; j += kBlock) sA[j] = AW(0);
  for (int j = tid; j < p; j += kBlock) sH[j] = 0u;
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
  const T r0 = boundary_distance<T, D, KIND>(P.dom, x, sSeg, P.nseg);
  const T d_over_r0 = T(D) / r0;
  const T r0sq = r0 * r0;

  // Per-step uniforms: Q steps per Philox block.  Every lane keeps its
  // current block and the next one; the next block is computed for all
  // lanes that need it on every Q-th iteration of the wavefront, so the
  // generator runs on full wavefronts instead of on the few lanes whose
  // block just ran out.  A lane uses at most one uniform (d = 2) or one
  // pair (d = 3) per iteration, so the next block is always ready in time.
  constexpr int Q = (D == 2) ? 4 : 2;
  constexpr int QM = Q - 1;

  // Lane state.  Besides its current walk, every lane holds one prepared
  // walk (its per-walk draws done, its ball-term and k = 0 tallies made).
  // Walks are prepared in batches, only when most lanes of the wavefront
  // need one, so the expensive per-walk work runs on nearly full
  // wavefronts; a lane whose walk stops bins its terminal point and swaps
  // in its prepared walk in a cheap service pass.
  constexpr int kIdle = 0, kActive = 1, kDone = 2;
  int state = kIdle;
  bool exhausted = false;  // the item's walk pool is used up for this lane
  T X[D], Y[D], w[D];
  T omd = T(0);
  int k = 0;
  uint32_t l = 0;
  uint4 cur = make_uint4(0u, 0u, 0u, 0u), nxt = cur;
  bool nxt_ok = false;
  int cb = 0;
  bool pvalid = false;  // prepared walk
  T pU1[D], pY[D];
  T pomd = T(0);
  uint32_t pl = 0;
  uint4 pcur = cur;
#pragma unroll
  for (int a = 0; a < D; ++a) X[a] = Y[a] = w[a] = pU1[a] = pY[a] = T(0);
  unsigned int lane_steps = 0, lane_walks = 0, lane_capped = 0, lane_maxk = 0;
  const unsigned long long lt_mask = __lanemask_lt();
  unsigned int iter = 0;

  while (true) {
    const unsigned long long act = __ballot(state == kActive);
    const unsigned long long live =
        __ballot(state != kIdle || pvalid || !exhausted);
    if (live == 0ull) break;

    // ---- prepare walks for the lanes that have none
    const unsigned long long need = __ballot(!pvalid && !exhausted);
    if (need != 0ull && (__popcll(need) >= P.regen_T || act == 0ull)) {
      const int nw = __popcll(need);
      const int leader = __ffsll((long long)need) - 1;
      unsigned int base = 0u;
      if ((int)__lane_id() == leader) base = atomicAdd(&s_next, (unsigned int)nw);
      base = __shfl(base, leader);
      if (!pvalid && !exhausted) {
        const int64_t lw = l_begin + (int64_t)base + __popcll(need & lt_mask);
        if (lw >= l_end) {
          exhausted = true;
        } else {
          // per-walk draws (counter blocks 0, 1 [, 2]) and the first step block
          pl = (uint32_t)lw;
          const uint4 b0 = philox(pl, (uint32_t)site, 0u, kTagWalk, P.k0, P.k1);
          const uint4 b1 = philox(pl, (uint32_t)site, 1u, kTagWalk, P.k0, P.k1);
          pcur = philox(pl, (uint32_t)site, (uint32_t)kStepBlock0, kTagWalk, P.k0, P.k1);
          const T u1 = u01<T>(b0.x), u2 = u01<T>(b0.y), u3 = u01<T>(b0.z);
          const T R = fmax(fmin(u1, u2), fmin(fmax(u1, u2), u3));  // median of three
          const T S = T(1) - dsqrt(u01<T>(b0.w));
          T Z[D], Zs[D];
          T om;
          if constexpr (D == 2) {
            dir2(u01<T>(b1.x), Z);
            dir2(u01<T>(b1.y), Zs);
            dir2(u01<T>(b1.z), pU1);
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
          const int4 rb = P.gv.rec[grid_cell<T, D>(P.gv, qb)];
          const int4 r0c = P.gv.rec[grid_cell<T, D>(P.gv, q0)];
          T poly = T(1) + S;
          if constexpr (D == 3) poly += S * S;
          const T bw = r0 * poly;
          const int jb = grid_resolve<T, D>(P.gv, vpts, rb, qb);
#pragma unroll
          for (int a = 0; a < D; ++a) Acc<ACC>::add(&sB[a * m + jb], bw * Zs[a]);
          const int j0 = grid_resolve<T, D>(P.gv, vpts, r0c, q0);
          Acc<ACC>::add(&sA[j0], pomd * r0sq);
          lane_steps += 1u;  // the k = 0 tally
          lane_walks += 1u;
          pvalid = true;
        }
      }
    }

    // ---- service: bin finished walks' terminal points, start prepared walks
    const unsigned long long serve = __ballot(state == kDone || (state == kIdle && pvalid));
    if (serve != 0ull && (__popcll(serve) >= P.serve_T || act == 0ull)) {
      if (state == kDone) {
        // terminal tallies (eqs. Estimator_H, Estimator_K)
        const int j = grid_nearest<T, D>(P.gg, P.gg.pts, X);
        atomicAdd(&sH[j], 1u);
#pragma unroll
        for (int a = 0; a < D; ++a) Acc<ACC>::add(&sK[a * p + j], w[a]);
        state = kIdle;
      }
      if (state == kIdle && pvalid) {
        // first step X_1 = x + r0 U1; w = (d / r0) U1
#pragma unroll
        for (int a = 0; a < D; ++a) {
          X[a] = x[a] + r0 * pU1[a];
          w[a] = d_over_r0 * pU1[a];
          Y[a] = pY[a];
        }
        omd = pomd;
        l = pl;
        cur = pcur;
        nxt_ok = false;
        cb = 0;
        k = 1;
        pvalid = false;
        state = kActive;
      }
    }

    // ---- wavefront-wide refill of the next step block
    if ((iter & QM) == 0u) {
      if (state == kActive && !nxt_ok) {
        nxt = philox(l, (uint32_t)site, (uint32_t)(kStepBlock0 + cb + 1), kTagWalk, P.k0, P.k1);
        nxt_ok = true;
      }
    }
    ++iter;

    if (state == kActive) {
      T r = boundary_distance<T, D, KIND>(P.dom, X, sSeg, P.nseg);
      bool stop;
      if (P.fixed_M > 0) {
        stop = k > P.fixed_M;
        r = fmax(r, T(0));
      } else {
        const bool near = r < P.eps;
        const bool over = k > P.max_steps;
        if (over && !near) lane_capped += 1u;
        stop = near || over;
      }
      if (stop) {
        state = kDone;
        lane_maxk = max(lane_maxk, (unsigned int)k);
      } else {
        // ---- chain tally point X_k + r Y; its cell record is loaded first and
        //      the move is computed while the load is in flight
        T q[D];
#pragma unroll
        for (int a = 0; a < D; ++a) q[a] = X[a] + r * Y[a];
        const int4 rec = P.gv.rec[grid_cell<T, D>(P.gv, q)];
        T U[D];
        const int s = (k - 1) & QM;
        if constexpr (D == 2) {
          const uint32_t word = (s == 0) ? cur.x : (s == 1) ? cur.y : (s == 2) ? cur.z : cur.w;
          dir2(u01<T>(word), U);
        } else {
          const uint32_t wa = s ? cur.z : cur.x;
          const uint32_t wb = s ? cur.w : cur.y;
          dir3(u01<T>(wa), u01<T>(wb), U);
        }
        if (s == QM) {
          cur = nxt;
          nxt_ok = false;
          cb += 1;
        }
        const T t = omd * r * r;
        // ---- A += t, B += t w at the cell of the tally point
        const int j = grid_resolve<T, D>(P.gv, vpts, rec, q);
        Acc<ACC>::add(&sA[j], t);
#pragma unroll
        for (int a = 0; a < D; ++a) Acc<ACC>::add(&sB[a * m + j], t * w[a]);
        // ---- move X_{k+1} = X_k + r U_k
#pragma unroll
        for (int a = 0; a < D; ++a) X[a] += r * U[a];
        k += 1;
        lane_steps += 1u;
      }
    }
  }

  atomicAdd(&s_steps, (unsigned long long)lane_steps);
  atomicAdd(&s_walks, (unsigned long long)lane_walks);
  if (lane_capped) atomicAdd(&s_capped, (unsigned long long)lane_capped);
  atomicMax(&s_maxk, lane_maxk);
  __syncthreads();

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
  switch (pick_block_for<T, D, KIND, PTS_LDS, ACC>(lds)) {
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

template <typename T>
hipError_t dispatch(const WalkerParams<T>& P, int dim, int kind, size_t lds, int items,
                    hipStream_t stream) {
  if (dim == 2) {
    switch (kind) {
      case WOS_BALL: return launch_typed<T, 2, WOS_BALL>(P, lds, items, stream);
      case WOS_BOX: return launch_typed<T, 2, WOS_BOX>(P, lds, items, stream);
      case WOS_POLYGON: return launch_typed<T, 2, WOS_POLYGON>(P, lds, items, stream);
      default: return hipErrorInvalidValue;
    }
  }
  switch (kind) {
    case WOS_BALL: return launch_typed<T, 3, WOS_BALL>(P, lds, items, stream);
    case WOS_BOX: return launch_typed<T, 3, WOS_BOX>(P, lds, items, stream);
    case WOS_BOX_MINUS_BALL: return launch_typed<T, 3, WOS_BOX_MINUS_BALL>(P, lds, items, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t walker_lds_bytes(int dim, int m, int p, int nseg, bool f64) {
  const size_t t = f64 ? 8 : 4;
  return 8 * ((size_t)(1 + dim) * m + (size_t)dim * p) + t * 5 * (size_t)nseg + 4 * (size_t)p;
}

// Workgroups per CU the launch can keep resident (estimate used to size
// the work split before the kernel variant is known).
int walker_block_size(size_t lds) {
  const int wgs = (int)(kLdsMax / std::max<size_t>(lds, 1));
  if (wgs >= 7) return 256;
  if (wgs >= 4) return 448;
  return 1024;
}

hipError_t launch_walker_f32(const WalkerParams<float>& P, int dim, int kind, int items,
                             hipStream_t stream) {
  return dispatch<float>(P, dim, kind, walker_lds_bytes(dim, P.m, P.p, P.nseg, false), items, stream);
}

hipError_t launch_walker_f64(const WalkerParams<double>& P, int dim, int kind, int items,
                             hipStream_t stream) {
  return dispatch<double>(P, dim, kind, walker_lds_bytes(dim, P.m, P.p, P.nseg, true), items, stream);
}

}  // namespace wos
