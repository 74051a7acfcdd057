// The toolbox walker: Alg. "WoS-LOT" in the refined form of Rem.
// "MC_no_singular", one pass per walk building A, B, H, K at once.
//
// Launch shape: one 256-lane workgroup per (site, walk-chunk) item.  The
// site's rows of A, B (d x m) and H, K (p, d x p) live in LDS for the whole
// item, so every tally is an LDS atomic; the rows are added to HBM once, at
// the end, scaled by 1/N (plain stores when one item covers a whole site).
//
// Lanes regenerate walks: a lane whose walk has stopped waits, with its
// terminal point, until the number of such lanes in its wavefront reaches
// `regen_T` (or no lane is walking); then those lanes bin their terminal
// points into H and K, take new walk indices from the workgroup's counter,
// draw their per-walk variables and make the ball-term and k = 0 tallies
// together.  The per-walk work therefore runs on mostly full wavefronts while
// the step loop keeps most lanes busy despite the long tail of walk lengths.
#include <hip/hip_runtime.h>

#include "wos_device.hpp"
#include "wos_kernels.hpp"

namespace wos {

namespace {

constexpr int kBlock = 256;

template <typename T, int D, int KIND>
__global__ __launch_bounds__(kBlock) void walker_kernel(WalkerParams<T> P) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned int s_next;
  __shared__ unsigned long long s_steps, s_walks, s_capped;
  __shared__ unsigned int s_maxk;

  const int item = blockIdx.x;
  const int site = item / P.items_per_site;
  const int chunk = item - site * P.items_per_site;
  const int64_t l_begin = (int64_t)chunk * P.walks_per_item;
  const int64_t l_end = min(P.walks, l_begin + (int64_t)P.walks_per_item);
  const int m = P.m, p = P.p;

  T* sA = reinterpret_cast<T*>(smem);
  T* sB = sA + m;
  T* sK = sB + (size_t)D * m;
  T* sSeg = sK + (size_t)D * p;
  unsigned int* sH = reinterpret_cast<unsigned int*>(sSeg + 5 * P.nseg);

  const int tid = threadIdx.x;
  for (int j = tid; j < (1 + D) * m + D * p; j += kBlock) sA[j] = T(0);
  for (int j = tid; j < p; j += kBlock) sH[j] = 0u;
  for (int j = tid; j < 5 * P.nseg; j += kBlock) sSeg[j] = P.segs[j];
  if (tid == 0) {
    s_next = 0u;
    s_steps = 0ull;
    s_walks = 0ull;
    s_capped = 0ull;
    s_maxk = 0u;
  }
  __syncthreads();

  T x[D];
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = P.sites[(size_t)site * PtStride<D>::value + a];
  const T r0 = boundary_distance<T, D, KIND>(P.dom, x, sSeg, P.nseg);
  const T d_over_r0 = T(D) / r0;
  const T r0sq = r0 * r0;

  // lane state
  constexpr int kIdle = 0, kActive = 1, kDone = 2;
  int state = kIdle;
  bool retired = false;
  T X[D], Y[D], w[D];
  T omd = T(0);
  int k = 0;
  uint32_t l = 0;
  uint4 sb = make_uint4(0u, 0u, 0u, 0u);
  unsigned int lane_steps = 0, lane_walks = 0, lane_capped = 0, lane_maxk = 0;
  const unsigned long long lt_mask = __lanemask_lt();

  while (true) {
    const unsigned long long act = __ballot(state == kActive);
    const unsigned long long pend = __ballot(state != kActive && !retired);
    if (act == 0ull && pend == 0ull) break;

    if (act == 0ull || __popcll(pend) >= P.regen_T) {
      // ---- terminal tallies of finished walks (eqs. Estimator_H, K)
      if (state == kDone) {
        const int j = grid_nearest<T, D>(P.gg, X);
        atomicAdd(&sH[j], 1u);
#pragma unroll
        for (int a = 0; a < D; ++a) atomicAdd(&sK[a * p + j], w[a]);
        state = kIdle;
      }
      // ---- take new walk indices, one LDS atomic per wavefront
      const unsigned long long want = __ballot(state == kIdle && !retired);
      const int nw = __popcll(want);
      unsigned int base = 0u;
      if (nw > 0) {
        const int leader = __ffsll((long long)want) - 1;
        if ((int)__lane_id() == leader) base = atomicAdd(&s_next, (unsigned int)nw);
        base = __shfl(base, leader);
      }
      if (state == kIdle && !retired) {
        const int64_t lw = l_begin + (int64_t)base + __popcll(want & lt_mask);
        if (lw >= l_end) {
          retired = true;
        } else {
          // ---- per-walk draws (counter block 0, 1 [, 2])
          l = (uint32_t)lw;
          const uint4 b0 = philox(l, (uint32_t)site, 0u, kTagWalk, P.k0, P.k1);
          const uint4 b1 = philox(l, (uint32_t)site, 1u, kTagWalk, P.k0, P.k1);
          const T u1 = u01<T>(b0.x), u2 = u01<T>(b0.y), u3 = u01<T>(b0.z);
          const T R = fmax(fmin(u1, u2), fmin(fmax(u1, u2), u3));  // median of three
          const T S = T(1) - dsqrt(u01<T>(b0.w));
          T Z[D], Zs[D], U1[D];
          T om;
          if constexpr (D == 2) {
            dir2(u01<T>(b1.x), Z);
            dir2(u01<T>(b1.y), Zs);
            dir2(u01<T>(b1.z), U1);
            om = omega2<T>(R);
          } else {
            const uint4 b2 = philox(l, (uint32_t)site, 2u, kTagWalk, P.k0, P.k1);
            dir3(u01<T>(b1.x), u01<T>(b1.y), Z);
            dir3(u01<T>(b1.z), u01<T>(b1.w), Zs);
            dir3(u01<T>(b2.x), u01<T>(b2.y), U1);
            om = T(1);
          }
          omd = om / T(D);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            Y[a] = R * Z[a];
            w[a] = d_over_r0 * U1[a];
          }
          // ---- ball term of B: r0 * sum_{k<d} S^k * Zs at the cell of x + r0 S Zs
          {
            T q[D];
#pragma unroll
            for (int a = 0; a < D; ++a) q[a] = x[a] + r0 * S * Zs[a];
            const int j = grid_nearest<T, D>(P.gv, q);
            T poly = T(1) + S;
            if constexpr (D == 3) poly += S * S;
            const T bw = r0 * poly;
#pragma unroll
            for (int a = 0; a < D; ++a) atomicAdd(&sB[a * m + j], bw * Zs[a]);
          }
          // ---- k = 0 term of A: omega r0^2 / d at the cell of x + r0 Y
          {
            T q[D];
#pragma unroll
            for (int a = 0; a < D; ++a) q[a] = x[a] + r0 * Y[a];
            const int j = grid_nearest<T, D>(P.gv, q);
            atomicAdd(&sA[j], omd * r0sq);
          }
          // ---- first step X_1 = x + r0 U1
#pragma unroll
          for (int a = 0; a < D; ++a) X[a] = x[a] + r0 * U1[a];
          k = 1;
          lane_steps += 1u;
          lane_walks += 1u;
          sb = philox(l, (uint32_t)site, (uint32_t)kStepBlock0, kTagWalk, P.k0, P.k1);
          state = kActive;
        }
      }
    }

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
        // ---- chain tally at the cell of X_k + r Y: A += t, B += t w
        const T t = omd * r * r;
        T q[D];
#pragma unroll
        for (int a = 0; a < D; ++a) q[a] = X[a] + r * Y[a];
        const int j = grid_nearest<T, D>(P.gv, q);
        atomicAdd(&sA[j], t);
#pragma unroll
        for (int a = 0; a < D; ++a) atomicAdd(&sB[a * m + j], t * w[a]);
        // ---- move X_{k+1} = X_k + r U_k
        T U[D];
        if constexpr (D == 2) {
          const int s = (k - 1) & 3;
          const uint32_t word = (s == 0) ? sb.x : (s == 1) ? sb.y : (s == 2) ? sb.z : sb.w;
          dir2(u01<T>(word), U);
          if (s == 3) sb = philox(l, (uint32_t)site, (uint32_t)(kStepBlock0 + k / 4), kTagWalk, P.k0, P.k1);
        } else {
          const int s = (k - 1) & 1;
          const uint32_t wa = s ? sb.z : sb.x;
          const uint32_t wb = s ? sb.w : sb.y;
          dir3(u01<T>(wa), u01<T>(wb), U);
          if (s == 1) sb = philox(l, (uint32_t)site, (uint32_t)(kStepBlock0 + k / 2), kTagWalk, P.k0, P.k1);
        }
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
  const T inv_N = P.inv_N;
  const size_t n = (size_t)P.n;
  T* gA = P.A + (size_t)site * m;
  unsigned int* gH = P.Hc + (size_t)site * p;
  if (P.direct_store) {
    for (int j = tid; j < m; j += kBlock) gA[j] = sA[j] * inv_N;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T* gB = P.B + (size_t)a * n * m + (size_t)site * m;
      for (int j = tid; j < m; j += kBlock) gB[j] = sB[a * m + j] * inv_N;
      T* gK = P.K + (size_t)a * n * p + (size_t)site * p;
      for (int j = tid; j < p; j += kBlock) gK[j] = sK[a * p + j] * inv_N;
    }
    for (int j = tid; j < p; j += kBlock) gH[j] = sH[j];
  } else {
    for (int j = tid; j < m; j += kBlock) {
      const T v = sA[j];
      if (v != T(0)) atomicAdd(&gA[j], v * inv_N);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T* gB = P.B + (size_t)a * n * m + (size_t)site * m;
      for (int j = tid; j < m; j += kBlock) {
        const T v = sB[a * m + j];
        if (v != T(0)) atomicAdd(&gB[j], v * inv_N);
      }
      T* gK = P.K + (size_t)a * n * p + (size_t)site * p;
      for (int j = tid; j < p; j += kBlock) {
        const T v = sK[a * p + j];
        if (v != T(0)) atomicAdd(&gK[j], v * inv_N);
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

template <typename T, int D, int KIND>
hipError_t launch_typed(const WalkerParams<T>& P, size_t lds, int items, hipStream_t stream) {
  auto kern = walker_kernel<T, D, KIND>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(items), dim3(kBlock), lds, stream, P);
  return hipGetLastError();
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
  return t * ((size_t)(1 + dim) * m + (size_t)dim * p + 5 * (size_t)nseg) + 4 * (size_t)p;
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
