// Device-side building blocks of the walker: the counter-based generator,
// uniforms, unit directions, the distance to the boundary r(x) and the
// nearest-centre grid lookup.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "wos_types.hpp"

namespace wos {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32->64 multiplies with XOR/permute mixing of the 128-bit counter, the
// 64-bit key advanced by the two Weyl constants between rounds.  The key is
// wave-uniform, so its schedule stays in scalar registers.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
  // An empty volatile statement that takes the key in scalar registers: it
  // keeps the compiler from hoisting all twenty round keys out of the walk
  // loop (they would be spilled to VGPR lanes and read back every round);
  // each round key is then one scalar add.
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product each (a single multiply-add instruction)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// ((x >> 9) + 1/2) * 2^-23: 24 significant bits, exact in float and double.
template <typename T>
__device__ __forceinline__ T u01(uint32_t x) {
  return (T(x >> 9) + T(0.5)) * T(1.0 / 8388608.0);
}

// ------------------------------------------------------------ directions
// d = 2: angle 2*pi*a.  float uses the hardware sine/cosine, whose input is
// in revolutions, so no range reduction is needed for a in (0,1).
__device__ __forceinline__ void dir2(float a, float* v) {
  v[0] = __builtin_amdgcn_cosf(a);
  v[1] = __builtin_amdgcn_sinf(a);
}
__device__ __forceinline__ void dir2(double a, double* v) {
  double s, c;
  sincospi(2.0 * a, &s, &c);
  v[0] = c;
  v[1] = s;
}
// d = 3: z = 2u - 1 uniform (Archimedes), azimuth 2*pi*b.
__device__ __forceinline__ void dir3(float u, float b, float* v) {
  const float z = 2.0f * u - 1.0f;
  const float s = __builtin_sqrtf(fmaxf(0.0f, 1.0f - z * z));
  v[0] = s * __builtin_amdgcn_cosf(b);
  v[1] = s * __builtin_amdgcn_sinf(b);
  v[2] = z;
}
__device__ __forceinline__ void dir3(double u, double b, double* v) {
  const double z = 2.0 * u - 1.0;
  const double s = sqrt(fmax(0.0, 1.0 - z * z));
  double sn, cs;
  sincospi(2.0 * b, &sn, &cs);
  v[0] = s * cs;
  v[1] = s * sn;
  v[2] = z;
}

__device__ __forceinline__ float dsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }

// -(2/3) ln R / (1 - R), the d = 2 weight that turns Beta(2,2) into the
// radial law of the ball-Green density.  R - 1 is exact for R > 1/2.
template <typename T>
__device__ __forceinline__ T omega2(T R) {
  const T lr = (R > T(0.5)) ? log1p(R - T(1)) : log(R);
  return T(-2.0 / 3.0) * lr / (T(1) - R);
}

// W_{-1}(y), y in [-1/e, 0): the lower real branch of the Lambert W function
// (w e^w = y, w <= -1).  Start from the series at the branch point,
// w = -1 + p - p^2/3 + 11 p^3/72 with p = -sqrt(2 (1 + e y)), when y is near
// -1/e, else from the expansion w = L1 - L2 + L2/L1 (L1 = ln(-y),
// L2 = ln(-L1)); then Halley's iteration on w e^w - y (cubic convergence:
// three steps reach the working precision from either start).
template <typename T>
__device__ __forceinline__ T lambert_wm1(T y) {
  const T q = fmax(T(0), T(2) * (T(1) + T(2.718281828459045) * y));
  T w;
  if (q < T(0.5)) {
    const T p = -sqrt(q);
    w = T(-1) + p * (T(1) + p * (T(-1.0 / 3.0) + p * T(11.0 / 72.0)));
  } else {
    const T l1 = log(-y), l2 = log(-l1);
    w = l1 - l2 + l2 / l1;
  }
  for (int k = 0; k < 3; ++k) {
    const T ew = exp(w);
    const T f = w * ew - y;
    const T wp1 = w + T(1);
    if (f == T(0) || wp1 == T(0)) break;
    w -= f / (ew * wp1 - (w + T(2)) * f / (T(2) * wp1));
  }
  return w;
}

// The exact radial law of Y in d = 2 (Prop. "removing singularities" (i.1)):
// R = exp((1 + W_{-1}(-u/e)) / 2), whose distribution function
// r^2 (1 - 2 ln r) equals u.
template <typename T>
__device__ __forceinline__ T radius_exact2(T u) {
  return exp(T(0.5) * (T(1) + lambert_wm1<T>(-u * T(0.36787944117144233))));
}

// ------------------------------------------------------------- geometry
// r(x): distance to the boundary (eq. r), specialised per domain kind.
// Polygon edges are read from LDS: (ax, ay, ex, ey, 1/|e|^2) per edge.
template <typename T, int D, int KIND>
__device__ __forceinline__ T boundary_distance(const DomainDev<T>& dom, const T* x, const T* seg,
                                               int nseg) {
  if constexpr (KIND == WOS_BALL) {
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T t = x[a] - dom.c[a];
      s += t * t;
    }
    return dom.rad - dsqrt(s);
  } else if constexpr (KIND == WOS_BOX) {
    T r = fmin(x[0] - dom.lo[0], dom.hi[0] - x[0]);
#pragma unroll
    for (int a = 1; a < D; ++a) r = fmin(r, fmin(x[a] - dom.lo[a], dom.hi[a] - x[a]));
    return r;
  } else if constexpr (KIND == WOS_POLYGON) {
    T best = T(3.0e38);
    for (int e = 0; e < nseg; ++e) {
      const T* s = seg + 5 * e;
      const T px = x[0] - s[0], py = x[1] - s[1];
      T t = (px * s[2] + py * s[3]) * s[4];
      t = fmin(fmax(t, T(0)), T(1));
      const T qx = px - t * s[2], qy = py - t * s[3];
      best = fmin(best, qx * qx + qy * qy);
    }
    return dsqrt(best);
  } else {  // WOS_BOX_MINUS_BALL
    T r = fmin(x[0] - dom.lo[0], dom.hi[0] - x[0]);
#pragma unroll
    for (int a = 1; a < D; ++a) r = fmin(r, fmin(x[a] - dom.lo[a], dom.hi[a] - x[a]));
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T t = x[a] - dom.c[a];
      s += t * t;
    }
    return fmin(r, dsqrt(s) - dom.rad);
  }
}

// ------------------------------------------------------ atomic adds
// Relaxed atomic adds with the address space stated: LDS (workgroup scope)
// or device memory (agent scope).  When an LDS add and a device add sit on
// the two sides of a branch, plain atomicAdd on generic pointers lets the
// compiler merge them into one generic (FLAT) atomic behind a pointer
// select, and a FLAT instruction makes the wave wait on both memory
// counters; with the address spaces stated they stay ds_add and
// global_atomic_add.
template <typename T>
__device__ __forceinline__ void lds_atomic_add(T* p, T v) {
  __hip_atomic_fetch_add((__attribute__((address_space(3))) T*)p, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void dev_atomic_add(T* p, T v) {
  __hip_atomic_fetch_add((__attribute__((address_space(1))) T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------ nearest centre
// Uniform grid over the bounding box.  Each cell's 16-byte record lists, in
// ascending order, every centre that can be nearest somewhere in the cell;
// a record with fewer than four candidates repeats its first one in the
// unused slots.  A cell with more than four candidates holds x = -(offset + 1)
// into a list [count, j_1 < j_2 < ...].  Candidates are compared with a
// strict '<' in order, so ties (and the repeats) go to the lowest index.
// `pts` (centres, PtStride<D> values each) may live in LDS or in global
// memory.
__device__ __forceinline__ float clamp_cell(float x, float top) { return __builtin_amdgcn_fmed3f(x, 0.0f, top); }
__device__ __forceinline__ double clamp_cell(double x, double top) { return fmin(fmax(x, 0.0), top); }

template <typename T, int D>
__device__ __forceinline__ int grid_cell(const GridDev<T>& g, const T* q) {
  // at most 2^24 cells, so the index arithmetic fits 24-bit multiplies; the
  // clamp is done before the conversion (a NaN converts to cell 0)
  unsigned int idx = 0u;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const unsigned int c = (unsigned int)(int)clamp_cell((q[a] - g.lo[a]) * g.inv_h[a], g.top[a]);
    idx = __umul24(idx, (unsigned int)g.n[a]) + c;
  }
  return (int)idx;
}

template <typename T, int D>
__device__ __forceinline__ T centre_d2(const T* pts, int j, const T* q) {
  const T* y = pts + (size_t)j * PtStride<D>::value;
  T d2 = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const T t = q[a] - y[a];
    d2 += t * t;
  }
  return d2;
}

// A point passed by value: the rare overflow lookup below is a real call,
// and a pointer to the caller's coordinates would force them (and any array
// they sit in) out of registers into scratch memory.
template <typename T, int D>
struct PointV {
  T x[D];
};

// One overflow entry: the centre (padded to three coordinates) and its
// index, loaded as one 16-byte (FP32) or 32-byte (FP64) vector.
template <typename T>
struct alignas(4 * sizeof(T)) OvfEntry {
  T v[4];
};
__device__ __forceinline__ int ovf_index(float x) { return __float_as_int(x); }
__device__ __forceinline__ int ovf_index(double x) { return (int)x; }

// A cell with more than four candidates (record x < 0, y = count, z = first
// entry): its entries are read four at a time, the four loads of a group in
// flight together, and compared in ascending index order with a strict '<'
// (a group's missing tail repeats the last entry, which changes nothing).
template <typename T, int D>
__device__ __noinline__ int grid_overflow(const GridDev<T>& g, int4 r, PointV<T, D> q) {
  const __attribute__((address_space(1))) OvfEntry<T>* e =
      (const __attribute__((address_space(1))) OvfEntry<T>*)(g.ovf) + r.z;
  const int cnt = r.y;
  int bj = 0;
  T best = T(0);
  for (int c0 = 0; c0 < cnt; c0 += 4) {
    OvfEntry<T> ev[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = min(c0 + k, cnt - 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) ev[k].v[i] = e[c].v[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      T d2 = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T t = q.x[a] - ev[k].v[a];
        d2 += t * t;
      }
      if ((c0 == 0 && k == 0) || d2 < best) {
        best = d2;
        bj = ovf_index(ev[k].v[3]);
      }
    }
  }
  return bj;
}

// Resolve a loaded record for the point q.  Unused slots repeat the first
// candidate, so a lane reads only the centres its own cell lists (LDS
// bandwidth, not issue slots, is what the lookups cost).
template <typename T, int D>
__device__ __forceinline__ int grid_resolve(const GridDev<T>& g, const T* pts, int4 r, const T* q) {
  if (r.x < 0) {
    PointV<T, D> qv;
#pragma unroll
    for (int a = 0; a < D; ++a) qv.x[a] = q[a];
    return grid_overflow<T, D>(g, r, qv);
  }
  int bj = r.x;
  if (r.y != r.x) {
    T best = centre_d2<T, D>(pts, r.x, q);
    const T d1 = centre_d2<T, D>(pts, r.y, q);
    if (d1 < best) {
      best = d1;
      bj = r.y;
    }
    if (r.z != r.x) {
      const T d2 = centre_d2<T, D>(pts, r.z, q);
      if (d2 < best) {
        best = d2;
        bj = r.z;
      }
      if (r.w != r.x) {
        const T d3 = centre_d2<T, D>(pts, r.w, q);
        if (d3 < best) bj = r.w;
      }
    }
  }
  return bj;
}

template <typename T, int D>
__device__ __forceinline__ int grid_nearest(const GridDev<T>& g, const T* pts, const T* q) {
  const int4 r = g.rec[grid_cell<T, D>(g, q)];
  return grid_resolve<T, D>(g, pts, r, q);
}

}  // namespace wos
