// wos_solve_noalloc: the FP64 Tikhonov solve of a linear problem with every
// work buffer carved from one fixed device array, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid allocation).  The array is a file-scope __device__
// object of kNoAllocScratchBytes (64 MiB), held by every GPU the library
// runs on until the process ends; its device address is taken once per
// device with hipGetSymbolAddress and only that address is handed to the
// kernels.  Every call on one GPU uses the same array: calls that overlap on
// one GPU race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "toolbox.hpp"
#include "wos_solve_kernels.hpp"

namespace wos {
void set_last_error(const char* msg);  // api.cpp
}

using namespace wos;

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

wos_status nfail(wos_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  wos::set_last_error(buf);
  return s;
}

// The device address of `scratch` on the current device, looked up on the
// first call on that device.
wos_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nfail(WOS_EDEVICE, "no current HIP device");
  if (dev < 0 || dev >= kMaxDevices) return nfail(WOS_EDEVICE, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return nfail(WOS_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WOS_OK;
}

// Hands out 256-byte aligned pieces of a fixed region, or records that it
// ran out.
struct Carver {
  unsigned char* base;
  size_t cap, used = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t at = (used + 255) & ~(size_t)255;
    used = at + std::max<size_t>(count * sizeof(T), 16);
    return used <= cap ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

// The buffers of the FP64 Tikhonov route of a linear solve: the weighted
// rows, Lambda, the normal matrix, the Cholesky work, the vector slots, the
// block vectors, the scalars and the partial sums of the transposed products.
void carve_tikhonov_f64(const wos_toolbox* tb, SolveWork& w, Carver& c) {
  const size_t n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  w.M = (int)(m + (m & 1));
  w.vlen = std::max(std::max(n, (size_t)w.M), std::max(p, d * n));
  w.R = c.take<double>((d + 1) * n * m);
  w.Lam = c.take<double>(m * m);
  w.Hess = c.take<double>(m * m);
  w.vec = c.take<double>(10 * w.vlen);
  w.red = c.take<double>(2);
  w.P64 = c.take<double>(chol_work_elems((int)m));
  w.blk = c.take<double>(2 * (d + 1) * std::max<size_t>(n, 1));
  w.regv = c.take<double>(2);
  w.info = c.take<int>(2);
  w.part_cap = gemv_part_elems((int)std::max(m, p), 1);
  w.part = c.take<double>(w.part_cap);
}

}  // namespace

extern "C" wos_status wos_solve_noalloc(wos_toolbox* tb, const wos_coeffs* co, const double* f, const double* g,
                                        double* u, double* grad_u, double* q, wos_solve_info* info, void* stream) {
  if (!tb || !co || !f || !g || !u) return nfail(WOS_EINVAL, "NULL argument");
  if (co->kind != WOS_LINEAR || co->solver != WOS_SOLVER_TIKHONOV || co->precision != WOS_SOLVE_F64)
    return nfail(WOS_EINVAL, "wos_solve_noalloc takes LINEAR problems with the TIKHONOV solver in FP64 only");
  void* base = nullptr;
  wos_status s = scratch_address(&base);
  if (s != WOS_OK) return s;
  SolveWork w;
  w.fixed = true;  // nothing is allocated or freed
  w.n = tb->n;
  w.m = tb->m;
  w.p = tb->p;
  w.d = tb->dim;
  Carver c{static_cast<unsigned char*>(base), kNoAllocScratchBytes};
  carve_tikhonov_f64(tb, w, c);
  if (c.used > c.cap)
    return nfail(WOS_ENOMEM, "the solve needs %zu bytes of work, the fixed scratch holds %zu (n = %d, m = %d, p = %d)",
                 c.used, c.cap, tb->n, tb->m, tb->p);
  w.ready = true;  // every buffer of the route is in place
  return solve_request(tb, w, co, f, g, u, grad_u, q, info, static_cast<hipStream_t>(stream));
}
