// Launch entry points of the toolbox walker (the kernel: walker_impl.hpp)
// and its LDS sizing.
#include "walker_impl.hpp"

namespace wos {

// per precision and dimension (walker_f32_2d.hip ... walker_f64_3d.hip)
hipError_t walker_dispatch_f32_2d(const WalkerParams<float>& P, int kind, size_t lds, int items, hipStream_t st);
hipError_t walker_dispatch_f32_3d(const WalkerParams<float>& P, int kind, size_t lds, int items, hipStream_t st);
hipError_t walker_dispatch_f64_2d(const WalkerParams<double>& P, int kind, size_t lds, int items, hipStream_t st);
hipError_t walker_dispatch_f64_3d(const WalkerParams<double>& P, int kind, size_t lds, int items, hipStream_t st);

size_t walker_window_lds_bytes(int dim, int pc, int pb, int npv, int npb, int nseg) {
  // 64-bit fixed-point sums of A, B (listed V pages) and K (listed boundary
  // pages), the 32-bit counts of H, the edges, the page lists (2 bytes each)
  // and the page -> slot tables (1 byte each)
  return 8 * (size_t)(1 + dim) * kPageCells * (size_t)pc + (8 * (size_t)dim + 4) * kPageCells * (size_t)pb +
         4 * 5 * (size_t)nseg + 2 * (size_t)(pc + pb) + (size_t)(npv + npb);
}

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
  const size_t lds = walker_lds_bytes(dim, P.m, P.p, P.nseg, false);
  return dim == 2 ? walker_dispatch_f32_2d(P, kind, lds, items, stream)
                  : walker_dispatch_f32_3d(P, kind, lds, items, stream);
}

hipError_t launch_walker_f64(const WalkerParams<double>& P, int dim, int kind, int items,
                             hipStream_t stream) {
  const size_t lds = walker_lds_bytes(dim, P.m, P.p, P.nseg, true);
  return dim == 2 ? walker_dispatch_f64_2d(P, kind, lds, items, stream)
                  : walker_dispatch_f64_3d(P, kind, lds, items, stream);
}

}  // namespace wos
