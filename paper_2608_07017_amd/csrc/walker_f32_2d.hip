// Walker instantiations: float, d = 2 (disk, box and polygon, each with the
// median-of-three or the exact radial sampler, and with the moments).
#include "walker_impl.hpp"

namespace wos {

hipError_t walker_dispatch_f32_2d(const WalkerParams<float>& P, int kind, size_t lds, int items, hipStream_t st) {
  if (P.mom) {  // with the moments of the test functionals (median-of-three sampler)
    if (P.exact_radius) return hipErrorInvalidValue;
    switch (kind) {
      case WOS_BALL: return launch_typed<float, 2, WOS_BALL | kMoments>(P, lds, items, st);
      case WOS_BOX: return launch_typed<float, 2, WOS_BOX | kMoments>(P, lds, items, st);
      case WOS_POLYGON: return launch_typed<float, 2, WOS_POLYGON | kMoments>(P, lds, items, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (kind) {
    case WOS_BALL:
      return P.exact_radius ? launch_typed<float, 2, WOS_BALL | kExactRadius>(P, lds, items, st)
                            : launch_typed<float, 2, WOS_BALL>(P, lds, items, st);
    case WOS_BOX:
      return P.exact_radius ? launch_typed<float, 2, WOS_BOX | kExactRadius>(P, lds, items, st)
                            : launch_typed<float, 2, WOS_BOX>(P, lds, items, st);
    case WOS_POLYGON:
      return P.exact_radius ? launch_typed<float, 2, WOS_POLYGON | kExactRadius>(P, lds, items, st)
                            : launch_typed<float, 2, WOS_POLYGON>(P, lds, items, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wos
