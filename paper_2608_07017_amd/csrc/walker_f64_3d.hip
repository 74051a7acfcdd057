// Walker instantiations: double, d = 3 (ball, box, box minus ball; with or
// without the moments).
#include "walker_impl.hpp"

namespace wos {

hipError_t walker_dispatch_f64_3d(const WalkerParams<double>& P, int kind, size_t lds, int items, hipStream_t st) {
  if (P.mom) {  // with the moments of the test functionals
    switch (kind) {
      case WOS_BALL: return launch_typed<double, 3, WOS_BALL | kMoments>(P, lds, items, st);
      case WOS_BOX: return launch_typed<double, 3, WOS_BOX | kMoments>(P, lds, items, st);
      case WOS_BOX_MINUS_BALL: return launch_typed<double, 3, WOS_BOX_MINUS_BALL | kMoments>(P, lds, items, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (kind) {
    case WOS_BALL: return launch_typed<double, 3, WOS_BALL>(P, lds, items, st);
    case WOS_BOX: return launch_typed<double, 3, WOS_BOX>(P, lds, items, st);
    case WOS_BOX_MINUS_BALL: return launch_typed<double, 3, WOS_BOX_MINUS_BALL>(P, lds, items, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wos
