// Launcher instantiations for 2D problems.
#include "impl.hpp"

namespace ader {

const ImplBase* make_impl_2d(int M, int sys, int prec) {
  switch (M) {
    case 0: return pick_impl<2, 0>(sys, prec);
    case 1: return pick_impl<2, 1>(sys, prec);
    case 2: return pick_impl<2, 2>(sys, prec);
    case 3: return pick_impl<2, 3>(sys, prec);
    default: return nullptr;
  }
}

}  // namespace ader
