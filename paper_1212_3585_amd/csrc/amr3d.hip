// AMR launcher instantiations for 3D problems.
#include "amr_impl.hpp"

namespace ader {

const AmrImplBase* make_amr_impl_3d(int M, int sys, int prec) {
  switch (M) {
    case 0: return pick_amr<3, 0>(sys, prec);
    case 1: return pick_amr<3, 1>(sys, prec);
    case 2: return pick_amr<3, 2>(sys, prec);
    case 3: return pick_amr<3, 3>(sys, prec);
    default: return nullptr;
  }
}
}  // namespace ader
