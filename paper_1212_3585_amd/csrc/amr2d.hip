// AMR launcher instantiations for 2D problems.
#include "amr_impl.hpp"

namespace ader {

const AmrImplBase* make_amr_impl_2d(int M, int sys, int prec) {
  switch (M) {
    case 0: return pick_amr<2, 0>(sys, prec);
    case 1: return pick_amr<2, 1>(sys, prec);
    case 2: return pick_amr<2, 2>(sys, prec);
    case 3: return pick_amr<2, 3>(sys, prec);
    default: return nullptr;
  }
}

hipError_t launch_amr_dt(const double* partial, AmrDtArgs a, AmrClock* clock, WsHeader* hdr,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_amr_dt<0>, dim3(1), dim3(64), 0, st, partial, a, clock, hdr);
  return hipGetLastError();
}

hipError_t launch_fill_list(double* u, int64_t ld, int nv, const int32_t* list, int64_t n,
                            double value, hipStream_t st) {
  if (n <= 0 || nv <= 0) return hipSuccess;
  const int64_t b = (n * nv + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_fill_list<0>, dim3((unsigned)b), dim3(kBlock), 0, st, u, ld, nv, list, n,
                     value);
  return hipGetLastError();
}

}  // namespace ader
