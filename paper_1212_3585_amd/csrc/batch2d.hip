// Instantiations of the batched 2D rounds of the solve server.
#include "../../include/ader.h"
#include "server.hpp"

namespace ader {
namespace {

template <int M, int SYS, typename R>
class BatchImpl final : public BatchImplBase {
 public:
  size_t trace_elem_size() const override { return sizeof(R); }
  hipError_t round(const SolveDesc* d_desc, SolveClock* d_mirror, int ns, long long dt_blocks,
                   long long cell_blocks, long long face_blocks, const DevConsts& c,
                   hipStream_t st) const override {
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_dt_batch<SYS>), dim3((unsigned)dt_blocks), dim3(kBlock), 0, st,
                       d_desc, ns, d_mirror);
    hipLaunchKernelGGL((k_cell2d_batch<M, SYS, kBatchTY, R>), dim3((unsigned)cell_blocks),
                       dim3(64 * kBatchTY), 0, st, d_desc, ns, c);
    hipLaunchKernelGGL((k_face2d_batch<M, SYS, R>), dim3((unsigned)face_blocks), dim3(kBlock),
                       0, st, d_desc, ns, c);
    return hipGetLastError();
  }
};

template <int M, int SYS>
const BatchImplBase* pick_prec(int precision) {
  static const BatchImpl<M, SYS, double> f64;
  static const BatchImpl<M, SYS, float> f32;
  return precision == ADER_PREC_FP64 ? static_cast<const BatchImplBase*>(&f64) : &f32;
}

template <int M>
const BatchImplBase* pick_sys(int system, int precision) {
  switch (system) {
    case ADER_SYS_LINADV: return pick_prec<M, 0>(precision);
    case ADER_SYS_EULER: return pick_prec<M, 1>(precision);
    case ADER_SYS_MHD_GLM: return pick_prec<M, 2>(precision);
  }
  return nullptr;
}

}  // namespace

const BatchImplBase* make_batch_impl_2d(int M, int system, int precision) {
  switch (M) {
    case 0: return pick_sys<0>(system, precision);
    case 1: return pick_sys<1>(system, precision);
    case 2: return pick_sys<2>(system, precision);
    case 3: return pick_sys<3>(system, precision);
  }
  return nullptr;
}

}  // namespace ader
