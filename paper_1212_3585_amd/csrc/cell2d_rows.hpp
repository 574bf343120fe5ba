// Body of one tile height's launcher (included once per height by
// cell2d_rows*.hip with CELL_ROWS defined).
#pragma once

#include "cell2d_launch.hpp"
#include "fused2d.hpp"

namespace ader {

template <int M, int SYS, int TY, typename R>
hipError_t launch_one_cell2d(const Cell2dArgs& a, const DevConsts& c, WsHeader* hdr,
                             hipStream_t st) {
  if constexpr (TY / 4 > CellWavesPerSimd<SYS, R>::v) {
    return hipErrorInvalidConfiguration;  // the block would not fit
  } else {
    dim3 grid((a.n0 + kCellTX - 1) / kCellTX, (a.n1 + TY - 1) / TY);
    hipLaunchKernelGGL((k_cell2d<M, SYS, TY, R>), grid, dim3(64 * TY), 0, st, a.u, a.ld,
                       static_cast<R*>(a.traces), a.dt, a.mp, c, hdr);
    return hipGetLastError();
  }
}

template <int M, int TY>
hipError_t launch_cell2d_m(int system, int precision, const Cell2dArgs& a, const DevConsts& c,
                           WsHeader* hdr, hipStream_t st) {
  const bool f64 = precision == 0;
  switch (system) {
    case 0: return f64 ? launch_one_cell2d<M, 0, TY, double>(a, c, hdr, st)
                       : launch_one_cell2d<M, 0, TY, float>(a, c, hdr, st);
    case 1: return f64 ? launch_one_cell2d<M, 1, TY, double>(a, c, hdr, st)
                       : launch_one_cell2d<M, 1, TY, float>(a, c, hdr, st);
    case 2: return f64 ? launch_one_cell2d<M, 2, TY, double>(a, c, hdr, st)
                       : launch_one_cell2d<M, 2, TY, float>(a, c, hdr, st);
    default: return hipErrorInvalidValue;
  }
}

template <>
hipError_t launch_cell2d_rows<CELL_ROWS>(int M, int system, int precision, const Cell2dArgs& a,
                                         const DevConsts& c, WsHeader* hdr, hipStream_t st) {
  switch (M) {
    case 0: return launch_cell2d_m<0, CELL_ROWS>(system, precision, a, c, hdr, st);
    case 1: return launch_cell2d_m<1, CELL_ROWS>(system, precision, a, c, hdr, st);
    case 2: return launch_cell2d_m<2, CELL_ROWS>(system, precision, a, c, hdr, st);
    case 3: return launch_cell2d_m<3, CELL_ROWS>(system, precision, a, c, hdr, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ader
