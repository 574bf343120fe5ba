// Launch of the fused 2D cell kernel (fused2d.hpp) with a run-time tile
// height: 'rows' tile rows of kCellTX cells, one wavefront per row.  Each
// height is compiled in its own translation unit (cell2d_rows*.hip); the
// plan's autotuner (ader_tune) picks the height per mesh.
#pragma once

#include "kernels.hpp"

namespace ader {

constexpr int kCellRowChoices[4] = {2, 4, 8, 16};
constexpr int kCellRowsDefault = 8;

struct Cell2dArgs {
  const double* u;
  int64_t ld;
  void* traces;  // predictor precision
  const double* dt;
  MeshParams mp;
  int n0, n1;    // mesh cells per axis
};

// Largest height whose block (rows wavefronts) fits the kernel's occupancy
// bound of the system and precision (rows / 4 wavefronts per SIMD).
inline int max_cell_rows(int system, int precision) {
  const int waves = system == 2 ? (precision == 0 ? 2 : 3) : (precision == 0 ? 4 : 5);
  return waves >= 4 ? 16 : 8;
}

template <int TY>
hipError_t launch_cell2d_rows(int M, int system, int precision, const Cell2dArgs& a,
                              const DevConsts& c, WsHeader* hdr, hipStream_t st);
// defined in cell2d_rows<TY>.hip
template <>
hipError_t launch_cell2d_rows<2>(int, int, int, const Cell2dArgs&, const DevConsts&, WsHeader*,
                                 hipStream_t);
template <>
hipError_t launch_cell2d_rows<4>(int, int, int, const Cell2dArgs&, const DevConsts&, WsHeader*,
                                 hipStream_t);
template <>
hipError_t launch_cell2d_rows<8>(int, int, int, const Cell2dArgs&, const DevConsts&, WsHeader*,
                                 hipStream_t);
template <>
hipError_t launch_cell2d_rows<16>(int, int, int, const Cell2dArgs&, const DevConsts&, WsHeader*,
                                  hipStream_t);

inline hipError_t launch_cell2d(int rows, int M, int system, int precision, const Cell2dArgs& a,
                                const DevConsts& c, WsHeader* hdr, hipStream_t st) {
  if (rows > max_cell_rows(system, precision)) return hipErrorInvalidConfiguration;
  switch (rows) {
    case 2: return launch_cell2d_rows<2>(M, system, precision, a, c, hdr, st);
    case 4: return launch_cell2d_rows<4>(M, system, precision, a, c, hdr, st);
    case 8: return launch_cell2d_rows<8>(M, system, precision, a, c, hdr, st);
    case 16: return launch_cell2d_rows<16>(M, system, precision, a, c, hdr, st);
    default: return hipErrorInvalidConfiguration;
  }
}

}  // namespace ader
