// Dimension-by-dimension WENO reconstruction of 3D cells through dense pass
// buffers (Section 2.2, eqs. rec.x, rec.y, rec.z, sigmas, omegas, weno).
//
// The x line of a cell depends only on the averages of its row and the y
// line only on the x lines of its column, so each is computed once per cell
// of the index space that some reconstruction reads, and kept in a dense
// buffer over that index space:
//
//   k_dense_weno_x   x pass: one line per (listed cell, variable),
//                    wx[(v n + p) wld + cell];
//   k_dense_weno_y   y pass: one line per (listed cell, variable, x node),
//                    wxy[((v n + p_y) n + p_x) wld + cell];
//   k_weno_z_aos     z pass of the cells to predict, written in the
//                    predictor's layout wh[(p NV + v) n^3 + a],
//                    a = p_x + n p_y + n^2 p_z; a block computes the lines of
//                    its cells into LDS and writes their w_h contiguously.
//
// On an AMR level the listed cells are the level's non-absent cells (active,
// virtual children, virtual mothers).  An active cell's (2M+1)^3 stencil
// patch lies in the mesh (r >= M), so every x line and y line its z pass
// reads is centred on a listed cell and is computed from listed cells only.
// Lines of the buffers that no active cell reads may hold values from absent
// cells; they are never read.  On a uniform mesh every cell is listed and the
// x and y passes are the uniform path's own.
#pragma once

#include "kernels.hpp"

namespace ader {

// Up to three cell lists (dense indices), or, when l[0] is null, the cells
// 0 .. n[0]-1 of a uniform mesh.
struct CellLists {
  const int32_t* l[3] = {nullptr, nullptr, nullptr};
  int64_t n[3] = {0, 0, 0};

  __host__ __device__ int64_t total() const { return n[0] + n[1] + n[2]; }

  __device__ __forceinline__ int64_t cell(int64_t e) const {
    if (!l[0]) return e;
    if (e < n[0]) return l[0][e];
    e -= n[0];
    if (e < n[1]) return l[1][e];
    return l[2][e - n[1]];
  }
};

__device__ __forceinline__ void coords3(int64_t cell, const MeshParams& mp, int (&c)[3]) {
  c[0] = (int)(cell % mp.n[0]);
  const int64_t r = cell / mp.n[0];
  c[1] = (int)(r % mp.n[1]);
  c[2] = (int)(r / mp.n[1]);
}

template <int M, int NV>
__global__ void __launch_bounds__(kBlock)
k_dense_weno_x(const double* __restrict__ u, int64_t ld, CellLists cl, MeshParams mp,
               double* __restrict__ wx, int64_t wld, DevConsts c) {
  constexpr int n = M + 1;
  const int64_t E = cl.total();
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= E * NV) return;
  const int64_t e = t % E;
  const int v = (int)(t / E);
  const int64_t cell = cl.cell(e);
  int cc[3];
  coords3(cell, mp, cc);
  const double* row = u + (int64_t)v * ld + (cell - cc[0]);
  double vals[2 * M + 1];
#pragma unroll
  for (int o = 0; o < 2 * M + 1; ++o) vals[o] = row[bc_map(cc[0] + o - M, mp.n[0], mp.bc[0])];
  double w[n];
  weno_line<M>(vals, c, w);
#pragma unroll
  for (int p = 0; p < n; ++p) wx[((int64_t)v * n + p) * wld + cell] = w[p];
}

template <int M, int NV>
__global__ void __launch_bounds__(kBlock)
k_dense_weno_y(const double* __restrict__ wx, CellLists cl, MeshParams mp,
               double* __restrict__ wxy, int64_t wld, DevConsts c) {
  constexpr int n = M + 1;
  const int64_t E = cl.total();
  // reverse block order: the first blocks read the x lines written last
  const int64_t b = (int64_t)(gridDim.x - 1 - blockIdx.x);
  const int64_t t = b * kBlock + threadIdx.x;
  if (t >= E * NV * n) return;
  const int64_t e = t % E;
  const int r = (int)(t / E);  // v n + px
  const int px = r % n, v = r / n;
  const int64_t cell = cl.cell(e);
  int cc[3];
  coords3(cell, mp, cc);
  const double* col = wx + ((int64_t)v * n + px) * wld + (cell - (int64_t)cc[1] * mp.n[0]);
  double vals[2 * M + 1];
#pragma unroll
  for (int o = 0; o < 2 * M + 1; ++o)
    vals[o] = col[(int64_t)bc_map(cc[1] + o - M, mp.n[1], mp.bc[1]) * mp.n[0]];
  double w[n];
  weno_line<M>(vals, c, w);
#pragma unroll
  for (int q = 0; q < n; ++q) wxy[(((int64_t)v * n + q) * n + px) * wld + cell] = w[q];
}

// Cells per block of the z pass: their w_h (NV n^3 doubles each) in LDS.
template <int M> struct ZPassCells {
  static constexpr int v = M <= 1 ? 32 : (M == 2 ? 16 : 8);
};

template <int M, int NV>
__global__ void __launch_bounds__(kBlock)
k_weno_z_aos(const double* __restrict__ wxy, int64_t wld, const int32_t* __restrict__ act,
             int64_t np, MeshParams mp, double* __restrict__ wh, DevConsts c) {
  constexpr int n = M + 1;
  constexpr int NS = n * n * n;
  constexpr int PER = NV * NS;
  constexpr int CPB = ZPassCells<M>::v;
  constexpr int LINES = NV * n * n;  // per cell: (v, p_x, p_y)
  __shared__ double sw[CPB * PER];
  const int64_t p0 = (int64_t)blockIdx.x * CPB;
  const int cpb = (int)(np - p0 < CPB ? np - p0 : CPB);
  const int64_t plane = (int64_t)mp.n[0] * mp.n[1];
  for (int item = threadIdx.x; item < cpb * LINES; item += kBlock) {
    const int lc = item % cpb;  // cell fastest: neighbouring lanes read neighbouring cells
    const int l = item / cpb;   // v n^2 + a2, a2 = p_x + n p_y
    const int v = l / (n * n), a2 = l % (n * n);
    const int64_t cell = act ? (int64_t)act[p0 + lc] : p0 + lc;
    int cc[3];
    coords3(cell, mp, cc);
    const double* line = wxy + ((int64_t)v * n * n + a2) * wld + (cell - cc[2] * plane);
    double vals[2 * M + 1];
#pragma unroll
    for (int o = 0; o < 2 * M + 1; ++o)
      vals[o] = line[(int64_t)bc_map(cc[2] + o - M, mp.n[2], mp.bc[2]) * plane];
    double w[n];
    weno_line<M>(vals, c, w);
#pragma unroll
    for (int q = 0; q < n; ++q) sw[(lc * NV + v) * NS + a2 + n * n * q] = w[q];
  }
  __syncthreads();
  double* dst = wh + p0 * PER;
  for (int i = threadIdx.x; i < cpb * PER; i += kBlock) dst[i] = sw[i];
}

}  // namespace ader
