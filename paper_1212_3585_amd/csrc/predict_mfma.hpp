// Space-time predictor for 2D problems on the fp64 matrix cores (gfx950).
//
// v_mfma_f64_4x4x4f64 multiplies four independent 4x4 blocks.  Writing a
// lane as (b0, b1, b2) = (lane & 3, (lane >> 2) & 3, lane >> 4), it reads
// A[b1][i = b0][k = b2] and B[b1][k = b2][j = b0] and returns
// D[b1][i = b2][j = b0]: the contraction always runs over b2.
//
// Layout: a wavefront holds four cells (b1).  Lane (b0, b1, b2) owns the
// spatial node p_x = b2, p_y = b0 of cell b1 and keeps, in registers, all
// conserved variables at all n time nodes of that node.  One Picard sweep of
// eq. stdg.final, with the tensor structure used dimension by dimension:
//   * nodal fluxes f*, g* at the lane's n space-time nodes (lane-local);
//   * x derivative: data as operand B against (dt/dx) D in operand A
//     (contracts p_x on b2, result stays in the home layout);
//   * y derivative: a lane transpose (b0 <-> b2 inside each cell, through
//     the LDS crossbar, not on the matrix pipe) moves p_y to b2, then data
//     as operand A against (dt/dy) D^T contracts p_y and returns the home
//     layout, accumulated onto the x part;
//   * time product with (time factor of K^1)^-1 diag(w) and the update
//     q = w_hat - ... are lane-local.
// A cell stops counting iterations when its largest update falls below
// tol * max(1, max |w_hat|); the wavefront sweeps until its last cell has
// converged.
// Degrees M < 3 pad the node axes to four with zero matrix entries and a
// benign state in the padding lanes.
#pragma once

#include "kernels.hpp"

namespace ader {

template <int n>
__device__ __forceinline__ double pick_entry(const double (&m)[4][4], int i, int k) {
  double r = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a)
#pragma unroll
    for (int b = 0; b < n; ++b) r = (i == a && k == b) ? m[a][b] : r;
  return r;
}

__device__ __forceinline__ double cell_max(double x) {
  // maximum over the 16 lanes of one cell: b0 (xor 1, 2) and b2 (xor 16, 32)
  x = fmax(x, __shfl_xor(x, 1, 64));
  x = fmax(x, __shfl_xor(x, 2, 64));
  x = fmax(x, __shfl_xor(x, 16, 64));
  x = fmax(x, __shfl_xor(x, 32, 64));
  return x;
}

// Byte address for lane_transpose: lane (b0, b1, b2) reads lane (b2, b1, b0).
__device__ __forceinline__ int transpose_addr(int lane) {
  return ((lane >> 4) | (lane & 0xC) | ((lane & 3) << 4)) << 2;
}

// Swaps the two node axes (b0 <-> b2) of every cell's 4 x 4 lanes with two
// ds_bpermute (the LDS crossbar; no LDS memory is used).  An identity product
// on the matrix cores would give the same values but hold the matrix pipe,
// the kernel's bottleneck, for 16 cycles.  Every lane must be active.
__device__ __forceinline__ double lane_transpose(double x, int addr) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

template <int M, int SYS, typename OUT, bool FUSE = false>
__global__ void __launch_bounds__(kBlock)
k_predict_mfma2d(const double* __restrict__ wh, OUT* __restrict__ qh, int64_t ncells,
                 const double* __restrict__ dt_dev, MeshParams mp, DevConsts c,
                 WsHeader* hdr, FuseWeno fw = FuseWeno()) {
  constexpr int DIM = 2;
  constexpr int n = M + 1;
  constexpr int NS = n * n;
  constexpr int NST = NS * n;
  constexpr int NV = NVars<SYS, DIM>::v;
  static_assert(n <= 4, "four-point blocks");

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int b0 = lane & 3, b1 = (lane >> 2) & 3, b2 = lane >> 4;
  const int64_t cell = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * 4 + b1;
  const bool cell_ok = cell < ncells;
  const bool node_ok = b0 < n && b2 < n;
  const bool active = cell_ok && node_ok;
  const int a = b2 + n * b0;  // spatial node index p_x + n p_y

  const double dt = *dt_dev;
  const double dval = pick_entry<n>(c.dmat, b0, b2);
  const double mx = (dt / mp.dx[0]) * dval;   // operand A: D[i=b0][k=b2]
  const double my = (dt / mp.dx[1]) * dval;   // operand B: D^T[k=b2][j=b0]
  const int taddr = transpose_addr(lane);
  const double gamma = mp.gamma;
  const double adv[3] = {mp.adv[0], mp.adv[1], mp.adv[2]};

  // w_hat: from the global reconstruction, or (FUSE) from the block's own
  // reconstruction in LDS
  const double* wsrc = wh;
  int64_t wcell = cell;
  if constexpr (FUSE) {
    constexpr int CPB = 4 * (kBlock / 64);
    __shared__ double sWh[CPB * NV * NS];
    weno2d_block<M, NV, CPB>(fw, (int64_t)blockIdx.x * CPB, ncells, mp, c, sWh);
    wsrc = sWh;
    wcell = wave * 4 + b1;
  }
  double w[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    w[v] = active ? wsrc[(wcell * NV + v) * NS + a] : (v == 0 || v == NV - 1 ? 1.0 : 0.0);
  double q[NV][n];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int s = 0; s < n; ++s) q[v][s] = w[v];

  // stopping threshold of the cell, fixed before the iteration:
  // tol * max(1, max |w_hat|) over the cell's variables and nodes
  double wmax = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) wmax = fmax(wmax, fabs(w[v]));
  const double thr = mp.tol * fmax(1.0, cell_max(node_ok ? wmax : 0.0));
  const uint64_t cell_lanes = 0x000F000F000F000FULL << (4 * b1);
  bool done = !cell_ok;
  int iters = 0;
  // converged: none of the cell's lanes moved by more than thr (padding
  // lanes hold a constant state and take no part); true when every cell of
  // the wavefront has
  auto converged = [&](double delta, int it) -> bool {
    const uint64_t moved = __ballot(node_ok && !(delta <= thr));
    if (!done && (moved & cell_lanes) == 0) {
      done = true;
      iters = it;
    }
    return !__any(!done);
  };
  // The first sweep starts from q = w_hat at every time node: one flux
  // evaluation and one pair of derivative products serve all n nodes, and
  // the time product reduces to the row sums of A (the same iterate as a
  // general sweep, in exact arithmetic).
  bool all_done;
  {
    double F[DIM][NV];
    phys_fluxes<SYS, DIM, double>(w, gamma, mp.ch, adv, F);
    double delta = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double rx = __builtin_amdgcn_mfma_f64_4x4x4f64(mx, F[0][v], 0.0, 0, 0, 0);
      const double gt = lane_transpose(F[1][v], taddr);
      const double r = __builtin_amdgcn_mfma_f64_4x4x4f64(gt, my, rx, 0, 0, 0);
#pragma unroll
      for (int s = 0; s < n; ++s) {
        double arow = 0.0;
#pragma unroll
        for (int sp = 0; sp < n; ++sp) arow += c.tinvw[s][sp];
        const double qn = w[v] - arow * r;
        delta = fmax(delta, fabs(qn - w[v]));
        q[v][s] = qn;
      }
    }
    all_done = converged(delta, 1);
  }
  for (int it = 2; !all_done && it <= mp.maxit; ++it) {
    double R[NV][n];
#pragma unroll
    for (int s = 0; s < n; ++s) {
      double qs[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) qs[v] = q[v][s];
      double F[DIM][NV];
      phys_fluxes<SYS, DIM, double>(qs, gamma, mp.ch, adv, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double rx = __builtin_amdgcn_mfma_f64_4x4x4f64(mx, F[0][v], 0.0, 0, 0, 0);
        const double gt = lane_transpose(F[1][v], taddr);
        R[v][s] = __builtin_amdgcn_mfma_f64_4x4x4f64(gt, my, rx, 0, 0, 0);
      }
    }
    double delta = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int s = 0; s < n; ++s) {
        const double qn = time_update<n>(w[v], R[v], c.tinvw, c.tinvw_f, s);
        delta = fmax(delta, fabs(qn - q[v][s]));
        // a cell that has converged keeps sweeping with its wavefront: each
        // further sweep moves q by less than the tolerance towards the fixed
        // point (its iteration count is the one at first convergence)
        q[v][s] = qn;
      }
    }
    all_done = converged(delta, it);
  }
  if (cell_ok && !done) iters = mp.maxit;
  block_report(cell_ok && lane == 4 * b1 ? (unsigned)iters : 0u,
               cell_ok && lane == 4 * b1 && !done ? kFlagNoConv : 0u, hdr);
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int s = 0; s < n; ++s) qh[(cell * NV + v) * NST + a + NS * s] = (OUT)q[v][s];
  }
}

}  // namespace ader
