// One step over an explicit list of cells: the leaf cells of one refinement
// level of a cell-by-cell AMR mesh, or any subset of a uniform mesh.
//
// The predictor is element-local, so it is the same on a level as on a
// uniform mesh; the reconstruction reads a layer of at least M same-level
// cells (real or virtual) around each cell (Section 3).  The caller hands
// over, per predicted cell, the state indices of its (2M+1)^d patch, and per
// updated cell the list positions of its 2d face neighbours.
//
//   k_level_weno_pass<K>  one WENO pass (Section 2.2) along axis K for every
//                         line of every patch that the later passes need;
//                         the x pass gathers the averages through the patch
//                         indices, later passes read the previous pass.
//   (predictor)           the uniform-mesh predictor kernels on the list.
//   k_level_update        per updated cell: predictor traces of the cell and
//                         of each face neighbour at the face Gauss points,
//                         Rusanov (eq. rusanov) or Osher-type (eq. osher)
//                         flux, Gauss sum (eqs.
//                         flux:F-H) and the update (eq. finite_vol).  A face
//                         shared by two updated cells is evaluated by both
//                         with the same operand order, hence bitwise equal.
#pragma once

#include "kernels.hpp"

namespace ader {

// Pass K of the patch WENO.  Lines of the pass: the patch offsets of the
// not-yet-reconstructed axes (> K) run over 2M+1 values, those of the
// reconstructed axes (< K) over n nodes.  Layout of a pass's output per
// (cell, variable): [nodes of axes <= K (x fastest)][offsets of axes > K].
//   K = 0 reads u through patch[(p * P) + ox + S oy + S^2 oz], S = 2M+1.
template <int DIM, int M, int NV, int K>
__global__ void __launch_bounds__(kBlock)
k_level_weno_pass(const double* __restrict__ u, int64_t ld, const int32_t* __restrict__ patch,
                  const double* __restrict__ src, double* __restrict__ dst, int64_t npred,
                  DevConsts c, unsigned int* flags_out) {
  constexpr int n = M + 1;
  constexpr int S = 2 * M + 1;
  constexpr int P = Pow<S, DIM>::v;
  // values per (cell, variable) before and after this pass
  constexpr int IN = Pow<n, K>::v * Pow<S, DIM - K>::v;
  constexpr int OUT = Pow<n, K + 1>::v * Pow<S, DIM - K - 1>::v;
  constexpr int LINES = IN / S;  // lines of this pass per (cell, variable)
  // the y pass runs in reverse block order, so that it reads first the x-pass
  // lines written last (still cached), and the z pass, forward, the y lines
  const int64_t blk = K == 1 ? (int64_t)(gridDim.x - 1 - blockIdx.x) : (int64_t)blockIdx.x;
  const int64_t t = blk * kBlock + threadIdx.x;
  if (t >= npred * NV * LINES) return;
  const int line = (int)(t % LINES);
  const int64_t pv = t / LINES;  // p * NV + v
  const int v = (int)(pv % NV);
  const int64_t p = pv / NV;
  // line -> (nodes of axes < K) x (offsets of axes > K)
  constexpr int NLO = Pow<n, K>::v;  // node combinations of the done axes
  const int lo = line % NLO;
  const int hi = line / NLO;          // offsets of axes > K, fastest first
  double vals[S];
  if constexpr (K == 0) {
    const int32_t* pp = patch + p * P;
    bool bad = false;
#pragma unroll
    for (int o = 0; o < S; ++o) {
      int32_t idx = pp[o + S * hi];
      if (idx < 0 || idx >= ld) {  // out-of-range index: flagged, never read
        bad = true;
        idx = 0;
      }
      vals[o] = u[(int64_t)v * ld + idx];
    }
    if (bad) atomicOr(flags_out, kFlagBadIndex);
  } else {
    const double* sp = src + pv * IN;
#pragma unroll
    for (int o = 0; o < S; ++o) vals[o] = sp[lo + NLO * (o + S * hi)];
  }
  double w[n];
  weno_line<M>(vals, c, w);
  double* dp = dst + pv * OUT;
#pragma unroll
  for (int q = 0; q < n; ++q) dp[lo + NLO * (q + n * hi)] = w[q];
}

// Trace of one cell's predictor on its face (axis k, side 0 = low / 1 =
// high) at transverse node index tb (x fastest over the axes != k) and time
// node s: sum_j psi_j(side) q[node with index j along k].
template <int DIM, int M, int NV, typename R>
__device__ __forceinline__ void cell_trace(const R* __restrict__ qc, int k, int side, int tb,
                                           int s, const DevConsts& c, double (&out)[NV]) {
  constexpr int n = M + 1;
  constexpr int NS = Pow<n, DIM>::v;
  constexpr int NST = NS * n;
  int t[2] = {tb % n, tb / n};
  int abase = 0, ti = 0;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    if (ax == k) continue;
    abase += t[ti] * (ax == 0 ? 1 : (ax == 1 ? n : n * n));
    ++ti;
  }
  const int stride = k == 0 ? 1 : (k == 1 ? n : n * n);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    R acc = R(0);
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const R psi = side ? cget<R>(c.psi1[j], c.psi1_f[j]) : cget<R>(c.psi0[j], c.psi0_f[j]);
      acc += psi * qc[v * NST + abase + j * stride + NS * s];
    }
    out[v] = (double)acc;
  }
}

template <int DIM, int M, int SYS, typename R>
__global__ void __launch_bounds__(kBlock)
k_level_update(const R* __restrict__ qh, const int32_t* __restrict__ pred_cells,
               const int32_t* __restrict__ upd, const int32_t* __restrict__ upd_nbr,
               int64_t nupd, int64_t npred, const double* __restrict__ u_in,
               double* __restrict__ u_out,
               int64_t ld, const double* __restrict__ dt_dev, double dx0, double dx1,
               double dx2, MeshParams mp, DevConsts c, WsHeader* hdr) {
  constexpr int n = M + 1;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int NST = Pow<n, DIM + 1>::v;
  constexpr int NT = Pow<n, DIM - 1>::v;  // transverse nodes of a face
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool in = t < nupd;
  const int64_t i = in ? t : 0;
  unsigned int flags = 0;
  int32_t me = in ? upd[i] : 0;
  if (in && (me < 0 || me >= npred)) {  // out-of-range position: flagged, skipped
    flags |= kFlagBadIndex;
    me = -1;
  }
  const int64_t cell = me >= 0 ? pred_cells[me] : 0;
  if (in && me >= 0 && (cell < 0 || cell >= ld)) flags |= kFlagBadIndex;
  if (in && me >= 0 && cell >= 0 && cell < ld) {
    const double dt = *dt_dev;
    const double dxk[3] = {dx0, dx1, dx2};
    double q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = u_in[(int64_t)v * ld + cell];
    for (int k = 0; k < DIM; ++k) {
      double F[2][NV];
      for (int side = 0; side < 2; ++side) {
        int32_t nb = upd_nbr[i * 2 * DIM + 2 * k + side];
        if (nb >= npred || nb < -1) {  // out of range: flagged, taken as outflow
          flags |= kFlagBadIndex;
          nb = -1;
        }
        // the face's left and right cells (list positions); -1 = outflow
        const int32_t left = side ? me : nb, right = side ? nb : me;
#pragma unroll
        for (int v = 0; v < NV; ++v) F[side][v] = 0.0;
        for (int s = 0; s < n; ++s) {
          for (int tb = 0; tb < NT; ++tb) {
            double qL[NV], qR[NV];
            if (left >= 0) cell_trace<DIM, M, NV, R>(qh + (int64_t)left * NV * NST, k, 1, tb, s, c, qL);
            if (right >= 0) cell_trace<DIM, M, NV, R>(qh + (int64_t)right * NV * NST, k, 0, tb, s, c, qR);
            if (left < 0) {
#pragma unroll
              for (int v = 0; v < NV; ++v) qL[v] = qR[v];
            }
            if (right < 0) {
#pragma unroll
              for (int v = 0; v < NV; ++v) qR[v] = qL[v];
            }
            double Fpt[NV];
            numerical_flux<SYS, DIM>(qL, qR, k, mp, c, Fpt);
            double wt = c.w[s];
            {
              int tt[2] = {tb % n, tb / n};
              for (int d = 0; d < DIM - 1; ++d) wt *= c.w[tt[d]];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v)
              F[side][v] += wt * Fpt[v];
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] -= (dt / dxk[k]) * (F[1][v] - F[0][v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      u_out[(int64_t)v * ld + cell] = q[v];
      if (q[v] != q[v]) flags |= kFlagNan;
    }
    if (!state_physical<SYS, DIM>(q, mp.gamma)) flags |= kFlagNonPhysical;
  }
  block_report(0u, flags, hdr);
}

}  // namespace ader
