// Space-time predictor with wavefront-local exchanges (3D, and the 2D AMR
// levels of the fp32-predictor form).
//
// The generic predictor (k_predict) gives every spatial node of a cell one
// lane and exchanges the nodal fluxes through LDS, with two block barriers
// per time node; in 3D that moves more LDS bytes per cell and sweep than the
// arithmetic needs cycles.  Here a cell owns a group of G >= n^d lanes inside
// one wavefront (WaveCells: in 3D a power of two, G = 8, 32, 64 for n^3 = 8,
// 27, 64; in 2D exactly n^2, seven cells of nine lanes at M = 2), so the
// derivative along axis k takes the n - 1 other nodes of the lane's line
// from lanes of the same wavefront: no block barriers in the sweeps, and the
// stopping test is a ballot over the cell's lanes.  With FUSE (2D) the block
// first reconstructs its own cells (weno2d_block).
//
// fp64: each lane publishes its nodal fluxes of one time node as one record
// per axis in wavefront-private LDS (NV values padded to whole 16-byte
// vectors) and reads its line partners' records with 16-byte loads.  A
// lane-to-lane fetch (ds_bpermute) moves 4 bytes per instruction, and with at
// most 15 LDS operations in flight per wavefront the sweep waited on its
// exchanges (86 waits per sweep against 33 with the records).  The LDS of one
// wavefront is read and written in issue order, so a compiler-only fence (no
// wait, no barrier) orders the records between its lanes.
// fp32: ds_bpermute.  The records raised its registers from 66 to 95 per lane
// (seven to five wavefronts per SIMD) and made it slower.
//
// One Picard sweep of eq. stdg.final per loop trip, dimension by dimension:
//   * nodal fluxes f_k at the lane's node and time node sp;
//   * sum_k (dt/dx_k) D^(k) f_k from the line partners (lane-uniform
//     offsets m = 1..n-1: partner (p_k + m) mod n, coefficient D[p_k][.]);
//   * time product with (time factor of K^1)^-1 diag(w) and the update from
//     w_hat (time_update);
// and the first sweep from q = w_hat evaluates the fluxes once for all time
// nodes (row sums of the time matrix).  A cell stops counting iterations at
// the first sweep whose largest change is within tol * max(1, max |w_hat|);
// its lanes sweep on with the wavefront, each further sweep moving q by less
// than the tolerance.
#pragma once

#include "kernels.hpp"
#include "predict_mfma.hpp"

namespace ader {

// lanes per cell: the smallest power of two that holds n^d nodes
template <int NS> struct WaveGroup {
  static constexpr int G = NS <= 1 ? 1 : NS <= 2 ? 2 : NS <= 4 ? 4 : NS <= 8 ? 8
                         : NS <= 16 ? 16 : NS <= 32 ? 32 : 64;
  static_assert(NS <= 64, "a cell must fit one wavefront");
};

// Lanes of the wave-local predictor: in 3D a power-of-two group per cell
// (WaveGroup); in 2D exactly n^2 lanes per cell, packed (M = 2: seven cells
// of nine lanes per wavefront, where a power-of-two group holds four), the
// lanes after the last whole cell idle.
template <int DIM, int NS> struct WaveCells {
  static constexpr int G = DIM == 2 ? NS : WaveGroup<NS>::G;
  static constexpr int CPW = 64 / G;  // cells per wavefront
};

template <typename R> __device__ __forceinline__ R lane_fetch(R x, int lane);
template <> __device__ __forceinline__ float lane_fetch<float>(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(lane << 2, __float_as_int(x)));
}

// 16-byte vector of R (two doubles or four floats)
template <typename R> struct Vec16;
template <> struct Vec16<double> { typedef double __attribute__((ext_vector_type(2))) T; };
template <> struct Vec16<float> { typedef float __attribute__((ext_vector_type(4))) T; };

// orders this wavefront's LDS accesses in the compiler only: the hardware
// already performs one wavefront's LDS operations in issue order
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// maximum over the G lanes of this lane's group (G a power of two <= 64)
template <int G, typename R>
__device__ __forceinline__ R group_max(R x) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// FUSE (2D): the block reconstructs its own cells first (weno2d_block, from
// the averages fw.u of the listed cells fw.act) instead of reading w_h.
template <int DIM, int M, int SYS, typename R, typename OUT, int BLK = kBlock, bool FUSE = false>
__global__ void __launch_bounds__(BLK)
k_predict_wave(const double* __restrict__ wh, OUT* __restrict__ qh, int64_t ncells,
               const double* __restrict__ dt_dev, MeshParams mp, DevConsts c, WsHeader* hdr,
               FuseWeno fw = FuseWeno{}) {
  constexpr int n = M + 1;
  constexpr int NS = Pow<n, DIM>::v;
  constexpr int NST = NS * n;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int G = WaveCells<DIM, NS>::G;
  constexpr int CPW = WaveCells<DIM, NS>::CPW;  // cells per wavefront
  constexpr int CPB = CPW * (BLK / 64);         // cells per block
  static_assert(!FUSE || DIM == 2, "fused reconstruction in 2D only");

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot_raw = lane / G;
  const bool slot_ok = slot_raw < CPW;     // lanes after the last whole cell idle
  const int slot = slot_ok ? slot_raw : 0;  // ... and address cell 0's lanes
  const int a_raw = lane % G;
  const bool node_ok = slot_ok && a_raw < NS;
  const int a = a_raw < NS ? a_raw : 0;  // padding lanes mirror node 0 (never written out)
  // 3D: reverse block order, so that the reconstructions written last by the
  // preceding pass are read first, while still cached (the face kernel then
  // runs forward); 2D (fused reconstruction): forward, the face kernel reverse
  const int64_t blk = FUSE ? (int64_t)blockIdx.x : (int64_t)(gridDim.x - 1 - blockIdx.x);
  const int lc = wave * CPW + slot;  // the cell's place in the block
  const int64_t cell = blk * CPB + lc;
  const bool cell_ok = slot_ok && cell < ncells;
  const bool active = cell_ok && node_ok;
  const uint64_t cell_lanes =
      slot_ok ? (G == 64 ? ~0ULL : ((1ULL << G) - 1ULL)) << (slot * G) : 0ULL;

  int ak[3] = {a % n, (a / n) % n, a / (n * n)};
  const double dt = *dt_dev;
  // coef[k][m]: (dt/dx_k) D[p_k][(p_k + m) mod n]; pl[k][m]: the lane holding
  // that node of this lane's line (m = 0 is the lane)
  R coef[DIM][n];
  int pl[DIM][n];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int stride = k == 0 ? 1 : (k == 1 ? n : n * n);
    const int base = slot * G + a - ak[k] * stride;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const int b = (ak[k] + m) % n;
      coef[k][m] = (R)((dt / mp.dx[k]) * pick_entry<n>(c.dmat, ak[k], b));
      pl[k][m] = base + b * stride;
    }
  }
  const R gamma = (R)mp.gamma;
  const R ch = (R)mp.ch;
  const R adv[3] = {(R)mp.adv[0], (R)mp.adv[1], (R)mp.adv[2]};

  const double* wsrc = wh + cell * NV * NS;
  if constexpr (FUSE) {
    __shared__ double sWh[CPB * NV * NS];
    weno2d_block<M, NV, CPB>(fw, blk * CPB, ncells, mp, c, sWh);
    wsrc = sWh + lc * NV * NS;
  }
  R w[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    w[v] = active ? (R)wsrc[v * NS + a] : (v == 0 || v == NV - 1 ? R(1) : R(0));

  // stopping threshold of the cell: tol * max(1, max |w_hat|) over its nodes
  R wmax = R(0);
#pragma unroll
  for (int v = 0; v < NV; ++v) wmax = fmax(wmax, fabs(w[v]));
  wmax = node_ok ? wmax : R(0);
  R cmax;
  if constexpr ((G & (G - 1)) == 0) {
    cmax = group_max<G>(wmax);
  } else {
    // a group that is not a power of two: through wavefront-private LDS
    __shared__ R smax[BLK / 64][64];
    smax[wave][lane] = wmax;
    wave_lds_order();
    cmax = R(0);
#pragma unroll
    for (int j = 0; j < NS; ++j) cmax = fmax(cmax, smax[wave][slot * G + j]);
  }
  const R thr = (R)mp.tol * fmax(R(1), cmax);

  // fp64 exchange: wavefront-private flux records [axis][lane][NV values,
  // padded to whole 16-byte vectors]; the full vectors move as 16-byte
  // accesses, the NV mod VPV values after them one by one
  constexpr bool kRec = sizeof(R) == 8;
  typedef typename Vec16<R>::T V;
  constexpr int VPV = 16 / (int)sizeof(R);       // values per 16-byte vector
  constexpr int NFULL = NV / VPV;                 // full vectors per record
  constexpr int RV = (NV + VPV - 1) / VPV * VPV;  // record length
  __shared__ __attribute__((aligned(16))) R xrec[kRec ? BLK / 64 : 1][DIM][kRec ? 64 : 1][RV];

  // sum_k (dt/dx_k) D^(k) f_k at this lane's node
  auto derivative = [&](const R (&F)[DIM][NV], R (&out)[NV]) {
    if constexpr (kRec) {
      // the lane's own terms first, so that its fluxes are dead once published
      R (&rec)[DIM][64][RV] = xrec[wave];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) acc += coef[k][0] * F[k][v];
        out[v] = acc;
      }
      wave_lds_order();  // the partners' reads of the previous records are issued
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
#pragma unroll
        for (int j = 0; j < NFULL; ++j) {
          V x;
#pragma unroll
          for (int e = 0; e < VPV; ++e) x[e] = F[k][VPV * j + e];
          reinterpret_cast<V*>(rec[k][lane])[j] = x;
        }
#pragma unroll
        for (int v = VPV * NFULL; v < NV; ++v) rec[k][lane][v] = F[k][v];
      }
      wave_lds_order();
#pragma unroll
      for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int m = 1; m < n; ++m) {
          const R* pr = rec[k][pl[k][m]];
#pragma unroll
          for (int j = 0; j < NFULL; ++j) {
            const V x = reinterpret_cast<const V*>(pr)[j];
#pragma unroll
            for (int e = 0; e < VPV; ++e) out[VPV * j + e] += coef[k][m] * x[e];
          }
#pragma unroll
          for (int v = VPV * NFULL; v < NV; ++v) out[v] += coef[k][m] * pr[v];
        }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          acc += coef[k][0] * F[k][v];
#pragma unroll
          for (int m = 1; m < n; ++m) acc += coef[k][m] * lane_fetch<R>(F[k][v], pl[k][m]);
        }
        out[v] = acc;
      }
    }
  };
  bool done = !cell_ok;
  int iters = 0;
  auto converged = [&](R delta, int it) -> bool {
    const uint64_t moved = __ballot(node_ok && !(delta <= thr));
    if (!done && (moved & cell_lanes) == 0) {
      done = true;
      iters = it;
    }
    return !__any(!done);
  };

  R q[NV][n];
  bool all_done;
  {
    // first sweep from q = w_hat at every time node
    R F[DIM][NV];
    phys_fluxes<SYS, DIM, R>(w, gamma, ch, adv, F);
    R r[NV];
    derivative(F, r);
    R delta = R(0);
#pragma unroll
    for (int s = 0; s < n; ++s) {
      R arow = R(0);
#pragma unroll
      for (int sp = 0; sp < n; ++sp) arow += cget<R>(c.tinvw[s][sp], c.tinvw_f[s][sp]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R qn = w[v] - arow * r[v];
        delta = fmax(delta, fabs(qn - w[v]));
        q[v][s] = qn;
      }
    }
    all_done = converged(delta, 1);
  }
  for (int it = 2; !all_done && it <= mp.maxit; ++it) {
    R Racc[NV][n];
#pragma unroll
    for (int s = 0; s < n; ++s) {
      R qs[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) qs[v] = q[v][s];
      R F[DIM][NV];
      phys_fluxes<SYS, DIM, R>(qs, gamma, ch, adv, F);
      R r[NV];
      derivative(F, r);
#pragma unroll
      for (int v = 0; v < NV; ++v) Racc[v][s] = r[v];
    }
    R delta = R(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int s = 0; s < n; ++s) {
        const R qn = time_update<n>(w[v], Racc[v], c.tinvw, c.tinvw_f, s);
        delta = fmax(delta, fabs(qn - q[v][s]));
        q[v][s] = qn;
      }
    }
    all_done = converged(delta, it);
  }
  if (cell_ok && !done) iters = mp.maxit;
  const bool lead = cell_ok && a_raw == 0;
  block_report(lead ? (unsigned)iters : 0u, lead && !done ? kFlagNoConv : 0u, hdr);
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int s = 0; s < n; ++s) qh[(cell * NV + v) * NST + a + NS * s] = (OUT)q[v][s];
  }
}

}  // namespace ader
