// Batched rounds of independent 2D solves (the solve server).
//
// A round advances every active solve of one kernel configuration (degree M,
// system, predictor precision) by one step, in three launches whose grids
// cover all those solves at once:
//   k_dt_batch      CFL step per solve (as k_dt), then the solve's clock:
//                   dt = min(CFL / max, t_end - t), t += dt, one more step;
//                   a solve whose clock has reached t_end is skipped;
//   k_cell2d_batch  cell kernel tiles of every active solve;
//   k_face2d_batch  face kernel tiles of every active solve.
// Each block finds its solve by a binary search of the per-solve block
// offsets.  Per-solve arithmetic is exactly that of the single-solve kernels:
// a result does not depend on which other solves share the round.
#pragma once

#include "fused2d.hpp"

namespace ader {

// Device-side clock of one solve (one slot of the server).
struct SolveClock {
  double t;                 // time reached by the completed steps
  double t_end;             // end time of the solve
  double dt;                // step of the current round
  unsigned long long step;  // completed steps; the state is u[step & 1]
  unsigned long long cur;   // step index of the current round (input u[cur & 1])
  int active;               // the current round computes a step
  int pad;
};

// Per-solve entry of a round's table (device memory, written by the host).
struct SolveDesc {
  double* u[2];        // ping-pong state buffers, SoA [v][ld]
  WsHeader* hdr;       // status bits and Picard counters of the solve
  double* partial;     // CFL block maxima (kDtMaxBlocks doubles)
  void* traces;        // face traces, predictor precision
  SolveClock* clock;
  MeshParams mp;
  double cfl;
  int tiles_x;         // cell kernel tiles along x (4 cells wide)
  int ftiles_x;        // face kernel tiles along x (16 cells wide)
  int dt_blocks;       // CFL blocks of the solve
  int pad;
  long long cell_block0, face_block0, dt_block0;  // first block of the solve
};


// Largest i with key(ds[i]) <= b (ds sorted by the key, key(ds[0]) = 0).
template <long long SolveDesc::*KEY>
__device__ __forceinline__ int find_solve(const SolveDesc* __restrict__ ds, int ns, long long b) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].*KEY <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// sum_k (|v_k| + c) / dx_k of one cell (the CFL wave-speed sum, reading R1)
template <int SYS>
__device__ __forceinline__ double cell_speed_sum(const double* __restrict__ u, int64_t cell,
                                                 const MeshParams& mp) {
  constexpr int NV = NVars<SYS, 2>::v;
  const double adv[3] = {mp.adv[0], mp.adv[1], mp.adv[2]};
  double q[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = u[v * mp.ld + cell];
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double f[NV], sp;
    phys_flux_dir<SYS, 2>(q, k, mp.gamma, mp.ch, adv, f, sp);
    s += sp / mp.dx[k];
  }
  return s;
}

__device__ __forceinline__ double nan_max(double a, double b) {
  // a NaN wins the maximum so that it reaches dt and the status word
  return (b != b || b > a) ? b : a;
}

// mirror[si] receives the clock of solve si after this round's update (the
// host copies the table back to decide which solves are done).
template <int SYS>
__global__ void __launch_bounds__(kBlock)
k_dt_batch(const SolveDesc* __restrict__ ds, int ns, SolveClock* __restrict__ mirror) {
  __shared__ double sw[kBlock / 64];
  __shared__ bool last;
  const int si = find_solve<&SolveDesc::dt_block0>(ds, ns, blockIdx.x);
  const SolveDesc& d = ds[si];
  SolveClock* ck = d.clock;
  const int lb = (int)(blockIdx.x - d.dt_block0);
  // t, t_end and step are rewritten only by the solve's last-arriving block,
  // after every block of the solve has read them
  const double t = ck->t, t_end = ck->t_end;
  if (!(t < t_end)) {  // finished (or failed with a NaN time): nothing to do
    if (lb == 0 && threadIdx.x == 0) {
      ck->active = 0;
      mirror[si] = *ck;
    }
    return;
  }
  const double* u = d.u[ck->step & 1];
  double smax = 0.0;
  for (int64_t cell = (int64_t)lb * kBlock + threadIdx.x; cell < d.mp.ncells;
       cell += (int64_t)d.dt_blocks * kBlock)
    smax = nan_max(smax, cell_speed_sum<SYS>(u, cell, d.mp));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) smax = nan_max(smax, __shfl_xor(smax, off, 64));
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sw[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) b = nan_max(b, sw[i]);
    d.partial[lb] = b;
    __threadfence();
    last = atomicAdd(&d.hdr->dt_blocks_done, 1u) == (unsigned)d.dt_blocks - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double m = 0.0;
  for (int i = threadIdx.x; i < d.dt_blocks; i += kBlock)
    m = nan_max(m, __hip_atomic_load(&d.partial[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sw[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) b = nan_max(b, sw[i]);
    double dt = d.cfl / b;
    const double rest = t_end - t;
    dt = rest < dt ? rest : dt;
    if (dt != dt) atomicOr(&d.hdr->status, kFlagNan);
    ck->dt = dt;
    ck->cur = ck->step;
    ck->step = ck->step + 1;
    ck->t = t + dt;  // a NaN time ends the solve at the next round
    ck->active = 1;
    mirror[si] = *ck;
    d.hdr->dt_blocks_done = 0u;
  }
}

template <int M, int SYS, int TY, typename R>
__global__ void __launch_bounds__(64 * TY, (CellWavesPerSimd<SYS, R>::v))
k_cell2d_batch(const SolveDesc* __restrict__ ds, int ns, DevConsts c) {
  const int si = find_solve<&SolveDesc::cell_block0>(ds, ns, blockIdx.x);
  const SolveDesc& d = ds[si];
  const SolveClock* ck = d.clock;
  if (!ck->active) return;  // the whole block leaves together
  const int lb = (int)(blockIdx.x - d.cell_block0);
  cell2d_tile<M, SYS, TY, R>(lb % d.tiles_x, lb / d.tiles_x, d.u[ck->cur & 1], d.mp.ld,
                             static_cast<R*>(d.traces), &ck->dt, d.mp, c, d.hdr);
}

template <int M, int SYS, typename TR>
__global__ void __launch_bounds__(kBlock)
k_face2d_batch(const SolveDesc* __restrict__ ds, int ns, DevConsts c) {
  const int si = find_solve<&SolveDesc::face_block0>(ds, ns, blockIdx.x);
  const SolveDesc& d = ds[si];
  const SolveClock* ck = d.clock;
  if (!ck->active) return;
  const int lb = (int)(blockIdx.x - d.face_block0);
  // the same flux instantiations as the single-solve face kernel, so a
  // solve's result is bitwise that of the step loop (uniform per block)
  if (SYS == 1 && d.mp.flux == 1)
    face2d_tile<M, SYS, TR, 1>(lb % d.ftiles_x, lb / d.ftiles_x, static_cast<const TR*>(d.traces),
                               d.u[ck->cur & 1], d.u[(ck->cur + 1) & 1], d.mp.ld, &ck->dt, d.mp,
                               c, d.hdr);
  else
    face2d_tile<M, SYS, TR, 0>(lb % d.ftiles_x, lb / d.ftiles_x, static_cast<const TR*>(d.traces),
                               d.u[ck->cur & 1], d.u[(ck->cur + 1) & 1], d.mp.ld, &ck->dt, d.mp,
                               c, d.hdr);
}

}  // namespace ader
