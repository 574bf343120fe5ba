// HIP kernels of the one-step ADER-WENO step for gfx950 (CDNA4, wave64).
//
// Stage kernels (one launch each, data between stages in the workspace):
//   k_dt           CFL time step: per-cell wave-speed sum, block maxima,
//                  last-arriving block reduces them (one launch).
//   k_weno_line    one 1D WENO pass (Section 2.2) along axis K over a
//                  structure-of-arrays field; the x pass reads the averages,
//                  the y (and z) passes read the previous pass's nodal values
//                  (eqs. rec.x, rec.y, rec.z, omegas, sigmas), always fp64.
//   k_predict      space-time DG predictor (Section 2.3, eq. stdg.final):
//                  one lane per spatial node of a cell, the lane holding all
//                  time nodes of all variables; spatial derivative products
//                  exchange fluxes through LDS, the time product is
//                  lane-local.  Picard until the relative update drops below
//                  the tolerance, per cell.
//   k_face_flux    predictor traces on both sides of a face, Rusanov flux
//                  (eq. rusanov) at the space-time Gauss points, Gauss sum
//                  (eqs. flux:F-H): one lane per point, a fixed-order sum.
//   k_update       conservative update (eq. finite_vol) and device checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace ader {

constexpr int kBlock = 256;

struct DevConsts {
  double dmat[4][4];   // dmat[a][b] = psi_b'(node_a)
  double tinvw[4][4];  // (time factor of K^1)^-1 diag(w)
  double psi0[4], psi1[4], w[4];
  double rec_inv[4][4][4];  // per stencil: [p][e]
  // [stencil][r][e]: stencil averages -> Legendre coefficients of the
  // reconstruction's derivatives (orders 1..M); their squares sum to sigma
  double sig_rows[4][6][4];
  double lam[4];
  double path_s[3], path_w[3];  // Osher path-integral Gauss-Legendre rule on [0, 1]
  float dmat_f[4][4];
  float tinvw_f[4][4];
  float psi0_f[4], psi1_f[4];
};

struct MeshParams {
  int n[3];
  int bc[3];          // 0 periodic, 1 transmissive
  double dx[3];
  double gamma;
  double ch;          // GLM cleaning speed (MHD)
  int flux;           // 0 Rusanov, 1 Osher-type
  double adv[3];
  double tol;
  int maxit;
  int64_t ncells;
  int64_t ld;
};

// Picard sweeps are counted in kCounterSlots slots (block b adds to slot
// b mod kCounterSlots) so that no single address takes an atomic from every
// block; the host sums the slots.
constexpr int kCounterSlots = 64;

struct WsHeader {
  unsigned int status;
  unsigned int dt_blocks_done;  // arrival counter of k_dt (zero between calls)
  unsigned long long iters[kCounterSlots];
};
constexpr size_t kHeaderBytes = 1024;
static_assert(sizeof(WsHeader) <= kHeaderBytes, "workspace header");

constexpr unsigned int kFlagNan = 1u, kFlagNonPhysical = 2u, kFlagNoConv = 4u,
                       kFlagBadIndex = 8u;

// Adds each thread's (Picard sweeps, status bits) to the workspace header
// with one global atomic of each kind per block (block-level reduction in
// LDS first).  Every thread of the block must call it.
__device__ __forceinline__ void block_report(unsigned int sweeps, unsigned int flags,
                                             WsHeader* hdr) {
  __shared__ unsigned long long s_sweeps;
  __shared__ unsigned int s_flags;
  if (threadIdx.x == 0) {
    s_sweeps = 0ull;
    s_flags = 0u;
  }
  __syncthreads();
  if (sweeps) atomicAdd(&s_sweeps, (unsigned long long)sweeps);
  if (flags) atomicOr(&s_flags, flags);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned slot = (blockIdx.x + 17u * blockIdx.y) % kCounterSlots;
    if (s_sweeps) atomicAdd(&hdr->iters[slot], s_sweeps);
    if (s_flags) atomicOr(&hdr->status, s_flags);
  }
}

template <int B, int E> struct Pow { static constexpr int v = B * Pow<B, E - 1>::v; };
template <int B> struct Pow<B, 0> { static constexpr int v = 1; };

// number of conserved variables: linear advection 1, Euler dim + 2
// conserved variables: linear advection 1, Euler d + 2, GLM-MHD 9
template <int SYS, int DIM> struct NVars {
  static constexpr int v = SYS == 0 ? 1 : (SYS == 1 ? DIM + 2 : 9);
};
constexpr double kInv4Pi = 0.25 / 3.14159265358979323846;  // 1 / (4 pi)
constexpr double kInv8Pi = 0.125 / 3.14159265358979323846;  // 1 / (8 pi)

// ---------------------------------------------------------------- physics
// 1/x from the hardware reciprocal estimate refined by Newton-Raphson
// (r <- r + r (1 - x r), quadratic convergence); within about one ulp of the
// correctly rounded quotient, at a fraction of the cost of a full division.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  r = fmaf(fmaf(-x, r, 1.0f), r, r);
  return r;
}

// Physical fluxes of all DIM directions at one state (eq. Euler-system, or
// linear advection f_k = a_k u).  F[k][v].
template <int SYS, int DIM, typename R>
__device__ __forceinline__ void phys_fluxes(const R (&q)[NVars<SYS, DIM>::v], R gamma, R ch,
                                            const R (&adv)[3],
                                            R (&F)[DIM][NVars<SYS, DIM>::v]) {
  if constexpr (SYS == 0) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) F[k][0] = adv[k] * q[0];
  } else if constexpr (SYS == 1) {
    const R inv_rho = recip(q[0]);
    R vel[DIM];
    R kin = R(0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      vel[k] = q[1 + k] * inv_rho;
      kin += q[1 + k] * vel[k];
    }
    const R E = q[DIM + 1];
    const R p = (gamma - R(1)) * (E - R(0.5) * kin);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      F[k][0] = q[1 + k];
#pragma unroll
      for (int m = 0; m < DIM; ++m) F[k][1 + m] = q[1 + m] * vel[k];
      F[k][1 + k] += p;
      F[k][DIM + 1] = vel[k] * (E + p);
    }
  } else {
    // GLM-MHD (Section 4.2): (rho, rho v (3), E, B (3), psi)
    const R inv_rho = recip(q[0]);
    R vel[3], B[3];
    R kin = R(0), B2 = R(0), vB = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      vel[i] = q[1 + i] * inv_rho;
      B[i] = q[5 + i];
      kin += q[1 + i] * vel[i];
      B2 += B[i] * B[i];
      vB += vel[i] * B[i];
    }
    const R E = q[4], psi = q[8];
    const R pm = B2 * R(kInv8Pi);
    const R pt = (gamma - R(1)) * (E - R(0.5) * kin - pm) + pm;  // p + |B|^2 / 8 pi
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      F[k][0] = q[1 + k];
#pragma unroll
      for (int i = 0; i < 3; ++i) F[k][1 + i] = q[1 + i] * vel[k] - B[i] * B[k] * R(kInv4Pi);
      F[k][1 + k] += pt;
      F[k][4] = vel[k] * (E + pt) - B[k] * vB * R(kInv4Pi);
#pragma unroll
      for (int i = 0; i < 3; ++i) F[k][5 + i] = i == k ? psi : vel[k] * B[i] - vel[i] * B[k];
      F[k][8] = ch * ch * B[k];
    }
  }
}

// flux along one axis k and |largest eigenvalue| along k (fp64)
template <int SYS, int DIM>
__device__ __forceinline__ void phys_flux_dir(const double (&q)[NVars<SYS, DIM>::v], int k,
                                              double gamma, double ch, const double (&adv)[3],
                                              double (&f)[NVars<SYS, DIM>::v], double& speed) {
  if constexpr (SYS == 0) {
    f[0] = adv[k] * q[0];
    speed = fabs(adv[k]);
  } else if constexpr (SYS == 1) {
    const double rho = q[0];
    const double inv_rho = recip(rho);  // one refined reciprocal, no divisions
    double vel[DIM];
    double kin = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
      vel[m] = q[1 + m] * inv_rho;
      kin += q[1 + m] * vel[m];
    }
    const double E = q[DIM + 1];
    const double p = (gamma - 1.0) * (E - 0.5 * kin);
    double vk = 0.0, mk = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m)
      if (m == k) { vk = vel[m]; mk = q[1 + m]; }
    f[0] = mk;
#pragma unroll
    for (int m = 0; m < DIM; ++m) f[1 + m] = q[1 + m] * vk;
#pragma unroll
    for (int m = 0; m < DIM; ++m)
      if (m == k) f[1 + m] += p;
    f[DIM + 1] = vk * (E + p);
    speed = fabs(vk) + sqrt(gamma * p * inv_rho);
  } else {
    // GLM-MHD (Section 4.2); |largest eigenvalue| = max(|v_k| + c_f, c_h)
    // with the textbook fast magnetosonic speed c_f
    const double rho = q[0];
    const double inv_rho = recip(rho);  // one refined reciprocal, no divisions
    double vel[3], B[3];
    double kin = 0.0, B2 = 0.0, vB = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      vel[i] = q[1 + i] * inv_rho;
      B[i] = q[5 + i];
      kin += q[1 + i] * vel[i];
      B2 += B[i] * B[i];
      vB += vel[i] * B[i];
    }
    double vk = 0.0, mk = 0.0, Bk = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (i == k) { vk = vel[i]; mk = q[1 + i]; Bk = B[i]; }
    const double E = q[4], psi = q[8];
    const double pm = B2 * kInv8Pi;
    const double p = (gamma - 1.0) * (E - 0.5 * kin - pm);
    const double pt = p + pm;
    f[0] = mk;
#pragma unroll
    for (int i = 0; i < 3; ++i) f[1 + i] = q[1 + i] * vk - B[i] * Bk * kInv4Pi;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (i == k) f[1 + i] += pt;
    f[4] = vk * (E + pt) - Bk * vB * kInv4Pi;
#pragma unroll
    for (int i = 0; i < 3; ++i) f[5 + i] = i == k ? psi : vk * B[i] - vel[i] * Bk;
    f[8] = ch * ch * Bk;
    const double a2 = gamma * p * inv_rho;
    const double b2 = B2 * kInv4Pi * inv_rho, bk2 = Bk * Bk * kInv4Pi * inv_rho;
    const double sum = a2 + b2;
    const double cf = sqrt(0.5 * (sum + sqrt(fmax(sum * sum - 4.0 * a2 * bk2, 0.0))));
    speed = fmax(fabs(vk) + cf, ch);
  }
}

// |A(q)| dq for the Euler flux along axis k: sum_i |lambda_i| r_i (l_i . dq)
// with the textbook right and left eigenvectors in conserved variables
// (lambda = v_k - c, v_k (entropy, d - 1 shear), v_k + c).
template <int DIM>
__device__ __forceinline__ void euler_abs_jacobian_apply(const double (&q)[DIM + 2], int k,
                                                         double gamma,
                                                         const double (&dq)[DIM + 2],
                                                         double (&out)[DIM + 2]) {
  const double rho = q[0];
  const double ir = 1.0 / rho;
  double v[DIM], q2 = 0.0, vdm = 0.0;
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    v[m] = q[1 + m] * ir;
    q2 += v[m] * v[m];
    vdm += v[m] * dq[1 + m];
  }
  const double p = (gamma - 1.0) * (q[DIM + 1] - 0.5 * rho * q2);
  const double c = sqrt(gamma * p * ir);
  const double H = (q[DIM + 1] + p) * ir;
  double un = 0.0, dmk = 0.0;
#pragma unroll
  for (int m = 0; m < DIM; ++m)
    if (m == k) { un = v[m]; dmk = dq[1 + m]; }
  const double b1 = (gamma - 1.0) / (c * c), b2 = 0.5 * b1 * q2;
  const double base = b1 * (dq[DIM + 1] - vdm);  // b1 (dE - v . dm)
  // characteristic amplitudes, each times |lambda|
  const double a1 = fabs(un - c) * 0.5 * (b2 * dq[0] + base - (dmk - un * dq[0]) / c);
  const double a4 = fabs(un + c) * 0.5 * (b2 * dq[0] + base + (dmk - un * dq[0]) / c);
  const double ae = fabs(un) * ((1.0 - b2) * dq[0] - base);
  out[0] = a1 + ae + a4;
#pragma unroll
  for (int m = 0; m < DIM; ++m) {
    // shear amplitude of direction m != k: (dm_m - v_m drho) |v_k|
    const double at = m == k ? 0.0 : fabs(un) * (dq[1 + m] - v[m] * dq[0]);
    out[1 + m] = (a1 + ae + a4) * v[m] + at + (m == k ? c * (a4 - a1) : 0.0);
  }
  double shear_e = 0.0;
#pragma unroll
  for (int m = 0; m < DIM; ++m)
    if (m != k) shear_e += fabs(un) * (dq[1 + m] - v[m] * dq[0]) * v[m];
  out[DIM + 1] = (a1 + a4) * H + un * c * (a4 - a1) + ae * 0.5 * q2 + shear_e;
}

// Numerical flux between traces qL | qR across a face normal to axis k:
// Rusanov (eq. rusanov) or the Osher-type flux (eq. osher, Euler only; for
// linear advection it equals the upwind flux, which Rusanov already is).
// FLUX = -1 selects by mp.flux at run time; 0 / 1 fix Rusanov / Osher at
// compile time (a kernel instantiated for one flux does not carry the
// registers of the other).
template <int SYS, int DIM, int FLUX = -1>
__device__ __forceinline__ void numerical_flux(const double (&qL)[NVars<SYS, DIM>::v],
                                               const double (&qR)[NVars<SYS, DIM>::v], int k,
                                               const MeshParams& mp, const DevConsts& c,
                                               double (&F)[NVars<SYS, DIM>::v]) {
  constexpr int NV = NVars<SYS, DIM>::v;
  const double adv[3] = {mp.adv[0], mp.adv[1], mp.adv[2]};
  double fL[NV], fR[NV], sL, sR;
  phys_flux_dir<SYS, DIM>(qL, k, mp.gamma, mp.ch, adv, fL, sL);
  phys_flux_dir<SYS, DIM>(qR, k, mp.gamma, mp.ch, adv, fR, sR);
  if constexpr (SYS == 1 && FLUX != 0) {
    if (FLUX == 1 || mp.flux == 1) {
      double dq[NV], acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        dq[v] = qR[v] - qL[v];
        acc[v] = 0.0;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double qs[NV], t[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) qs[v] = qL[v] + c.path_s[j] * dq[v];
        euler_abs_jacobian_apply<DIM>(qs, k, mp.gamma, dq, t);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += c.path_w[j] * t[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * acc[v];
      return;
    }
  }
  const double smax = fmax(sL, sR);
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * smax * (qR[v] - qL[v]);
}

// Density and pressure positive (Euler, GLM-MHD); always true for advection.
template <int SYS, int DIM>
__device__ __forceinline__ bool state_physical(const double (&q)[NVars<SYS, DIM>::v],
                                               double gamma) {
  if constexpr (SYS == 0) {
    return true;
  } else if constexpr (SYS == 1) {
    double kin = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) kin += q[1 + m] * q[1 + m] / q[0];
    const double p = (gamma - 1.0) * (q[DIM + 1] - 0.5 * kin);
    return q[0] > 0.0 && p > 0.0;
  } else {
    double kin = 0.0, B2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      kin += q[1 + i] * q[1 + i] / q[0];
      B2 += q[5 + i] * q[5 + i];
    }
    const double p = (gamma - 1.0) * (q[4] - 0.5 * kin - B2 * kInv8Pi);
    return q[0] > 0.0 && p > 0.0;
  }
}

// ------------------------------------------------------------- indexing
__device__ __forceinline__ int bc_map(int i, int n, int bc) {
  if (bc == 0) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ------------------------------------------------------------- WENO line
template <int M> struct Stencils;
template <> struct Stencils<0> { static constexpr int ns = 3; };
template <> struct Stencils<1> { static constexpr int ns = 4; };
template <> struct Stencils<2> { static constexpr int ns = 3; };
template <> struct Stencils<3> { static constexpr int ns = 4; };

template <int M>
__device__ __forceinline__ constexpr int stencil_left(int s) {
  if constexpr (M % 2 == 0) {
    return s == 0 ? M / 2 : (s == 1 ? M : 0);
  } else {
    return s == 0 ? M / 2 + 1 : (s == 1 ? M / 2 : (s == 2 ? M : 0));
  }
}

// One-dimensional WENO on 2M+1 averages v[] (home cell at index M) -> the
// n nodal values of the combined polynomial (eqs. rec.x, sigmas, omegas, weno)
template <int M>
__device__ __forceinline__ void weno_line(const double (&v)[2 * M + 1], const DevConsts& c,
                                          double (&out)[M + 1]) {
  constexpr int n = M + 1;
  constexpr int NSt = Stencils<M>::ns;
  double ws[NSt][n];
  double om[NSt];
#pragma unroll
  for (int s = 0; s < NSt; ++s) {
    const int base = M - stencil_left<M>(s);
#pragma unroll
    for (int p = 0; p < n; ++p) {
      double acc = 0.0;
#pragma unroll
      for (int e = 0; e < n; ++e) acc += c.rec_inv[s][p][e] * v[base + e];
      ws[s][p] = acc;
    }
    // sigma = sum_alpha int_0^1 (d^alpha w / dxi^alpha)^2 (eq. sigmas): each
    // derivative expanded in Legendre polynomials orthonormal on [0, 1], so
    // the integral of its square is the sum of its squared coefficients.
    // The rows map the stencil averages straight to those coefficients and
    // annihilate constants, so a large mean value does not cancel in sigma.
    constexpr int NR = M * (M + 1) / 2;
    double sig = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double d = 0.0;
#pragma unroll
      for (int e = 0; e < n; ++e) d += c.sig_rows[s][r][e] * v[base + e];
      sig += d * d;
    }
    double x = sig + 1.0e-14;
    x = x * x;  // ^2
    x = x * x;  // ^4
    x = x * x;  // ^8
    om[s] = c.lam[s] * recip(x);
  }
  double tot = 0.0;
#pragma unroll
  for (int s = 0; s < NSt; ++s) tot += om[s];
  const double inv_tot = recip(tot);
#pragma unroll
  for (int s = 0; s < NSt; ++s) om[s] *= inv_tot;
#pragma unroll
  for (int p = 0; p < n; ++p) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < NSt; ++s) acc += om[s] * ws[s][p];
    out[p] = acc;
  }
}

// Reconstruction fused into a predictor (2D level lists): the block first
// reconstructs its own cells from the dense grid into LDS.  u, ld: the level's
// averages; act: the dense indices of the predicted cells.
struct FuseWeno {
  const double* u = nullptr;
  int64_t ld = 0;
  const int32_t* act = nullptr;
};

// The prologue of a fused predictor block: cells first_cell + lc, lc < CPB,
// reconstructed into sWh[(lc NV + v) n^2 + px + n py] by all the block's
// threads in two passes (the same line operations as the two-pass kernels):
// the 2M+1 x lines of every (cell, variable) from the dense grid (boundary
// maps of mp) into LDS, then the n y lines.
template <int M, int NV, int CPB>
__device__ __forceinline__ void weno2d_block(const FuseWeno& fw, int64_t first_cell,
                                             int64_t ncells, const MeshParams& mp,
                                             const DevConsts& c, double* sWh) {
  constexpr int n = M + 1;
  constexpr int S = 2 * M + 1;
  constexpr int NS = n * n;
  __shared__ double sX[CPB * NV * S * n];  // x lines [(lc NV + v) S + row][px]
  // x lines: item = lc + CPB (row + S v), neighbouring threads on
  // neighbouring cells of the list
  for (int item = threadIdx.x; item < CPB * NV * S; item += blockDim.x) {
    const int lc = item % CPB;
    const int oy = (item / CPB) % S;
    const int v = item / (CPB * S);
    const int64_t cell = first_cell + lc;
    if (cell >= ncells) continue;
    const int32_t idx = fw.act[cell];
    const int cx = (int)(idx % mp.n[0]), cy = (int)(idx / mp.n[0]);
    const int gy = bc_map(cy + oy - M, mp.n[1], mp.bc[1]);
    const int64_t row = (int64_t)v * fw.ld + (int64_t)mp.n[0] * gy;
    double vals[S];
#pragma unroll
    for (int o = 0; o < S; ++o) vals[o] = fw.u[row + bc_map(cx + o - M, mp.n[0], mp.bc[0])];
    double w[n];
    weno_line<M>(vals, c, w);
#pragma unroll
    for (int px = 0; px < n; ++px) sX[((lc * NV + v) * S + oy) * n + px] = w[px];
  }
  __syncthreads();
  // y lines: item = lc + CPB (px + n v)
  for (int item = threadIdx.x; item < CPB * NV * n; item += blockDim.x) {
    const int lc = item % CPB;
    const int px = (item / CPB) % n;
    const int v = item / (CPB * n);
    if (first_cell + lc >= ncells) continue;
    double vals[S];
#pragma unroll
    for (int o = 0; o < S; ++o) vals[o] = sX[((lc * NV + v) * S + o) * n + px];
    double w[n];
    weno_line<M>(vals, c, w);
#pragma unroll
    for (int q = 0; q < n; ++q) sWh[(lc * NV + v) * NS + px + n * q] = w[q];
  }
  __syncthreads();
}

// WENO pass along axis K.  The input field holds 'nin' nodal components per
// variable (1 for the averages; n for the y pass; n^2 for the z pass), laid
// out src[(v * nin + comp) * sld + cell].  Each thread handles one
// (variable, component, cell) line and writes n outputs.
//   OUT_AOS = false: dst[((v * n + p) * nin + comp) * C + cell], so that the
//                    next pass sees nin' = n * nin components comp' =
//                    comp + nin * p (earlier axes fastest)
//   OUT_AOS = true : dst[(cell * NV + v) * n^DIM + node(comp, p)] where the
//                    new index p becomes the slowest spatial index (x, y, z
//                    order), i.e. node = comp + nin * p.
template <int DIM, int M, int NV, int K, bool OUT_AOS>
__global__ void __launch_bounds__(kBlock)
k_weno_pass(const double* __restrict__ src, int64_t sld, int nin, double* __restrict__ dst,
            MeshParams mp, DevConsts c) {
  constexpr int n = M + 1;
  const int64_t C = mp.ncells;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= C * NV * nin) return;
  const int64_t cell = t % C;
  const int64_t vc = t / C;  // v * nin + comp
  const int comp = (int)(vc % nin);
  const int v = (int)(vc / nin);
  int idx[3];
  idx[0] = (int)(cell % mp.n[0]);
  idx[1] = (int)((cell / mp.n[0]) % mp.n[1]);
  idx[2] = DIM == 3 ? (int)(cell / ((int64_t)mp.n[0] * mp.n[1])) : 0;
  const int64_t stride = K == 0 ? 1 : (K == 1 ? (int64_t)mp.n[0] : (int64_t)mp.n[0] * mp.n[1]);
  double vals[2 * M + 1];
  const double* row = src + vc * sld + (cell - (int64_t)idx[K] * stride);
#pragma unroll
  for (int o = 0; o < 2 * M + 1; ++o) {
    const int j = bc_map(idx[K] + o - M, mp.n[K], mp.bc[K]);
    vals[o] = row[(int64_t)j * stride];
  }
  double w[n];
  weno_line<M>(vals, c, w);
  if constexpr (OUT_AOS) {
    constexpr int NS = Pow<n, DIM>::v;
#pragma unroll
    for (int p = 0; p < n; ++p) dst[(cell * NV + v) * NS + comp + nin * p] = w[p];
  } else {
#pragma unroll
    for (int p = 0; p < n; ++p) dst[(((int64_t)v * n + p) * nin + comp) * C + cell] = w[p];
  }
}

// ------------------------------------------------------------- predictor
template <typename R> struct Bits;
template <> struct Bits<double> {
  using U = unsigned long long;
  static __device__ __forceinline__ U of(double x) { return __double_as_longlong(x); }
  static __device__ __forceinline__ double val(U u) { return __longlong_as_double((long long)u); }
};
template <> struct Bits<float> {
  using U = unsigned int;
  static __device__ __forceinline__ U of(float x) { return __float_as_uint(x); }
  static __device__ __forceinline__ float val(U u) { return __uint_as_float(u); }
};

template <typename R> __device__ __forceinline__ R cget(const double& d, const float& f);
template <> __device__ __forceinline__ double cget<double>(const double& d, const float&) { return d; }
template <> __device__ __forceinline__ float cget<float>(const double&, const float& f) { return f; }

// New predictor value at time node s of eq. stdg.final:
// w_hat - sum_sp A[s][sp] r[sp], with A the time factor of (K^1)^-1 diag(w).
// fp64: one chain of fused multiply-adds that starts from w_hat.  fp32: the
// sum first, then one subtraction.  A chain from w_hat rounds every step at
// the scale of |w_hat|; the fp32 stopping threshold (1e-6 relative) is only
// about eight ulps of that, and the sweeps would then stall above it.  In
// fp64 the threshold (1e-14) is about 45 ulps.
template <int n, typename R>
__device__ __forceinline__ R time_update(R w_hat, const R (&r)[n], const double (&A)[4][4],
                                         const float (&Af)[4][4], int s) {
  if constexpr (std::is_same<R, double>::value) {
    R q = w_hat;
#pragma unroll
    for (int sp = 0; sp < n; ++sp) q -= A[s][sp] * r[sp];
    return q;
  } else {
    R acc = R(0);
#pragma unroll
    for (int sp = 0; sp < n; ++sp) acc += Af[s][sp] * r[sp];
    return w_hat - acc;
  }
}

// Select row 'a' of a 4x4 constant table into registers (unrolled selects, so
// a lane-dependent row never turns into an indexed private-memory access).
template <int n, typename R>
__device__ __forceinline__ void pick_row(const DevConsts& c, int a, R (&row)[n]) {
#pragma unroll
  for (int b = 0; b < n; ++b) {
    R r = cget<R>(c.dmat[0][b], c.dmat_f[0][b]);
#pragma unroll
    for (int aa = 1; aa < n; ++aa)
      r = (a == aa) ? cget<R>(c.dmat[aa][b], c.dmat_f[aa][b]) : r;
    row[b] = r;
  }
}

// Space-time predictor of 'ncells' cells whose nodal reconstructions are
// wh[(cell * NV + v) * NS + a].  Output qh[(cell * NV + v) * NST + a + NS * s]
// in type OUT.  One lane per spatial node a; CPB cells per BLK-thread block.
template <int DIM, int M, int SYS, typename R, typename OUT, int BLK = kBlock>
__global__ void __launch_bounds__(BLK)
k_predict(const double* __restrict__ wh, OUT* __restrict__ qh, int64_t ncells,
          const double* __restrict__ dt_dev, MeshParams mp, DevConsts c, WsHeader* hdr) {
  constexpr int n = M + 1;
  constexpr int NS = Pow<n, DIM>::v;
  constexpr int NST = NS * n;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int G = NS;
  constexpr int CPB = BLK / G;
  using U = typename Bits<R>::U;
  __shared__ R shF[DIM * NV * BLK];
  __shared__ U shDelta[CPB];
  __shared__ U shMag[CPB];

  const int tid = threadIdx.x;
  const int lc = tid / G;
  const int a = tid - lc * G;
  const int64_t cell = (int64_t)blockIdx.x * CPB + lc;
  const bool active = lc < CPB && cell < ncells;
  int ak[3];
  ak[0] = a % n;
  ak[1] = (a / n) % n;
  ak[2] = a / (n * n);

  const double dt = *dt_dev;
  R cour[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) cour[k] = (R)(dt / mp.dx[k]);
  const R gamma = (R)mp.gamma;
  const R ch = (R)mp.ch;
  R adv[3] = {(R)mp.adv[0], (R)mp.adv[1], (R)mp.adv[2]};

  R drow[DIM][n];
#pragma unroll
  for (int k = 0; k < DIM; ++k) pick_row<n, R>(c, ak[k], drow[k]);

  R w[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    w[v] = active ? (R)wh[(cell * NV + v) * NS + a] : (v == 0 || v == NV - 1 ? R(1) : R(0));
  R q[NV][n];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int s = 0; s < n; ++s) q[v][s] = w[v];

  // stopping threshold of the cell, fixed before the iteration:
  // tol * max(1, max |w_hat|) over the cell's variables and nodes
  if (tid < CPB) shMag[tid] = 0;
  __syncthreads();
  {
    R wmax = R(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) wmax = fmax(wmax, fabs(w[v]));
    if (active) atomicMax(&shMag[lc], Bits<R>::of(wmax));
  }
  __syncthreads();
  const R thr = (R)mp.tol * fmax(R(1), lc < CPB ? Bits<R>::val(shMag[lc]) : R(0));
  bool done = !active;
  int iters = 0;
  // sum_k (dt/dx_k) D^(k) f_k at this lane's node from the fluxes F of the
  // block's nodes at one time level (through LDS; synchronises the block)
  auto derivative = [&](const R (&F)[DIM][NV], R (&out)[NV]) {
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) shF[(k * NV + v) * BLK + tid] = cour[k] * F[k][v];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R acc = R(0);
      // lanes past the last whole cell of the block read nothing
      if (lc < CPB) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const int stride = k == 0 ? 1 : (k == 1 ? n : n * n);
          const int base = tid - ak[k] * stride;
#pragma unroll
          for (int b = 0; b < n; ++b)
            acc += drow[k][b] * shF[(k * NV + v) * BLK + base + b * stride];
        }
      }
      out[v] = acc;
    }
    __syncthreads();
  };
  // records this sweep's largest change per cell; true when every cell of
  // the block has converged (block-uniform)
  auto converged = [&](R delta, int it) -> bool {
    if (!done) atomicMax(&shDelta[lc], Bits<R>::of(delta));
    __syncthreads();
    if (!done) {
      const R dcell = Bits<R>::val(shDelta[lc]);
      if (dcell <= thr) {
        done = true;
        iters = it;
      }
    }
    return __syncthreads_and(done);
  };
  // The first sweep starts from q = w_hat at every time node: one flux
  // evaluation and one derivative serve all n nodes, and the time product
  // reduces to the row sums of A (the same iterate as a general sweep, in
  // exact arithmetic).
  bool all_done;
  {
    if (tid < CPB) shDelta[tid] = 0;
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
    if (tid < CPB) shDelta[tid] = 0;
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
        if (!done) q[v][s] = qn;
      }
    }
    all_done = converged(delta, it);
  }
  if (active && !done) iters = mp.maxit;
  block_report(active && a == 0 ? (unsigned)iters : 0u,
               active && a == 0 && !done ? kFlagNoConv : 0u, hdr);
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int s = 0; s < n; ++s) qh[(cell * NV + v) * NST + a + NS * s] = (OUT)q[v][s];
  }
}

// ------------------------------------------------------------- face fluxes
// Faces along axis K are indexed on the mesh extended by one along K:
// f = i + Ex * (j + Ey * k) with E = n except E_K = n_K + 1.  Face index i_K
// separates cells i_K - 1 and i_K.  F[v * nf + f].  The blocks walk the
// faces of fp64 predictors with i_K fastest, so that the faces of a block
// are consecutive along K and read each cell's q_h about once (in the
// natural order a cell's two z faces are a plane of faces apart): 3D
// face fluxes at 192^3 18.4 -> 16.6 ms per step.  With fp32 q_h (half the
// bytes) the natural order, whose blocks read contiguous runs of cells,
// measured faster (11.7 against 12.0-12.3 ms).
template <int DIM, int M, int SYS, typename R, int K>
__global__ void __launch_bounds__(kBlock)
k_face_flux(const R* __restrict__ qh, double* __restrict__ F, int64_t nfaces, MeshParams mp,
            DevConsts c) {
  constexpr int n = M + 1;
  constexpr int NS = Pow<n, DIM>::v;
  constexpr int NST = NS * n;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int NT = NS / n;  // transverse nodes
  constexpr int G = NS;       // (transverse points) x (time points)
  constexpr int FPB = kBlock / G;
  __shared__ double sh[NV * kBlock];

  const int tid = threadIdx.x;
  const int lf = tid / G;
  const int l = tid - lf * G;
  const int64_t fw = (int64_t)blockIdx.x * FPB + lf;  // position in the walk order
  constexpr bool kWalk = std::is_same<R, double>::value;
  const bool active = lf < FPB && fw < nfaces;
  int e[3] = {mp.n[0], mp.n[1], DIM == 3 ? mp.n[2] : 1};
  e[K] += 1;
  // the other two axes, in increasing order
  constexpr int A1 = K == 0 ? 1 : 0, A2 = K == 2 ? 1 : 2;
  int fi[3];
  if constexpr (kWalk) {
    fi[K] = (int)(fw % e[K]);
    fi[A1] = (int)((fw / e[K]) % e[A1]);
    fi[A2] = (int)(fw / ((int64_t)e[K] * e[A1]));
  } else {
    fi[0] = (int)(fw % e[0]);
    fi[1] = (int)((fw / e[0]) % e[1]);
    fi[2] = (int)(fw / ((int64_t)e[0] * e[1]));
  }
  const int64_t f = fi[0] + (int64_t)e[0] * (fi[1] + (int64_t)e[1] * fi[2]);

  double wpt = 0.0;
  if (active) {
    // neighbouring cells along K
    const int iL = fi[K] - 1, iR = fi[K];
    const bool outL = iL < 0, outR = iR >= mp.n[K];
    int cl[3] = {fi[0], fi[1], fi[2]}, cr[3] = {fi[0], fi[1], fi[2]};
    cl[K] = bc_map(iL, mp.n[K], mp.bc[K]);
    cr[K] = bc_map(iR, mp.n[K], mp.bc[K]);
    const int64_t cellL = cl[0] + (int64_t)mp.n[0] * (cl[1] + (int64_t)mp.n[1] * cl[2]);
    const int64_t cellR = cr[0] + (int64_t)mp.n[0] * (cr[1] + (int64_t)mp.n[1] * cr[2]);
    // lane -> (transverse node b, time node s)
    const int b = l % NT;
    const int s = l / NT;
    int tb[2] = {b % n, b / n};  // transverse axes in increasing order
    int strideK = K == 0 ? 1 : (K == 1 ? n : n * n);
    int abase = 0;
    {
      int ti = 0;
#pragma unroll
      for (int ax = 0; ax < DIM; ++ax) {
        if (ax == K) continue;
        const int st = ax == 0 ? 1 : (ax == 1 ? n : n * n);
        abase += tb[ti] * st;
        ++ti;
      }
    }
    double qL[NV], qR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R accL = R(0), accR = R(0);
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const int node = abase + j * strideK + NS * s;
        accL += cget<R>(c.psi1[j], c.psi1_f[j]) * qh[(cellL * NV + v) * NST + node];
        accR += cget<R>(c.psi0[j], c.psi0_f[j]) * qh[(cellR * NV + v) * NST + node];
      }
      qL[v] = (double)accL;
      qR[v] = (double)accR;
    }
    if (mp.bc[K] != 0) {
      if (outL) {
#pragma unroll
        for (int v = 0; v < NV; ++v) qL[v] = qR[v];
      }
      if (outR) {
#pragma unroll
        for (int v = 0; v < NV; ++v) qR[v] = qL[v];
      }
    }
    double Fpt[NV];
    numerical_flux<SYS, DIM>(qL, qR, K, mp, c, Fpt);
    double wt = c.w[s];
    {
      int ti = 0;
#pragma unroll
      for (int ax = 0; ax < DIM; ++ax) {
        if (ax == K) continue;
        wt *= c.w[tb[ti]];
        ++ti;
      }
    }
    wpt = wt;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      sh[v * kBlock + tid] = wt * Fpt[v];
  }
  (void)wpt;
  __syncthreads();
  if (active && l == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
      for (int j = 0; j < G; ++j) acc += sh[v * kBlock + tid + j];
      F[v * nfaces + f] = acc;
    }
  }
}

// ------------------------------------------------------------- update
template <int DIM, int SYS>
__global__ void __launch_bounds__(kBlock)
k_update(const double* __restrict__ u_in, double* __restrict__ u_out, const double* __restrict__ Fx,
         const double* __restrict__ Fy, const double* __restrict__ Fz, int64_t nfx, int64_t nfy,
         int64_t nfz, const double* __restrict__ dt_dev, MeshParams mp, WsHeader* hdr) {
  constexpr int NV = NVars<SYS, DIM>::v;
  const int64_t cell_raw = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool in = cell_raw < mp.ncells;
  const int64_t cell = in ? cell_raw : 0;
  const int i = (int)(cell % mp.n[0]);
  const int j = (int)((cell / mp.n[0]) % mp.n[1]);
  const int k = DIM == 3 ? (int)(cell / ((int64_t)mp.n[0] * mp.n[1])) : 0;
  const double dt = *dt_dev;
  const int nx = mp.n[0], ny = mp.n[1];
  const int64_t fx0 = i + (int64_t)(nx + 1) * (j + (int64_t)ny * k);
  const int64_t fy0 = i + (int64_t)nx * (j + (int64_t)(ny + 1) * k);
  const int64_t fz0 = cell;
  double q[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double u = u_in[v * mp.ld + cell];
    u -= (dt / mp.dx[0]) * (Fx[v * nfx + fx0 + 1] - Fx[v * nfx + fx0]);
    u -= (dt / mp.dx[1]) * (Fy[v * nfy + fy0 + nx] - Fy[v * nfy + fy0]);
    if constexpr (DIM == 3)
      u -= (dt / mp.dx[2]) * (Fz[v * nfz + fz0 + (int64_t)nx * ny] - Fz[v * nfz + fz0]);
    if (in) u_out[v * mp.ld + cell] = u;
    q[v] = u;
  }
  unsigned int flags = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (q[v] != q[v]) flags |= kFlagNan;
  if (!state_physical<SYS, DIM>(q, mp.gamma)) flags |= kFlagNonPhysical;
  block_report(0u, in ? flags : 0u, hdr);
}

// ------------------------------------------------------------- time step
template <int DIM>
__global__ void k_clear_status(WsHeader* hdr) {
  if (blockIdx.x == 0 && threadIdx.x < kCounterSlots) hdr->iters[threadIdx.x] = 0ull;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hdr->status = 0u;
    hdr->dt_blocks_done = 0u;
  }
}

// few blocks: every block adds one arrival to a single counter
constexpr int kDtMaxBlocks = 128;
// the uniform mesh's time step: one block per compute unit
constexpr int kDtUniformBlocks = 256;
// cells per thread whose loads are issued together in k_dt
constexpr int kDtCellsPerTrip = 4;

// Time step in one launch: per-block maximum of sum_k (|v_k| + c)/dx_k over
// a grid-stride range of cells, written to partial[block]; the last block to
// arrive (arrival counter in the header) reduces the partials, clips to the
// end time, writes dt and re-arms the counter.
template <int DIM, int SYS>
__global__ void __launch_bounds__(kBlock)
k_dt(const double* __restrict__ u, MeshParams mp, WsHeader* hdr, double* partial, double cfl,
     double t, double t_end, double* dt_out) {
  constexpr int NV = NVars<SYS, DIM>::v;
  __shared__ double sw[kBlock / 64];
  __shared__ bool last;
  double smax = 0.0;
  const double adv[3] = {mp.adv[0], mp.adv[1], mp.adv[2]};
  // grid-stride over the cells, kDtCellsPerTrip cells per thread and trip:
  // their loads are issued before any of them is evaluated
  constexpr int U = kDtCellsPerTrip;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x; first < mp.ncells;
       first += U * stride) {
    double q[U][NV];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t cell = first + j * stride;
#pragma unroll
      for (int v = 0; v < NV; ++v) q[j][v] = cell < mp.ncells ? u[v * mp.ld + cell] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (first + j * stride >= mp.ncells) continue;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        double f[NV], sp;
        phys_flux_dir<SYS, DIM>(q[j], k, mp.gamma, mp.ch, adv, f, sp);
        s += sp / mp.dx[k];
      }
      // a NaN must win the maximum so that it reaches dt and the status word
      smax = (s != s || s > smax) ? s : smax;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(smax, off, 64);
    smax = (o != o || o > smax) ? o : smax;
  }
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sw[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) b = (sw[i] != sw[i] || sw[i] > b) ? sw[i] : b;
    partial[blockIdx.x] = b;
    __threadfence();
    last = atomicAdd(&hdr->dt_blocks_done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double m = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kBlock) {
    const double o = __hip_atomic_load(&partial[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    m = (o != o || o > m) ? o : m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = (o != o || o > m) ? o : m;
  }
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sw[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) b = (sw[i] != sw[i] || sw[i] > b) ? sw[i] : b;
    double dt = cfl / b;
    const double rest = t_end - t;
    dt = rest < dt ? rest : dt;
    if (dt != dt) atomicOr(&hdr->status, kFlagNan);
    *dt_out = dt;
    hdr->dt_blocks_done = 0u;
  }
}

}  // namespace ader
