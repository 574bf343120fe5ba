// Fused 2D step: a cell kernel (WENO + predictor + face traces) and a face
// kernel (Rusanov fluxes + Gauss sums + update).  R is the predictor
// precision: double (derivative products on the fp64 matrix cores) or float
// (fp32 FMAs on exchanged lane values, fp32 accumulation).
//
// k_cell2d   one block = a 4 x TY tile of cells, TY wavefronts; wavefront w
//            holds the tile's row w (16 lanes per cell).
//   1. the averages of the tile plus M ghost layers are staged in LDS
//      (periodic or zero-gradient ghosts);
//   2. WENO x pass (Section 2.2, eqs. rec.x, sigmas, omegas, weno) on every
//      row of the tile and M rows above and below, into LDS;
//   3. WENO y pass per x degree of freedom (eqs. rec.y, weno.y) -> w_h in LDS;
//   4. Picard iteration of the space-time predictor (Section 2.3, eq.
//      stdg.final): fp64 on the matrix cores as in predict_mfma.hpp; fp32
//      with DPP lane exchanges inside each cell's row of 16 lanes;
//   5. predictor traces on the four faces at the face Gauss points in space
//      and time (used by eqs. flux:F, flux:G): contraction with psi(0) and
//      psi(1); fp64 along x by one MFMA, along y by a transpose and one
//      MFMA; fp32 by the same DPP exchanges.
//   Traces go to HBM as trace[face][cell][v][s][b] (b: transverse node,
//   s: time node), face = x-low, x-high, y-low, y-high.
//
// k_face2d   one block = a 16 x 8 tile of cells; one 16-lane group per face,
//            one lane per space-time Gauss point of the face: Rusanov flux
//            (eq. rusanov) or Osher-type flux (eq. osher) between the two traces, weighted by the Gauss
//            weights and summed over the group (eqs. flux:F, flux:G); then the
//            conservative update of the tile's cells (eq. finite_vol).  A face
//            on a tile edge is computed by both tiles with the same code and
//            the same operands, hence bitwise the same flux: the update stays
//            exactly conservative.
#pragma once

#include <type_traits>

#include "predict_mfma.hpp"

namespace ader {

constexpr int kCellTX = 4;  // tile width of the cell kernel = cells per wavefront
// Occupancy the cell kernel is compiled for (waves per SIMD; the register
// budget is 512 / waves VGPRs per lane): Euler and advection fp64 4
// (<= 128 VGPRs), fp32 5; GLM-MHD (nine variables) fp64 2, fp32 3.
template <int SYS, typename R> struct CellWavesPerSimd {
  static constexpr bool f64 = std::is_same<R, double>::value;
  static constexpr int v = SYS == 2 ? (f64 ? 2 : 3) : (f64 ? 4 : 5);
};
// lanes of matrix block b1 = 0 (b0 + 16 b2); block b1 is this mask << 4 b1
constexpr uint64_t kCellLanes = 0x000F000F000F000FULL;

// fp32 lane exchanges without the LDS crossbar: DPP quad permutations give
// lane ^ 1, ^ 2, ^ 3 (the b0 axis); row rotations (below) the b1 axis.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E;  // quad_perm [1,0,3,2], [2,3,0,1]

// Lane-local coefficients of the quad exchange (fp32 predictor): the node
// p ^ m of the same line is fetched from lane ^ m (b0 axis);
// coef[m] = scale * D[p][p ^ m] (zero where p ^ m is a padding node).
template <int n>
__device__ __forceinline__ void xor_row(const DevConsts& c, int p, double scale, float (&coef)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) coef[m] = (float)(scale * pick_entry<n>(c.dmat, p, p ^ m));
}

// acc + coef * x(lane permuted by the DPP control) as one v_fmac_f32 with a
// DPP source operand, where the compiler emits a DPP move and a separate
// FMA: the same rounding (one fused multiply-add), one VALU instruction
// fewer per exchange (fp32 step 12% faster, bitwise the same results).
// Hazards the compiler does not cover ahead of inline assembly: a DPP read
// of a VGPR needs two wait states after a VALU write of it (the s_nop 1;
// it also covers the one wait state after a transcendental op), and five
// after a VALU write of EXEC, which these kernels never make (the compiler
// lowers their branches with scalar EXEC writes; no v_cmpx in their code).
#define ADER_FMAC_DPP(NAME, CTRL)                                                      \
  __device__ __forceinline__ float NAME(float acc, float coef, float x) {              \
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 " CTRL                                    \
        " row_mask:0xf bank_mask:0xf bound_ctrl:1"                                     \
        : "+v"(acc)                                                                    \
        : "v"(x), "v"(coef));                                                          \
    return acc;                                                                        \
  }
ADER_FMAC_DPP(fmac_quad_xor1, "quad_perm:[1,0,3,2]")
ADER_FMAC_DPP(fmac_quad_xor2, "quad_perm:[2,3,0,1]")
ADER_FMAC_DPP(fmac_quad_xor3, "quad_perm:[3,2,1,0]")
ADER_FMAC_DPP(fmac_row_ror4, "row_ror:4")
ADER_FMAC_DPP(fmac_row_ror8, "row_ror:8")
ADER_FMAC_DPP(fmac_row_ror12, "row_ror:12")
#undef ADER_FMAC_DPP

// sum_m coef[m] * x(lane ^ m) over the quad (the b0 axis), m = 0..3 in order
__device__ __forceinline__ float xor_line_b0(float x, const float (&coef)[4]) {
  float acc = coef[0] * x;
  acc = fmac_quad_xor1(acc, coef[1], x);
  acc = fmac_quad_xor2(acc, coef[2], x);
  acc = fmac_quad_xor3(acc, coef[3], x);
  return acc;
}
// Row rotations inside each row of 16 lanes (DPP row_ror: lane i receives
// lane (i - 4 m) mod 16 of its row for row_ror:4m), i.e. along the b1 axis
// the lane with index p receives the value of index (p - m) mod 4.
template <int CTRL>
__device__ __forceinline__ float ror_f(float x) {
  return dpp_f<CTRL>(x);
}
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128;

// sum_m coef[m] * x(b1 index (p - m) mod 4), m = 0..3 in order
__device__ __forceinline__ float ror_line_b1(float x, const float (&coef)[4]) {
  float acc = coef[0] * x;
  acc = fmac_row_ror4(acc, coef[1], x);
  acc = fmac_row_ror8(acc, coef[2], x);
  acc = fmac_row_ror12(acc, coef[3], x);
  return acc;
}
// xor_line_b0(fx, cx) + ror_line_b1(fy, cy) as one chain of fused
// multiply-adds (the x terms, then the y terms)
__device__ __forceinline__ float line_sum_xy(float fx, const float (&cx)[4], float fy,
                                             const float (&cy)[4]) {
  float acc = xor_line_b0(fx, cx);
  acc = fmaf(cy[0], fy, acc);
  acc = fmac_row_ror4(acc, cy[1], fy);
  acc = fmac_row_ror8(acc, cy[2], fy);
  acc = fmac_row_ror12(acc, cy[3], fy);
  return acc;
}
// coef[m] = scale * D[p][(p - m) mod 4] (zero where that node is padding)
template <int n>
__device__ __forceinline__ void ror_row(const DevConsts& c, int p, double scale, float (&coef)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) coef[m] = (float)(scale * pick_entry<n>(c.dmat, p, (p - m) & 3));
}
// maximum over the 16 lanes of a row
__device__ __forceinline__ float row_max_f(float x) {
  x = fmaxf(x, dpp_f<kQuadXor1>(x));
  x = fmaxf(x, dpp_f<kQuadXor2>(x));
  x = fmaxf(x, ror_f<kRowRor4>(x));
  x = fmaxf(x, ror_f<kRowRor8>(x));
  return x;
}

// One 4 x TY tile (tile indices tile_x, tile_y) of the cell kernel.  Every
// thread of the block calls it (it synchronises the block).
template <int M, int SYS, int TY, typename R>
__device__ __forceinline__ void cell2d_tile(int tile_x, int tile_y, const double* __restrict__ u,
                                            int64_t ld, R* __restrict__ traces,
                                            const double* __restrict__ dt_dev,
                                            const MeshParams& mp, const DevConsts& c,
                                            WsHeader* hdr) {
  constexpr int DIM = 2;
  constexpr int n = M + 1;
  constexpr int NS = n * n;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int TX = kCellTX;
  constexpr int RX = TX + 2 * M;   // staged columns
  constexpr int RY = TY + 2 * M;   // staged rows
  constexpr int NT = 64 * TY;      // threads
  __shared__ double sU[NV * RY * RX];
  __shared__ double sWx[NV * RY * TX * n];
  __shared__ double sWh[TX * TY * NV * NS];

  const int tid = threadIdx.x;
  const int x0 = tile_x * TX;
  const int y0 = tile_y * TY;
  const int nx = mp.n[0], ny = mp.n[1];

  // Wave priority (fp64): the staging and WENO phases are bounded by
  // barriers and latency, the Picard sweeps by issue; a block in the former
  // takes issue slots before a co-resident block's sweeps.  Measured faster
  // for the fp64 kernel and slower for the fp32 one, which keeps the default.
  constexpr bool kPrio = std::is_same<R, double>::value;
  if constexpr (kPrio) __builtin_amdgcn_s_setprio(2);
  // 1. stage the averages (tile + M ghost layers)
  for (int e = tid; e < NV * RY * RX; e += NT) {
    const int rx = e % RX;
    const int ry = (e / RX) % RY;
    const int v = e / (RX * RY);
    const int gi = bc_map(x0 + rx - M, nx, mp.bc[0]);
    const int gj = bc_map(y0 + ry - M, ny, mp.bc[1]);
    sU[e] = u[(int64_t)v * ld + gi + (int64_t)nx * gj];
  }
  __syncthreads();
  // 2. x pass: one thread per (variable, staged row, tile column)
  for (int e = tid; e < NV * RY * TX; e += NT) {
    const int cx = e % TX;
    const int ry = (e / TX) % RY;
    const int v = e / (TX * RY);
    double vals[2 * M + 1];
#pragma unroll
    for (int o = 0; o < 2 * M + 1; ++o) vals[o] = sU[(v * RY + ry) * RX + cx + o];
    double w[n];
    weno_line<M>(vals, c, w);
#pragma unroll
    for (int p = 0; p < n; ++p) sWx[((v * RY + ry) * TX + cx) * n + p] = w[p];
  }
  __syncthreads();
  // 3. y pass: one thread per (tile cell, variable, x node)
  for (int e = tid; e < TX * TY * NV * n; e += NT) {
    const int px = e % n;
    const int v = (e / n) % NV;
    const int cl = e / (n * NV);  // tile cell: cx + TX cy
    const int cx = cl % TX, cy = cl / TX;
    double vals[2 * M + 1];
#pragma unroll
    for (int o = 0; o < 2 * M + 1; ++o) vals[o] = sWx[((v * RY + cy + o) * TX + cx) * n + px];
    double w[n];
    weno_line<M>(vals, c, w);
#pragma unroll
    for (int p = 0; p < n; ++p) sWh[(cl * NV + v) * NS + px + n * p] = w[p];
  }
  __syncthreads();

  // 4. predictor: wavefront = tile row, four cells per wavefront.  Lane
  //    roles (b0, b1, b2) = (lane & 3, (lane >> 2) & 3, lane >> 4):
  //    fp64: p_x = b2, p_y = b0, cell = b1 -- the matrix-core layout of
  //          predict_mfma.hpp (one cell per matrix block);
  //    fp32: p_x = b0, p_y = b1, cell = b2 -- a cell is a row of 16 lanes, so
  //          both node axes are exchanged by DPP inside the row (p_x by quad
  //          permutations, p_y by row rotations), fp32 FMAs, fp32 sums.
  constexpr bool kMatrix = std::is_same<R, double>::value;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int b0 = lane & 3, b1 = (lane >> 2) & 3, b2 = lane >> 4;
  const int px = kMatrix ? b2 : b0;
  const int py = kMatrix ? b0 : b1;
  const int slot = kMatrix ? b1 : b2;
  const int gi = x0 + slot, gj = y0 + wave;
  const bool cell_ok = gi < nx && gj < ny;
  const bool node_ok = px < n && py < n;
  const int64_t cell = gi + (int64_t)nx * gj;
  const int cl = slot + TX * wave;
  const bool lead = px == 0 && py == 0;  // first lane of the cell
  // the 16 lanes of this lane's cell
  const uint64_t cell_lanes = kMatrix ? kCellLanes << (4 * b1) : 0xFFFFULL << (16 * b2);

  const double dt = *dt_dev;
  const double dval = pick_entry<n>(c.dmat, b0, b2);
  const double mx = (dt / mp.dx[0]) * dval;
  const double my = (dt / mp.dx[1]) * dval;
  const int taddr = transpose_addr(lane);
  float cxm[4], cyr[4];
  xor_row<n>(c, px, dt / mp.dx[0], cxm);
  ror_row<n>(c, py, dt / mp.dx[1], cyr);
  const R gamma = (R)mp.gamma;
  const R ch = (R)mp.ch;
  const R adv[3] = {(R)mp.adv[0], (R)mp.adv[1], (R)mp.adv[2]};

  R w[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    w[v] = node_ok ? (R)sWh[(cl * NV + v) * NS + px + n * py] : (v == 0 || v == NV - 1 ? R(1) : R(0));
  R q[NV][n];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int s = 0; s < n; ++s) q[v][s] = w[v];

  // stopping threshold of the cell, fixed before the iteration:
  // tol * max(1, max |w_hat|) over the cell's variables and nodes
  R wmax = R(0);
#pragma unroll
  for (int v = 0; v < NV; ++v) wmax = fmax(wmax, fabs(w[v]));
  wmax = node_ok ? wmax : R(0);
  R wcell;
  if constexpr (kMatrix)
    wcell = cell_max(wmax);
  else
    wcell = row_max_f(wmax);
  const R thr = (R)mp.tol * fmax(R(1), wcell);
  bool done = !cell_ok;
  int iters = 0;
  // one Picard sweep from qa into qb; returns this lane's largest change
  auto sweep = [&](const R (&qa)[NV][n], R (&qb)[NV][n]) -> R {
    R Rs[NV][n];
#pragma unroll
    for (int s = 0; s < n; ++s) {
      R qs[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) qs[v] = qa[v][s];
      R F[DIM][NV];
      phys_fluxes<SYS, DIM, R>(qs, gamma, ch, adv, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (kMatrix) {
          const double rx = __builtin_amdgcn_mfma_f64_4x4x4f64(mx, F[0][v], 0.0, 0, 0, 0);
          const double gt = lane_transpose(F[1][v], taddr);
          Rs[v][s] = __builtin_amdgcn_mfma_f64_4x4x4f64(gt, my, rx, 0, 0, 0);
        } else {
          Rs[v][s] = line_sum_xy(F[0][v], cxm, F[1][v], cyr);
        }
      }
    }
    R delta = R(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int s = 0; s < n; ++s) {
        const R qn = time_update<n>(w[v], Rs[v], c.tinvw, c.tinvw_f, s);
        delta = fmax(delta, fabs(qn - qa[v][s]));
        qb[v][s] = qn;
      }
    }
    return delta;
  };
  // The first sweep starts from q = w_hat at every time node: one flux
  // evaluation and one pair of derivative products serve all n nodes, and
  // the time product reduces to the row sums of A (the same iterate as a
  // general sweep, in exact arithmetic).
  R arow[n];
#pragma unroll
  for (int s = 0; s < n; ++s) {
    R acc = R(0);
#pragma unroll
    for (int sp = 0; sp < n; ++sp) acc += cget<R>(c.tinvw[s][sp], c.tinvw_f[s][sp]);
    arow[s] = acc;
  }
  auto first_sweep = [&](R (&qb)[NV][n]) -> R {
    R F[DIM][NV];
    phys_fluxes<SYS, DIM, R>(w, gamma, ch, adv, F);
    R delta = R(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R r;
      if constexpr (kMatrix) {
        const double rx = __builtin_amdgcn_mfma_f64_4x4x4f64(mx, F[0][v], 0.0, 0, 0, 0);
        const double gt = lane_transpose(F[1][v], taddr);
        r = __builtin_amdgcn_mfma_f64_4x4x4f64(gt, my, rx, 0, 0, 0);
      } else {
        r = line_sum_xy(F[0][v], cxm, F[1][v], cyr);
      }
#pragma unroll
      for (int s = 0; s < n; ++s) {
        const R qn = w[v] - arow[s] * r;
        delta = fmax(delta, fabs(qn - w[v]));
        qb[v][s] = qn;
      }
    }
    return delta;
  };
  // a cell has converged when none of its 16 lanes moved by more than thr;
  // returns true when every cell of the wavefront has
  auto converged = [&](R delta, int it) -> bool {
    const uint64_t moved = __ballot(node_ok && !(delta <= thr));
    if (!done && (moved & cell_lanes) == 0) {
      done = true;
      iters = it;
    }
    return !__any(!done);
  };
  // two sweeps per trip, alternating the two state arrays (no copies); the
  // exits are wavefront-uniform
  if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
  R q2[NV][n];
  bool in_q2 = false;
  const bool first_done = converged(first_sweep(q), 1);
  for (int it = 2; !first_done && it <= mp.maxit; it += 2) {
    if (converged(sweep(q, q2), it)) {
      in_q2 = true;
      break;
    }
    if (it + 1 > mp.maxit) {
      in_q2 = true;
      break;
    }
    if (converged(sweep(q2, q), it + 1)) break;
  }
  if (in_q2) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int s = 0; s < n; ++s) q[v][s] = q2[v][s];
  }
  if (cell_ok && !done) iters = mp.maxit;
  block_report(cell_ok && lead ? (unsigned)iters : 0u,
               cell_ok && lead && !done ? kFlagNoConv : 0u, hdr);

  // 5. face traces.  fp64: x faces: operand A row 0 = psi(0), row 1 = psi(1)
  //    (A[i=b0][k=b2]); result lane (b0 = y node, b2 = 0 / 1 = low / high).
  //    y faces: transpose, then operand B column 0 = psi(0), column 1 =
  //    psi(1) (B[k=b2][j=b0]); result lane (b0 = 0 / 1 = low / high, b2 = x
  //    node).  fp32: every lane forms the traces of its own line by DPP
  //    exchanges; lanes p_x = 0 write the x faces, lanes p_y = 0 the y faces.
  const int64_t C = mp.ncells;
  constexpr int TRC = NV * n * n;  // values per trace
  if constexpr (kMatrix) {
    double ex = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      const double p0 = c.psi0[k], p1 = c.psi1[k];
      ex = (b2 == k) ? (b0 == 0 ? p0 : (b0 == 1 ? p1 : 0.0)) : ex;
    }
    const double ey = ex;  // same lane pattern: B[k=b2][j=b0] = psi_k(j)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int s = 0; s < n; ++s) {
        const double tx = __builtin_amdgcn_mfma_f64_4x4x4f64(ex, q[v][s], 0.0, 0, 0, 0);
        const double qt = lane_transpose(q[v][s], taddr);
        const double ty = __builtin_amdgcn_mfma_f64_4x4x4f64(qt, ey, 0.0, 0, 0, 0);
        if (cell_ok) {
          if (b2 < 2 && b0 < n)  // x face b2 (0 low, 1 high), transverse node b0
            traces[((int64_t)b2 * C + cell) * TRC + (v * n + s) * n + b0] = tx;
          if (b0 < 2 && b2 < n)  // y face b0, transverse node b2
            traces[((int64_t)(2 + b0) * C + cell) * TRC + (v * n + s) * n + b2] = ty;
        }
      }
    }
  } else {
    // e?x[m]: weight of node p_x ^ m (quad exchange); e?y[m]: weight of
    // node (p_y - m) mod 4 (row rotation); zero for padding nodes
    float e0x[4], e1x[4], e0y[4], e1y[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float a0 = 0.f, a1 = 0.f, c0 = 0.f, c1 = 0.f;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        a0 = ((px ^ m) == k) ? c.psi0_f[k] : a0;
        a1 = ((px ^ m) == k) ? c.psi1_f[k] : a1;
        c0 = (((py - m) & 3) == k) ? c.psi0_f[k] : c0;
        c1 = (((py - m) & 3) == k) ? c.psi1_f[k] : c1;
      }
      e0x[m] = a0;
      e1x[m] = a1;
      e0y[m] = c0;
      e1y[m] = c1;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int s = 0; s < n; ++s) {
        const R x = q[v][s];
        const R tx0 = xor_line_b0(x, e0x), tx1 = xor_line_b0(x, e1x);
        const R ty0 = ror_line_b1(x, e0y), ty1 = ror_line_b1(x, e1y);
        if (cell_ok) {
          if (px == 0 && py < n) {
            traces[((int64_t)0 * C + cell) * TRC + (v * n + s) * n + py] = tx0;
            traces[((int64_t)1 * C + cell) * TRC + (v * n + s) * n + py] = tx1;
          }
          if (py == 0 && px < n) {
            traces[((int64_t)2 * C + cell) * TRC + (v * n + s) * n + px] = ty0;
            traces[((int64_t)3 * C + cell) * TRC + (v * n + s) * n + px] = ty1;
          }
        }
      }
    }
  }
}

template <int M, int SYS, int TY, typename R>
__global__ void __launch_bounds__(64 * TY, (CellWavesPerSimd<SYS, R>::v))
k_cell2d(const double* __restrict__ u, int64_t ld, R* __restrict__ traces,
         const double* __restrict__ dt_dev, MeshParams mp, DevConsts c, WsHeader* hdr) {
  cell2d_tile<M, SYS, TY, R>(blockIdx.x, blockIdx.y, u, ld, traces, dt_dev, mp, c, hdr);
}

constexpr int kFaceTX = 16, kFaceTY = 8;

// One 16 x 8 tile of the face kernel (every thread of the block calls it).
// FLUX: -1 numerical flux chosen at run time, 0 Rusanov, 1 Osher-type.
template <int M, int SYS, typename TR, int FLUX = -1>
__device__ __forceinline__ void face2d_tile(int tile_x, int tile_y, const TR* __restrict__ traces,
                                            const double* __restrict__ u_in,
                                            double* __restrict__ u_out, int64_t ld,
                                            const double* __restrict__ dt_dev,
                                            const MeshParams& mp, const DevConsts& c,
                                            WsHeader* hdr) {
  constexpr int DIM = 2;
  constexpr int n = M + 1;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int TRC = NV * n * n;
  constexpr int TX = kFaceTX, TY = kFaceTY;
  constexpr int NFX = (TX + 1) * TY;  // x faces of the tile
  constexpr int NFY = TX * (TY + 1);  // y faces of the tile
  constexpr int NF = NFX + NFY;
  constexpr int GROUPS = kBlock / 16;
  __shared__ double sF[NF * NV];

  const int tid = threadIdx.x;
  const int grp = tid >> 4;
  const int l = tid & 15;  // Gauss point l = b + n s of the face
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int nx = mp.n[0], ny = mp.n[1];
  const int64_t C = mp.ncells;
  const bool point_ok = l < n * n;
  const int b = point_ok ? l % n : 0;
  const int s = point_ok ? l / n : 0;
  const double wts = point_ok ? c.w[b] * c.w[s] : 0.0;

  // the same trip count for every group keeps the shuffles below uniform
  for (int base = 0; base < NF; base += GROUPS) {
    const int f = base + grp;
    const bool f_in = f < NF;
    int k, fi, fj;  // axis, face index (i along x, j along y)
    if (f < NFX) {
      k = 0;
      fi = x0 + f % (TX + 1);
      fj = y0 + f / (TX + 1);
    } else {
      k = 1;
      fi = x0 + (f - NFX) % TX;
      fj = y0 + (f - NFX) / TX;
    }
    const int nk = k == 0 ? nx : ny;
    const int ik = k == 0 ? fi : fj;       // index along the axis: separates ik-1 | ik
    const bool face_ok = f_in && fi <= nx && fj <= ny && (k == 0 ? fj < ny : fi < nx);
    double Fp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fp[v] = 0.0;
    if (face_ok && point_ok) {
      const bool outL = ik - 1 < 0, outR = ik >= nk;
      const int iL = bc_map(ik - 1, nk, mp.bc[k]), iR = bc_map(ik, nk, mp.bc[k]);
      const int64_t cL = k == 0 ? iL + (int64_t)nx * fj : fi + (int64_t)nx * iL;
      const int64_t cR = k == 0 ? iR + (int64_t)nx * fj : fi + (int64_t)nx * iR;
      // high-side trace of the left cell, low-side trace of the right cell
      const TR* tL = traces + ((int64_t)(2 * k + 1) * C + cL) * TRC;
      const TR* tR = traces + ((int64_t)(2 * k) * C + cR) * TRC;
      double qL[NV], qR[NV];  // traces in the predictor precision, flux in fp64
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qL[v] = (double)__builtin_nontemporal_load(&tL[(v * n + s) * n + b]);
        qR[v] = (double)__builtin_nontemporal_load(&tR[(v * n + s) * n + b]);
      }
      if (mp.bc[k] != 0) {
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
      numerical_flux<SYS, 2, FLUX>(qL, qR, k, mp, c, Fpt);
#pragma unroll
      for (int v = 0; v < NV; ++v) Fp[v] = wts * Fpt[v];
    }
    // Gauss sum over the 16 lanes of the group (fixed butterfly order)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double x = Fp[v];
      x += __shfl_xor(x, 8, 16);
      x += __shfl_xor(x, 4, 16);
      x += __shfl_xor(x, 2, 16);
      x += __shfl_xor(x, 1, 16);
      if (l == 0 && f_in) sF[f * NV + v] = x;
    }
  }
  __syncthreads();

  // update: one thread per tile cell
  const int cx = tid % TX, cy = tid / TX;
  unsigned int flags = 0;
  if (tid < TX * TY) {
    const int gi = x0 + cx, gj = y0 + cy;
    if (gi < nx && gj < ny) {
      const int64_t cell = gi + (int64_t)nx * gj;
      const double dt = *dt_dev;
      const double cxf = dt / mp.dx[0], cyf = dt / mp.dx[1];
      const int fxl = cx + (TX + 1) * cy, fxh = fxl + 1;
      const int fyl = NFX + cx + TX * cy, fyh = fyl + TX;
      double q[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double uu = u_in[(int64_t)v * ld + cell];
        uu -= cxf * (sF[fxh * NV + v] - sF[fxl * NV + v]);
        uu -= cyf * (sF[fyh * NV + v] - sF[fyl * NV + v]);
        u_out[(int64_t)v * ld + cell] = uu;
        q[v] = uu;
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (q[v] != q[v]) flags |= kFlagNan;
      if (!state_physical<SYS, DIM>(q, mp.gamma)) flags |= kFlagNonPhysical;
    }
  }
  block_report(0u, flags, hdr);
  (void)C;
}

template <int M, int SYS, typename TR, int FLUX = -1>
__global__ void __launch_bounds__(kBlock)
k_face2d(const TR* __restrict__ traces, const double* __restrict__ u_in,
         double* __restrict__ u_out, int64_t ld, const double* __restrict__ dt_dev,
         MeshParams mp, DevConsts c, WsHeader* hdr) {
  // tiles in the reverse of the cell kernel's order: the traces written last
  // are the ones still held in the caches when this kernel starts
  const int tx = (int)(gridDim.x - 1 - blockIdx.x), ty = (int)(gridDim.y - 1 - blockIdx.y);
  face2d_tile<M, SYS, TR, FLUX>(tx, ty, traces, u_in, u_out, ld, dt_dev, mp, c, hdr);
}

}  // namespace ader
