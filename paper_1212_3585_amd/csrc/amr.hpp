// Kernels of cell-by-cell AMR with local time stepping (Section 3) on the
// dense per-level representation (amr_plan.hpp): every level is an array over
// its whole index space with a status per cell; the work runs over per-level
// lists (active cells, virtual children, virtual mothers).
//
//   k_amr_cfl       block maxima of sum_k speed_k / dx_k over each level's
//                   active cells (the CFL rule, reading R1), all levels in
//                   one launch
//   k_amr_dt        level-0 step from all levels' maxima, level steps, clock
//   k_amr_average   virtual mothers = mean of their r^d children (eq. average)
//   k_amr_prepare   one launch per level substep for the averaging, the
//                   projection and the clearing of the finer level's memory,
//                   and the level's update of its previous substep (all but
//                   the last substep of a run defer it to this launch)
//   k_amr_weno_x    first WENO pass of the active cells, stencil indices from
//                   the dense grid; later passes and the predictor are the
//                   level-list kernels (level.hpp, predictor kernels)
//   k_amr_subavg    a regrid's new (and virtual) children: the average of
//                   the mother's reconstruction w_h over the child's sub-cell
//   k_fill_list     one value into listed cells of every variable (the
//                   memory of the virtual children before a level's substeps)
//   k_amr_cf_faces  the list of a level's coarse-fine faces and the kind of
//                   every face of its active cells (when the lists change)
//   k_amr_flux      face fluxes of the active cells, one group of lanes per
//                   (cell, axis), one lane per space-time point of the face;
//                   each face once (a cell's high faces, and its low faces
//                   not shared with an active cell of the level): same-level
//                   faces as on a uniform mesh; its first blocks take the
//                   listed coarse-fine faces, a group per face: a face to a
//                   virtual child (coarser neighbour) takes the coarse
//                   predictor at this face's Gauss points and this
//                   substep's time nodes and stores the flux in the virtual
//                   child's memory; a face to a virtual mother (finer
//                   neighbour) averages the memory of this cell's virtual
//                   children on that face (eq. memory.sum)
//   k_amr_apply     conservative update of the active cells from those fluxes
//                   (amr_apply_cell) where no other launch carries it: a
//                   finer level's updates ride in k_amr_prepare of its next
//                   substep and, after the last substep of a run, in the
//                   coarser level's k_amr_flux
#pragma once

#include "amr_plan.hpp"
#include "level.hpp"
#include "predict_wave.hpp"

namespace ader {

template <int DIM>
__device__ __forceinline__ void dense_coords(int64_t idx, const int (&n)[3], int (&c)[3]) {
  c[0] = (int)(idx % n[0]);
  c[1] = DIM > 1 ? (int)((idx / n[0]) % n[1]) : 0;
  c[2] = DIM > 2 ? (int)(idx / ((int64_t)n[0] * n[1])) : 0;
}

template <int DIM>
__device__ __forceinline__ int64_t dense_index(const int (&c)[3], const int (&n)[3]) {
  return c[0] + (int64_t)n[0] * (c[1] + (int64_t)n[1] * (DIM > 2 ? c[2] : 0));
}

__device__ __forceinline__ double nan_max_d(double a, double b) {
  return (b != b || b > a) ? b : a;  // a NaN wins, so it reaches dt
}

// The CFL block maxima of every level in one launch: level l takes nb
// blocks from block 'first' of the grid, and block lb of it writes
// partial[l kDtMaxBlocks + lb].
struct AmrCflLevel {
  const double* u = nullptr;
  const int32_t* act = nullptr;
  int64_t nact = 0;
  MeshParams mp{};
  int nb = 0;
  int first = 0;
};
struct AmrCflArgs {
  AmrCflLevel lv[kAmrMaxLevels];
  int nlev = 0;
};

template <int DIM, int SYS>
__global__ void __launch_bounds__(kBlock)
k_amr_cfl(AmrCflArgs args, double* __restrict__ partial) {
  constexpr int NV = NVars<SYS, DIM>::v;
  __shared__ double sw[kBlock / 64];
  int l = 0;  // the block's level (uniform in the block)
  while (l + 1 < args.nlev && (int)blockIdx.x >= args.lv[l + 1].first) ++l;
  const AmrCflLevel& L = args.lv[l];
  const int lb = (int)blockIdx.x - L.first;
  const double* __restrict__ u = L.u;
  const int32_t* __restrict__ act = L.act;
  const int64_t nact = L.nact;
  const MeshParams& mp = L.mp;
  const double adv[3] = {mp.adv[0], mp.adv[1], mp.adv[2]};
  double m = 0.0;
  for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < nact; i += (int64_t)L.nb * kBlock) {
    const int64_t cell = act[i];
    double q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = u[v * mp.ld + cell];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      double f[NV], sp;
      phys_flux_dir<SYS, DIM>(q, k, mp.gamma, mp.ch, adv, f, sp);
      s += sp / mp.dx[k];
    }
    m = nan_max_d(m, s);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = nan_max_d(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sw[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) b = nan_max_d(b, sw[i]);
    partial[l * kDtMaxBlocks + lb] = b;
  }
}

// One wavefront (64 threads): the level-0 step of the AMR run and the level
// steps.  The lanes read the levels' block maxima in parallel and combine
// them with a butterfly (a maximum in any order, a NaN winning, so that it
// reaches dt); lane 0 finishes.  (A template so that the header can be
// included by several units.)
template <int TAG>
__global__ void k_amr_dt(const double* __restrict__ partial, AmrDtArgs a, AmrClock* clock,
                         WsHeader* hdr) {
  if (blockIdx.x != 0) return;
  const int lane = threadIdx.x;
  double best = 1.0 / 0.0;
  double rl = 1.0;  // r^l
  for (int l = 0; l < a.nlev; ++l) {
    if (a.nb[l] > 0) {  // uniform
      double m = 0.0;
      for (int i = lane; i < a.nb[l]; i += 64) m = nan_max_d(m, partial[l * kDtMaxBlocks + i]);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = nan_max_d(m, __shfl_xor(m, o, 64));
      const double cand = rl * a.cfl / m;
      best = (cand != cand || cand < best) ? cand : best;
    }
    rl *= a.r;
  }
  if (lane != 0) return;
  const double t = clock->t;
  const double rest = clock->t_end - t;
  double dt = rest < best ? rest : best;
  if (!(dt > 0.0)) dt = dt != dt ? dt : 0.0;  // finished runs take empty steps
  if (dt != dt) atomicOr(&hdr->status, kFlagNan);
  clock->dt[0] = dt;
  for (int l = 1; l < a.nlev; ++l) clock->dt[l] = clock->dt[l - 1] / a.r;
  clock->t = t + dt;
  clock->steps = clock->steps + 1;
}

template <int TAG>
__global__ void __launch_bounds__(kBlock)
k_fill_list(double* __restrict__ u, int64_t ld, int nv, const int32_t* __restrict__ list,
            int64_t n, double value) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * nv) return;
  u[(t / n) * ld + list[t % n]] = value;
}

// Children from their mothers' reconstruction at a regrid: target i of the
// fine level (dense index targets[i]) takes, for every variable,
//   sum_p  prod_k sub_avg[a_k][p_k]  w_h[slot][v][p],   a_k = c_k mod r,
// with w_h of mother slot tslot[i] in the layout of the WENO passes
// ([slot][v][px + n py + n^2 pz]).  Contracted along x, then y, then z.
template <int DIM, int M, int NV>
__global__ void __launch_bounds__(kBlock)
k_amr_subavg(double* __restrict__ u, int64_t ld, const int32_t* __restrict__ targets,
             const int32_t* __restrict__ tslot, int64_t nt, int n0, int n1, int n2,
             const double* __restrict__ wh, AmrConsts ac) {
  constexpr int n = M + 1;
  constexpr int NS = Pow<n, DIM>::v;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nt * NV) return;
  const int v = (int)(t % NV);
  const int64_t i = t / NV;
  const int nn[3] = {n0, n1, n2};
  int cc[3];
  dense_coords<DIM>(targets[i], nn, cc);
  const int r = ac.r;
  if (tslot[i] < 0) return;  // no reconstructed mother (never for a consistent mesh)
  const double* w = wh + ((int64_t)tslot[i] * NV + v) * NS;
  double acc_z = 0.0;
#pragma unroll
  for (int pz = 0; pz < (DIM > 2 ? n : 1); ++pz) {
    double acc_y = 0.0;
#pragma unroll
    for (int py = 0; py < (DIM > 1 ? n : 1); ++py) {
      double acc_x = 0.0;
#pragma unroll
      for (int px = 0; px < n; ++px)
        acc_x += ac.sub_avg[cc[0] % r][px] * w[px + n * (py + n * pz)];
      acc_y += DIM > 1 ? ac.sub_avg[cc[1] % r][py] * acc_x : acc_x;
    }
    acc_z += DIM > 2 ? ac.sub_avg[cc[2] % r][pz] * acc_y : acc_y;
  }
  u[(int64_t)v * ld + targets[i]] = acc_z;
}

template <int DIM, int NV>
__global__ void __launch_bounds__(kBlock)
k_amr_average(double* __restrict__ uc, int64_t ldc, const double* __restrict__ uf, int64_t ldf,
              const int32_t* __restrict__ vm, int64_t nvm, int nc0, int nc1, int nc2, int nf0,
              int nf1, int nf2, int r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nvm) return;
  const int nc[3] = {nc0, nc1, nc2}, nf[3] = {nf0, nf1, nf2};
  const int64_t cell = vm[i];
  int c[3];
  dense_coords<DIM>(cell, nc, c);
  const int nchild = DIM == 2 ? r * r : r * r * r;
  double sum[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) sum[v] = 0.0;
  for (int a = 0; a < nchild; ++a) {
    int f[3] = {c[0] * r + a % r, DIM > 1 ? c[1] * r + (a / r) % r : 0,
                DIM > 2 ? c[2] * r + a / (r * r) : 0};
    const int64_t child = dense_index<DIM>(f, nf);
#pragma unroll
    for (int v = 0; v < NV; ++v) sum[v] += uf[v * ldf + child];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) uc[v * ldc + cell] = sum[v] / nchild;
}

// Value of a coarse cell's predictor q (nodal, [v][s][pz][py][px]) at the
// tensor point with per-axis basis weights wax[axis][p] and time weights wt[s].
template <int DIM, int M, int NV, typename R>
__device__ __forceinline__ void eval_predictor(const R* __restrict__ q, const double (&wt)[4],
                                               const double (&wax)[3][4], double (&out)[NV]) {
  constexpr int n = M + 1;
  constexpr int NS = Pow<n, DIM>::v;
  constexpr int NST = NS * n;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < n; ++s) {
      double sp = 0.0;
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        const int px = a % n, py = (a / n) % n, pz = a / (n * n);
        double w = wax[0][px] * wax[1][py];
        if (DIM == 3) w *= wax[2][pz];
        sp += w * (double)q[v * NST + a + NS * s];
      }
      acc += wt[s] * sp;
    }
    out[v] = acc;
  }
}

// The work of one level substep before its reconstruction, in one launch:
//   blocks [0, nab)             the level's conservative update of its
//                               previous substep (amr_apply_cell), when the
//                               caller defers it to this launch: it writes
//                               the active cells, which nothing below reads
//                               or writes;
//   then, counting threads from block nab:
//   threads [0, nvm)            virtual mothers of the level = mean of their
//                               children (eq. average);
//   threads [nvm, nvm + nvc)    virtual children of the level = sub-cell
//                               average of the mother's predictor at the
//                               substep's mother-local time (Section 3.1.3);
//   the rest                    the finer level's memory at its virtual
//                               children cleared (its r substeps follow).
// The sets are disjoint; nothing reads what another writes.
struct AmrPrepArgs {
  double* u;
  int64_t ld;
  int n[3];
  const int32_t* vm;
  int64_t nvm;
  const int32_t* vc;
  int64_t nvc;
  const double* uf;  // finer level (averages), null on the finest level
  int64_t ldf;
  int nf[3];
  const int32_t* pos_c;  // coarser level (projection), null on level 0
  const void* qh_c;
  int nc[3];
  double* mem_f;          // finer level's memory, its virtual children vcf
  const int32_t* vcf;
  int64_t nvcf;
  int sub;
};

// First WENO pass (along x) of the active cells; the (2M+1)^d stencil is
// addressed on the dense grid with the boundary maps.  Output layout as
// k_level_weno_pass<K = 0>.
template <int DIM, int M, int NV>
__global__ void __launch_bounds__(kBlock)
k_amr_weno_x(const double* __restrict__ u, int64_t ld, const int32_t* __restrict__ act,
             int64_t nact, MeshParams mp, double* __restrict__ dst, DevConsts c) {
  constexpr int n = M + 1;
  constexpr int S = 2 * M + 1;
  constexpr int LINES = Pow<S, DIM - 1>::v;
  constexpr int OUT = n * LINES;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nact * NV * LINES) return;
  const int line = (int)(t % LINES);
  const int64_t pv = t / LINES;
  const int v = (int)(pv % NV);
  const int64_t p = pv / NV;
  int cc[3];
  dense_coords<DIM>(act[p], mp.n, cc);
  const int oy = line % S, oz = line / S;
  const int gy = DIM > 1 ? bc_map(cc[1] + oy - M, mp.n[1], mp.bc[1]) : 0;
  const int gz = DIM > 2 ? bc_map(cc[2] + oz - M, mp.n[2], mp.bc[2]) : 0;
  const int64_t row = (int64_t)mp.n[0] * (gy + (int64_t)mp.n[1] * gz);
  double vals[S];
#pragma unroll
  for (int o = 0; o < S; ++o)
    vals[o] = u[(int64_t)v * ld + row + bc_map(cc[0] + o - M, mp.n[0], mp.bc[0])];
  double w[n];
  weno_line<M>(vals, c, w);
  double* dp = dst + pv * OUT;
#pragma unroll
  for (int q = 0; q < n; ++q) dp[q + n * line] = w[q];
}

struct AmrUpdArgs {
  double* u;
  const int8_t* st;
  const int32_t* pos;
  const int32_t* act;
  int64_t nact;
  const void* qh;
  const int32_t* pos_c;  // coarser level (null on level 0)
  const void* qh_c;
  int nc[3];
  double* mem;            // this level's memory [DIM][2][NV][ncells] (null on level 0)
  const double* mem_f;    // finer level's memory (null on the finest level)
  int nf[3];
  int64_t ldf;
  const double* dt;
  int sub;
  int r;
  // kind of each face of the active cells, fc[(2 k + side) nact + i]
  // (k_amr_cf_faces): >= 0 the list position of the same-level active
  // neighbour, kFaceOut a transmissive boundary, kFaceCoarseFine a listed
  // coarse-fine face (the first blocks of k_amr_flux), kFaceBad no flux (an
  // index outside the lists)
  const int32_t* fc;
};

constexpr int32_t kFaceOut = -1, kFaceCoarseFine = -2, kFaceBad = -3;

// Shape of the face-flux kernel: a group of G lanes per (cell, axis k); lane
// g < NPT of a group owns space-time point (s = g / NT, tb = g % NT) of the
// face.  CPB cells per block.
// PACK (2D M = 2): a face's nine points take nine lanes and a wavefront
// holds three cells (54 lanes), where power-of-two groups of 16 hold two;
// the lanes after the last whole cell (or group) idle.
template <int DIM, int M, int TB = kBlock>
struct AmrFluxShape {
  static constexpr int n = M + 1;
  static constexpr int NT = Pow<n, DIM - 1>::v;  // transverse nodes of a face
  static constexpr int NPT = n * NT;              // space-time points of a face
  static constexpr int P2 = NPT <= 4 ? 4 : (NPT <= 8 ? 8 : (NPT <= 16 ? 16 : (NPT <= 32 ? 32 : 64)));
  static constexpr bool PACK = DIM == 2 && P2 != NPT && NPT > 4;
  static constexpr int G = PACK ? NPT : P2;       // lanes per face
  static constexpr int LPC = DIM * G;             // lanes per cell
  static constexpr int CPW = 64 / LPC;            // cells per wavefront (PACK)
  static constexpr int CPB = PACK ? CPW * (TB / 64) : (LPC >= TB ? 1 : TB / LPC);
  static constexpr int BLOCK = PACK ? TB : CPB * LPC;
  static constexpr int GPB = PACK ? (64 / G) * (TB / 64) : BLOCK / G;  // listed faces per block
};

// Kind of the face of active cell cc on (axis k, side): 0 an active cell of
// the same level (its list position in *pn), 1 outflow through a
// transmissive boundary, 2 a virtual child (the coarse mother's list
// position in *pn, the child's offsets in off), 3 a virtual mother (finer
// neighbour), -1 no flux (an index outside the lists: flagged).
template <int DIM>
__device__ __forceinline__ int amr_face_kind(const AmrUpdArgs& a, const MeshParams& mp,
                                             const int (&cc)[3], int k, int side, int64_t* nb,
                                             int32_t* pn, int (&off)[3]) {
  const int raw = cc[k] + (side ? 1 : -1);
  if ((raw < 0 || raw >= mp.n[k]) && mp.bc[k] != 0) return 1;
  int nbc[3] = {cc[0], cc[1], cc[2]};
  nbc[k] = bc_map(raw, mp.n[k], mp.bc[k]);
  *nb = dense_index<DIM>(nbc, mp.n);
  const int8_t s = a.st[*nb];
  if (s == kActive) {
    *pn = a.pos[*nb];
    return *pn >= 0 ? 0 : -1;
  }
  if (s == kVChild && a.pos_c) {
    int m[3];
    for (int ax = 0; ax < 3; ++ax) {
      m[ax] = nbc[ax] / a.r;
      off[ax] = nbc[ax] % a.r;
    }
    *pn = a.pos_c[dense_index<DIM>(m, a.nc)];
    return *pn >= 0 ? 2 : -1;
  }
  if (s == kVMother && a.mem_f) return 3;
  return -1;
}

// Flux of one face of active cell i (axis k, side) of the given kind (see
// amr_face_kind), by a group of G lanes, lane g owning space-time point
// (s = g / NT, tb = g % NT); the face average goes to
// fbuf[(i * 2 DIM + 2 k + side) * NV + v].  A face to a virtual child also
// adds its flux to the child's memory.  The group takes one path.
// trc: the group's NV n NT doubles of LDS for a face to a virtual child
// (unused by the other kinds).
template <int DIM, int M, int SYS, typename R, int G, int FLUX>
__device__ __forceinline__ void amr_face_flux(const AmrUpdArgs& a, const MeshParams& mp,
                                              const DevConsts& c, const AmrConsts& ac,
                                              double* __restrict__ fbuf, int64_t i,
                                              const int (&cc)[3], int k, int side, int type,
                                              int64_t nb, int32_t pn, const int (&off)[3],
                                              int g, double* __restrict__ trc,
                                              double* __restrict__ gsum) {
  constexpr int n = M + 1;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int NS = Pow<n, DIM>::v;
  constexpr int NST = NS * n;
  constexpr int NT = Pow<n, DIM - 1>::v;
  constexpr int NPT = n * NT;
  constexpr int FS = 2 * DIM;
  double F[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = 0.0;
  if (type == 3) {
    // this lane's share of the memory of the cell's virtual children on the face
    const int nsub = DIM == 2 ? a.r : a.r * a.r;
    for (int j = g; j < nsub; j += G) {
      int ch[3] = {0, 0, 0};
      int t = 0;
      for (int ax = 0; ax < DIM; ++ax) {
        if (ax == k) {
          ch[ax] = cc[ax] * a.r + (side ? a.r - 1 : 0);
        } else {
          const int aj = DIM == 2 ? j : (t == 0 ? j / a.r : j % a.r);
          ch[ax] = cc[ax] * a.r + aj;
          ++t;
        }
      }
      const int64_t chd = dense_index<DIM>(ch, a.nf);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        F[v] += a.mem_f[((int64_t)(k * 2 + side) * NV + v) * a.ldf + chd];
    }
  } else {
    // tangential axes of the face, in increasing order
    const int ta0 = k == 0 ? 1 : 0, ta1 = k == 2 ? 1 : 2;
    if (type == 2) {
      // The coarse predictor on the face: contracted along the normal (coarse
      // basis at the virtual child's face) and in time (coarse basis at this
      // substep's time nodes) once per face, the group's lanes sharing the
      // NV n NT values [v][s][tangential nodes] through LDS; each lane then
      // contracts the tangential axes at its own Gauss point.
      const R* qc = static_cast<const R*>(a.qh_c) + (int64_t)pn * NV * NST;
      const int sk = k == 0 ? 1 : (k == 1 ? n : n * n);
      const int s0 = ta0 == 0 ? 1 : (ta0 == 1 ? n : n * n);
      const int s1 = ta1 == 1 ? n : n * n;
      for (int idx = g; idx < NV * NPT; idx += G) {
        const int v = idx / NPT, s = (idx / NT) % n, tb = idx % NT;
        const int base = (tb % n) * s0 + (DIM == 3 ? (tb / n) * s1 : 0);
        double acc = 0.0;
#pragma unroll
        for (int pt = 0; pt < n; ++pt) {
          double sp = 0.0;
#pragma unroll
          for (int pn = 0; pn < n; ++pn)
            sp += ac.at_face[off[k]][1 - side][pn] *
                  (double)qc[v * NST + NS * pt + base + pn * sk];
          acc += ac.at_nodes[a.sub][s][pt] * sp;
        }
        trc[idx] = acc;
      }
      wave_lds_order();
    }
    if (g < NPT) {
      const int s = g / NT, tb = g % NT;
      double qm[NV], qp[NV];
      cell_trace<DIM, M, NV, R>(static_cast<const R*>(a.qh) + i * NV * NST, k, side, tb, s, c,
                                qm);
      if (type == 0) {
        cell_trace<DIM, M, NV, R>(static_cast<const R*>(a.qh) + (int64_t)pn * NV * NST, k,
                                  1 - side, tb, s, c, qp);
      } else if (type == 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) qp[v] = qm[v];
      } else {
        // coarse predictor at this face point and time node
        double w0[4], w1[4];
#pragma unroll
        for (int p = 0; p < n; ++p) {
          w0[p] = ac.at_nodes[off[ta0]][tb % n][p];
          w1[p] = DIM == 3 ? ac.at_nodes[off[ta1]][tb / n][p] : 1.0;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double* tv = trc + v * NPT + s * NT;
          double acc = 0.0;
#pragma unroll
          for (int p1 = 0; p1 < (DIM == 3 ? n : 1); ++p1) {
            double sp = 0.0;
#pragma unroll
            for (int p0 = 0; p0 < n; ++p0) sp += w0[p0] * tv[p0 + n * p1];
            acc += w1[p1] * sp;
          }
          qp[v] = acc;
        }
      }
      double Fpt[NV];
      if (side)
        numerical_flux<SYS, DIM, FLUX>(qm, qp, k, mp, c, Fpt);
      else
        numerical_flux<SYS, DIM, FLUX>(qp, qm, k, mp, c, Fpt);
      double wtp = c.w[s];
      {
        const int tt[2] = {tb % n, tb / n};
        for (int dd = 0; dd < DIM - 1; ++dd) wtp *= c.w[tt[dd]];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = wtp * Fpt[v];
    }
  }
  if constexpr ((G & (G - 1)) == 0) {
    // group sum by a fixed butterfly
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] += __shfl_xor(F[v], o, 64);
  } else {
    // a group of G lanes that is not a power of two: its first lane sums
    // the lanes' values in order, through the wavefront's LDS (gsum, NV
    // doubles per lane)
    const int ln = threadIdx.x & 63;
    wave_lds_order();
#pragma unroll
    for (int v = 0; v < NV; ++v) gsum[ln * NV + v] = F[v];
    wave_lds_order();
    if (g == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
        for (int j = 0; j < G; ++j) acc += gsum[(ln + j) * NV + v];
        F[v] = acc;
      }
    }
  }
  if (g == 0) {
    if (type == 3) {
      const double inv = 1.0 / (DIM == 2 ? (double)(a.r * a.r) : (double)(a.r * a.r * a.r));
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] *= inv;
    }
    double* fo = fbuf + (i * FS + 2 * k + side) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) fo[v] = F[v];
    if (type == 2) {  // the face flux also goes to the coarse cell's memory
#pragma unroll
      for (int v = 0; v < NV; ++v)
        a.mem[((int64_t)(k * 2 + (1 - side)) * NV + v) * mp.ld + nb] += F[v];
    }
  }
}

// Flux of listed coarse-fine face e (a record of k_amr_cf_faces) by a group
// of G lanes; trc is the group's LDS (see amr_face_flux).
template <int DIM, int M, int SYS, typename R, int G, int FLUX>
__device__ __forceinline__ void amr_cf_entry(const AmrUpdArgs& a, const MeshParams& mp,
                                             const DevConsts& c, const AmrConsts& ac,
                                             const int32_t* __restrict__ list, int64_t e,
                                             double* __restrict__ fbuf, int g,
                                             double* __restrict__ trc, double* __restrict__ gsum) {
  const int4 rec = reinterpret_cast<const int4*>(list)[e];
  const int32_t t = rec.x;
  const int64_t i = t / (2 * DIM);
  const int k = (t % (2 * DIM)) >> 1, side = t & 1;
  int cc[3] = {0, 0, 0};
  if constexpr (DIM == 2) {
    const int type = rec.y & 0xFF;
    const int off[3] = {(rec.y >> 8) & 0xFF, (rec.y >> 16) & 0xFF, (rec.y >> 24) & 0xFF};
    if (type == 3) dense_coords<DIM>(a.act[i], mp.n, cc);  // the face's fine children
    amr_face_flux<DIM, M, SYS, R, G, FLUX>(a, mp, c, ac, fbuf, i, cc, k, side, type, rec.z,
                                           rec.w, off, g, trc, gsum);
  } else {
    // 3D: deriving the kind again from the lists measured faster with the
    // fp64 predictor (93.5 against 118.5 us per launch on the 3D blast;
    // 65 against 60 us with the fp32 one)
    dense_coords<DIM>(a.act[i], mp.n, cc);
    int64_t nb = 0;
    int32_t pn = -1;
    int off[3] = {0, 0, 0};
    const int type = amr_face_kind<DIM>(a, mp, cc, k, side, &nb, &pn, off);
    if (type < 2) return;
    amr_face_flux<DIM, M, SYS, R, G, FLUX>(a, mp, c, ac, fbuf, i, cc, k, side, type, nb, pn,
                                           off, g, trc, gsum);
  }
}

// Conservative update of active cell i (eq. finite_vol) from the face
// fluxes of k_amr_flux: the low face on axis k is the low neighbour's high
// face when that neighbour is an active cell of the same level.
template <int DIM, int SYS>
__device__ __forceinline__ void amr_apply_cell(const AmrUpdArgs& a, const MeshParams& mp,
                                               const double* __restrict__ fbuf, int64_t i,
                                               unsigned int& flags) {
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int FS = 2 * DIM;
  const int64_t ld = mp.ld;
  const int64_t cell = a.act[i];
  const double dt = *a.dt;
  double q[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = a.u[v * ld + cell];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int32_t code = a.fc[(2 * k) * a.nact + i];  // the low face
    const double* fhi = fbuf + (i * FS + 2 * k + 1) * NV;
    const double* flo = code >= 0 ? fbuf + ((int64_t)code * FS + 2 * k + 1) * NV
                                  : fbuf + (i * FS + 2 * k) * NV;
    if (code == kFaceBad) flags |= kFlagBadIndex;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      q[v] -= (dt / mp.dx[k]) * (fhi[v] - (code == kFaceBad ? 0.0 : flo[v]));
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    a.u[v * ld + cell] = q[v];
    if (q[v] != q[v]) flags |= kFlagNan;
  }
  if (!state_physical<SYS, DIM>(q, mp.gamma)) flags |= kFlagNonPhysical;
}

// Face fluxes of the active cells: each cell computes its high face on every
// axis, and its low face where the low neighbour is not an active cell of
// the same level (that face is the neighbour's high face), so every face is
// evaluated once.  This kernel takes the faces to active cells of the level
// and through the boundary, a group of lanes per (cell, axis); the
// coarse-fine faces (virtual children and virtual mothers) are listed once
// per mesh (k_amr_cf_faces) and done by the first ncb blocks of the same
// launch, a group of G lanes per listed face (amr_cf_entry), so that their
// gathers overlap the bulk of the same-level faces and the level substep
// needs no launch of its own for them.  In 2D the next nab blocks apply the
// finer level's update of the last substep of its run (ua, deferred to this
// launch): it writes that level's active cells, which this level's faces do
// not read (they read its memory, written by its face kernel).  In 3D that
// path held the kernel at 98 instead of 73 VGPRs, so nab is 0 there.  Deriving their kinds in the
// same-level path instead took 167 instead of 78 VGPRs at 3D M = 2 fp64.
template <int DIM, int M, int SYS, typename R, int TB = kBlock, int FLUX = -1>
__global__ void __launch_bounds__((AmrFluxShape<DIM, M, TB>::BLOCK))
k_amr_flux(AmrUpdArgs a, MeshParams mp, DevConsts c, AmrConsts ac, double* __restrict__ fbuf,
           WsHeader* hdr, const int32_t* __restrict__ cfl, int64_t ncf, unsigned ncb,
           AmrUpdArgs ua, MeshParams ump, const double* __restrict__ ufbuf, WsHeader* uhdr,
           unsigned nab) {
  using Sh = AmrFluxShape<DIM, M, TB>;
  constexpr int G = Sh::G;
  constexpr int NV = NVars<SYS, DIM>::v;
  const int tid = threadIdx.x;
  const int ln = tid & 63;
  // PACK: the wavefront's group sums through its LDS
  __shared__ double s_gsum[Sh::PACK ? Sh::BLOCK : 1][Sh::PACK ? NV : 1];
  double* gsum = Sh::PACK ? &s_gsum[tid - ln][0] : nullptr;
  if (blockIdx.x < ncb) {  // coarse-fine faces (uniform in the block)
    __shared__ double s_trc[Sh::GPB][NV * Sh::NPT];
    const int grp = Sh::PACK ? (tid >> 6) * (64 / G) + ln / G : tid / G;
    const bool grp_ok = !Sh::PACK || ln / G < 64 / G;
    const int64_t e = (int64_t)blockIdx.x * Sh::GPB + grp;
    if (grp_ok && e < ncf)  // uniform in the group
      amr_cf_entry<DIM, M, SYS, R, G, FLUX>(a, mp, c, ac, cfl, e, fbuf,
                                            Sh::PACK ? ln % G : tid % G, s_trc[grp], gsum);
    return;
  }
  if constexpr (DIM == 2) {
    if (blockIdx.x < ncb + nab) {  // the finer level's deferred update (uniform in the block)
      const int64_t ia = (int64_t)(blockIdx.x - ncb) * Sh::BLOCK + tid;
      unsigned int uflags = 0;
      if (ia < ua.nact) amr_apply_cell<DIM, SYS>(ua, ump, ufbuf, ia, uflags);
      block_report(0u, uflags, uhdr);
      return;
    }
  }
  // (cell in the block, axis, lane in the face group)
  const int lt = Sh::PACK ? ln : tid;
  const bool lane_ok = !Sh::PACK || lt / Sh::LPC < Sh::CPW;
  const int cs = Sh::PACK ? (tid >> 6) * Sh::CPW + (lane_ok ? lt / Sh::LPC : 0) : tid / Sh::LPC;
  const int k = (lt % Sh::LPC) / G;
  const int g = lt % G;
  // groups in the reverse of the predictor's order (2D: predictor forward;
  // 3D: predictor reversed): the q_h written last are read first, while
  // still cached
  const int64_t bm = (int64_t)blockIdx.x - ncb - nab, nbm = (int64_t)gridDim.x - ncb - nab;
  const int64_t blk = DIM == 2 ? nbm - 1 - bm : bm;
  const int64_t i = blk * Sh::CPB + cs;
  const bool valid = lane_ok && i < a.nact;
  unsigned int flags = 0;
  const int cc[3] = {0, 0, 0};  // not read for same-level and boundary faces
  const int off[3] = {0, 0, 0};
  for (int side = 1; side >= 0; --side) {
    const int32_t code = valid ? a.fc[(2 * k + side) * a.nact + i] : kFaceCoarseFine;
    if (code == kFaceBad) flags |= kFlagBadIndex;
    // uniform in the group: the low face of an active neighbour is its high
    // face; coarse-fine faces are the listed ones of the first blocks
    if (code == kFaceCoarseFine || code == kFaceBad || (side == 0 && code >= 0)) continue;
    const int type = code >= 0 ? 0 : 1;
    amr_face_flux<DIM, M, SYS, R, G, FLUX>(a, mp, c, ac, fbuf, i, cc, k, side, type, 0,
                                           code >= 0 ? code : -1, off, g, nullptr, gsum);
  }
  block_report(0u, flags, hdr);
}

// The coarse-fine faces of a level's active cells (kinds 2 and 3 of
// amr_face_kind), built when the level's lists change, as records of four
// int32 (kAmrCfRecord): the entry i * 2 DIM + 2 k + side, the kind with the
// child's sub-cell offsets (kind | off_x << 8 | off_y << 16 | off_z << 24),
// the neighbour's dense index and its list position.  The order of the
// records does not matter: each face's flux is computed on its own and
// written to its own slots.
// The same pass also writes every face's kind for the per-step kernels
// (AmrUpdArgs::fc), so that they read one code instead of gathering the
// neighbour's status and list position.
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_amr_cf_faces(AmrUpdArgs a, MeshParams mp, int32_t* __restrict__ list, int* __restrict__ count,
               int32_t* __restrict__ fc) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= a.nact * 2 * DIM) return;
  const int64_t i = t / (2 * DIM);
  const int f = (int)(t % (2 * DIM));
  int cc[3] = {0, 0, 0};
  dense_coords<DIM>(a.act[i], mp.n, cc);
  int64_t nb = 0;
  int32_t pn = -1;
  int off[3] = {0, 0, 0};
  const int type = amr_face_kind<DIM>(a, mp, cc, f >> 1, f & 1, &nb, &pn, off);
  if (type >= 2) {
    int32_t* rec = list + (int64_t)atomicAdd(count, 1) * kAmrCfRecord;
    rec[0] = (int32_t)t;
    rec[1] = type | (off[0] << 8) | (off[1] << 16) | (off[2] << 24);
    rec[2] = (int32_t)nb;
    rec[3] = pn;
  }
  fc[f * a.nact + i] = type == 0 ? pn : (type == 1 ? kFaceOut : (type >= 2 ? kFaceCoarseFine
                                                                           : kFaceBad));
}

template <int DIM, int SYS>
__global__ void __launch_bounds__(kBlock)
k_amr_apply(AmrUpdArgs a, MeshParams mp, const double* __restrict__ fbuf, WsHeader* hdr) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned int flags = 0;
  if (i < a.nact) amr_apply_cell<DIM, SYS>(a, mp, fbuf, i, flags);
  block_report(0u, flags, hdr);
}

// The launch of one level substep before its reconstruction (AmrPrepArgs).
template <int DIM, int M, int SYS, typename R>
__global__ void __launch_bounds__(kBlock)
k_amr_prepare(AmrPrepArgs a, AmrConsts ac, WsHeader* hdr, AmrUpdArgs ua, MeshParams ump,
              const double* __restrict__ fbuf, unsigned nab) {
  constexpr int n = M + 1;
  constexpr int NV = NVars<SYS, DIM>::v;
  constexpr int NST = Pow<n, DIM + 1>::v;
  unsigned int flags = 0;
  if (blockIdx.x < nab) {  // the level's update of its previous substep (uniform in the block)
    const int64_t ia = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (ia < ua.nact) amr_apply_cell<DIM, SYS>(ua, ump, fbuf, ia, flags);
    block_report(0u, flags, hdr);
    return;
  }
  const int64_t i = (int64_t)(blockIdx.x - nab) * kBlock + threadIdx.x;
  const int r = ac.r;
  if (i < a.nvm) {
    const int64_t cell = a.vm[i];
    int c[3];
    dense_coords<DIM>(cell, a.n, c);
    const int nchild = DIM == 2 ? r * r : r * r * r;
    double sum[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sum[v] = 0.0;
    for (int b = 0; b < nchild; ++b) {
      int f[3] = {c[0] * r + b % r, DIM > 1 ? c[1] * r + (b / r) % r : 0,
                  DIM > 2 ? c[2] * r + b / (r * r) : 0};
      const int64_t child = dense_index<DIM>(f, a.nf);
#pragma unroll
      for (int v = 0; v < NV; ++v) sum[v] += a.uf[v * a.ldf + child];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) a.u[v * a.ld + cell] = sum[v] / nchild;
  } else if (i < a.nvm + a.nvc) {
    const int64_t cell = a.vc[i - a.nvm];
    int c[3], m[3], o[3];
    dense_coords<DIM>(cell, a.n, c);
    for (int k = 0; k < 3; ++k) {
      m[k] = c[k] / r;
      o[k] = c[k] % r;
    }
    const int32_t mp = a.pos_c[dense_index<DIM>(m, a.nc)];
    if (mp < 0) {
      flags |= kFlagBadIndex;  // a virtual child whose mother is not active
    } else {
      double wt[4], wax[3][4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        wt[p] = p < n ? ac.at_sub[a.sub][p] : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) wax[k][p] = p < n ? ac.sub_avg[o[k]][p] : 0.0;
      }
      double val[NV];
      eval_predictor<DIM, M, NV, R>(static_cast<const R*>(a.qh_c) + (int64_t)mp * NV * NST, wt,
                                    wax, val);
#pragma unroll
      for (int v = 0; v < NV; ++v) a.u[v * a.ld + cell] = val[v];
    }
  } else {
    const int64_t j = i - a.nvm - a.nvc;
    constexpr int E = 2 * DIM * NV;  // memory entries per cell
    if (j < a.nvcf * E) a.mem_f[(j / a.nvcf) * a.ldf + a.vcf[j % a.nvcf]] = 0.0;
  }
  block_report(0u, flags, hdr);
}

}  // namespace ader
