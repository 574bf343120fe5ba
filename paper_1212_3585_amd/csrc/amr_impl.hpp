// Launchers of the AMR kernels for one (dimension, degree, system, predictor
// precision).
#pragma once

#include <type_traits>

#include "amr.hpp"
#include "predict_mfma.hpp"
#include "predict_wave.hpp"
#include "weno3d.hpp"

namespace ader {

inline unsigned amr_blocks(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : b);
}

template <int DIM, int M, int SYS, typename R>
class AmrImpl final : public AmrImplBase {
  static constexpr int n = M + 1;
  static constexpr int S = 2 * M + 1;
  static constexpr int NV = NVars<SYS, DIM>::v;

 public:
  size_t qh_elem_size() const override { return sizeof(R); }
  size_t weno_scratch_per_cell() const override {
    return (size_t)NV * (n * Pow<S, DIM - 1>::v + (DIM == 3 ? n * n * S : 0));
  }
  size_t wh_per_cell() const override { return (size_t)NV * Pow<n, DIM>::v; }
  size_t dense_weno_per_cell() const override { return DIM == 3 ? (size_t)NV * (n + n * n) : 0; }
  size_t fbuf_per_cell() const override { return (size_t)2 * DIM * NV; }

  hipError_t cfl(const AmrLevel* lv, int nlev, double* partial, const int* nb,
                 hipStream_t st) const override {
    AmrCflArgs args;
    int blocks = 0;
    for (int l = 0; l < nlev; ++l) {
      AmrCflLevel& L = args.lv[l];
      L.u = lv[l].u;
      L.act = lv[l].act;
      L.nact = lv[l].nact;
      L.mp = lv[l].mp;
      L.nb = lv[l].nact > 0 ? nb[l] : 0;
      L.first = blocks;
      blocks += L.nb;
    }
    args.nlev = nlev;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_amr_cfl<DIM, SYS>), dim3(blocks), dim3(kBlock), 0, st, args, partial);
    return hipGetLastError();
  }

  hipError_t average(const AmrLevel& c, const AmrLevel& f, int r, hipStream_t st) const override {
    if (c.nvm == 0) return hipSuccess;
    hipLaunchKernelGGL((k_amr_average<DIM, NV>), dim3(amr_blocks(c.nvm)), dim3(kBlock), 0, st,
                       c.u, c.ncells, f.u, f.ncells, c.vm, c.nvm, c.n[0], c.n[1], c.n[2],
                       f.n[0], f.n[1], f.n[2], r);
    return hipGetLastError();
  }

  hipError_t prepare(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                     const AmrConsts& ac, int sub, const double* apply_dt,
                     hipStream_t st) const override {
    AmrPrepArgs a{};
    a.u = lv.u;
    a.ld = lv.ncells;
    for (int k = 0; k < 3; ++k) a.n[k] = lv.n[k];
    if (fine) {
      a.vm = lv.vm;
      a.nvm = lv.nvm;
      a.uf = fine->u;
      a.ldf = fine->ncells;
      for (int k = 0; k < 3; ++k) a.nf[k] = fine->n[k];
      a.mem_f = fine->mem;
      a.vcf = fine->vc;
      a.nvcf = fine->nvc;
    }
    if (coarse) {
      a.vc = lv.vc;
      a.nvc = lv.nvc;
      a.pos_c = coarse->pos;
      a.qh_c = coarse->qh;
      for (int k = 0; k < 3; ++k) a.nc[k] = coarse->n[k];
    }
    a.sub = sub;
    const int64_t total = a.nvm + a.nvc + a.nvcf * 2 * DIM * NV;
    // the level's deferred update of its previous substep in the first blocks
    const AmrUpdArgs ua = upd_args(lv, coarse, fine, apply_dt, sub, ac);
    const unsigned nab = apply_dt && lv.nact > 0 ? amr_blocks(lv.nact) : 0u;
    const unsigned npb = (unsigned)((total + kBlock - 1) / kBlock);
    if (nab + npb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_amr_prepare<DIM, M, SYS, R>), dim3(nab + npb), dim3(kBlock), 0, st, a,
                       ac, lv.hdr, ua, lv.mp, (const double*)lv.fbuf, nab);
    return hipGetLastError();
  }

  // 2D fp64: the matrix-core predictor with the fused reconstruction (fixed
  // 256-thread blocks).  The dense wave-local predictor (seven cells of nine
  // lanes per wavefront at M = 2) made the 2D explosion step 5% slower in
  // fp64 and 4.5% faster with the fp32 predictor, which uses it.
  static constexpr bool kMfmaPredictor = DIM == 2 && std::is_same<R, double>::value;

  // the wave-local predictor's LDS for a block of BLK threads: the fp64 flux
  // records, the stopping thresholds' scratch and (2D) the fused
  // reconstruction's x lines and w_h, within the 160 KiB of a CU
  template <int BLK>
  static constexpr bool pred_fits() {
    constexpr int NS = Pow<n, DIM>::v;
    constexpr int CPB = WaveCells<DIM, NS>::CPW * (BLK / 64);
    constexpr size_t VPV = 16 / sizeof(R);
    constexpr size_t RV = (NV + VPV - 1) / VPV * VPV;
    constexpr size_t rec = std::is_same<R, double>::value ? (size_t)(BLK / 64) * DIM * 64 * RV * 8 : 0;
    constexpr size_t fuse = DIM == 2 ? (size_t)CPB * NV * (NS + S * n) * 8 : 0;
    return rec + fuse + (size_t)(BLK / 64) * 64 * sizeof(R) + 1024 <= 163840;
  }

  bool pred_block_ok(int block) const override {
    if (kMfmaPredictor) return block == 256;
    switch (block) {
      case 128: return pred_fits<128>();
      case 256: return pred_fits<256>();
      case 512: return pred_fits<512>();
      default: return false;
    }
  }

  template <int BLK>
  hipError_t launch_predict(const AmrLevel& lv, const double* dt, const DevConsts& c,
                            hipStream_t st) const {
    if constexpr (!pred_fits<BLK>()) {
      return hipErrorInvalidConfiguration;
    } else {
      constexpr int NS = Pow<n, DIM>::v;
      const int64_t np = lv.nact;
      // wavefront-local exchanges (no block barriers in the sweeps)
      constexpr int WCPB = WaveCells<DIM, NS>::CPW * (BLK / 64);
      const dim3 wgrid((unsigned)((np + WCPB - 1) / WCPB));
      if constexpr (DIM == 2) {  // reconstruction fused into the predictor
        FuseWeno fw;
        fw.u = lv.u;
        fw.ld = lv.ncells;
        fw.act = lv.act;
        hipLaunchKernelGGL((k_predict_wave<DIM, M, SYS, R, R, BLK, true>), wgrid, dim3(BLK), 0,
                           st, (const double*)nullptr, static_cast<R*>(lv.qh), np, dt, lv.mp, c,
                           lv.hdr, fw);
      } else {
        hipLaunchKernelGGL((k_predict_wave<DIM, M, SYS, R, R, BLK>), wgrid, dim3(BLK), 0, st,
                           (const double*)lv.wh, static_cast<R*>(lv.qh), np, dt, lv.mp, c,
                           lv.hdr, FuseWeno{});
      }
      return hipGetLastError();
    }
  }

  hipError_t predict(const AmrLevel& lv, const double* dt, const DevConsts& c,
                     const AmrShape& sh, hipStream_t st) const override {
    const int64_t np = lv.nact;
    if (np == 0) return hipSuccess;
    unsigned int* flags = &lv.hdr->status;
    double* pass0 = lv.wa;
    double* pass1 = DIM == 2 ? lv.wh : lv.wb;
    (void)flags;
    (void)pass0;
    (void)pass1;
    if constexpr (DIM == 3) {
      // x and y lines once per non-absent cell of the level into its dense
      // pass buffers, then the z pass of the active cells into w_h
      CellLists cl;
      cl.l[0] = lv.act;
      cl.n[0] = np;
      cl.l[1] = lv.vc;
      cl.n[1] = lv.nvc;
      cl.l[2] = lv.vm;
      cl.n[2] = lv.nvm;
      const int64_t E = cl.total();
      double* dwxy = lv.dwx + (size_t)NV * n * lv.ncells;
      hipLaunchKernelGGL((k_dense_weno_x<M, NV>), dim3(amr_blocks(E * NV)), dim3(kBlock), 0, st,
                         lv.u, lv.ncells, cl, lv.mp, lv.dwx, lv.ncells, c);
      hipLaunchKernelGGL((k_dense_weno_y<M, NV>), dim3(amr_blocks(E * NV * n)), dim3(kBlock), 0,
                         st, (const double*)lv.dwx, cl, lv.mp, dwxy, lv.ncells, c);
      constexpr int ZC = ZPassCells<M>::v;
      hipLaunchKernelGGL((k_weno_z_aos<M, NV>), dim3((unsigned)((np + ZC - 1) / ZC)),
                         dim3(kBlock), 0, st, (const double*)dwxy, lv.ncells, lv.act, np, lv.mp,
                         lv.wh, c);
    }
    if constexpr (kMfmaPredictor) {
      FuseWeno fw;
      fw.u = lv.u;
      fw.ld = lv.ncells;
      fw.act = lv.act;
      hipLaunchKernelGGL((k_predict_mfma2d<M, SYS, R, true>),
                         dim3((unsigned)((np + 4 * (kBlock / 64) - 1) / (4 * (kBlock / 64)))),
                         dim3(kBlock), 0, st, (const double*)nullptr, static_cast<R*>(lv.qh), np,
                         dt, lv.mp, c, lv.hdr, fw);
      return hipGetLastError();
    } else {
      switch (sh.pred_block) {
        case 128: return launch_predict<128>(lv, dt, c, st);
        case 512: return launch_predict<512>(lv, dt, c, st);
        default: return launch_predict<256>(lv, dt, c, st);
      }
    }
  }

  hipError_t children(const AmrLevel& cl, const int32_t* moth, int64_t nm, double* wa,
                      double* wb, double* wh, const AmrLevel& fl, const int32_t* targets,
                      const int32_t* tslot, int64_t nt, const DevConsts& c, const AmrConsts& ac,
                      hipStream_t st) const override {
    if (nm == 0 || nt == 0) return hipSuccess;
    unsigned int* flags = &cl.hdr->status;
    double* pass1 = DIM == 2 ? wh : wb;
    hipLaunchKernelGGL((k_amr_weno_x<DIM, M, NV>), dim3(amr_blocks(nm * NV * Pow<S, DIM - 1>::v)),
                       dim3(kBlock), 0, st, cl.u, cl.ncells, moth, nm, cl.mp, wa, c);
    hipLaunchKernelGGL((k_level_weno_pass<DIM, M, NV, 1>),
                       dim3(amr_blocks(nm * NV * n * Pow<S, DIM - 2>::v)), dim3(kBlock), 0, st,
                       (const double*)nullptr, (int64_t)0, (const int32_t*)nullptr,
                       (const double*)wa, pass1, nm, c, flags);
    if constexpr (DIM == 3) {
      hipLaunchKernelGGL((k_level_weno_pass<DIM, M, NV, 2>), dim3(amr_blocks(nm * NV * n * n)),
                         dim3(kBlock), 0, st, (const double*)nullptr, (int64_t)0,
                         (const int32_t*)nullptr, (const double*)wb, wh, nm, c, flags);
    }
    hipLaunchKernelGGL((k_amr_subavg<DIM, M, NV>), dim3(amr_blocks(nt * NV)), dim3(kBlock), 0, st,
                       fl.u, fl.ncells, targets, tslot, nt, fl.n[0], fl.n[1], fl.n[2],
                       (const double*)wh, ac);
    return hipGetLastError();
  }

  static AmrUpdArgs upd_args(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                             const double* dt, int sub, const AmrConsts& ac) {
    AmrUpdArgs a{};
    a.u = lv.u;
    a.st = lv.st;
    a.pos = lv.pos;
    a.act = lv.act;
    a.nact = lv.nact;
    a.qh = lv.qh;
    a.fc = lv.fc;
    if (coarse) {
      a.pos_c = coarse->pos;
      a.qh_c = coarse->qh;
      for (int k = 0; k < 3; ++k) a.nc[k] = coarse->n[k];
      a.mem = lv.mem;
    }
    if (fine) {
      a.mem_f = fine->mem;
      for (int k = 0; k < 3; ++k) a.nf[k] = fine->n[k];
      a.ldf = fine->ncells;
    }
    a.dt = dt;
    a.sub = sub;
    a.r = ac.r;
    return a;
  }

  // pend / pend_dt: a finer level whose update (with step *pend_dt) rides in
  // this launch, or null
  template <int TB>
  static hipError_t launch_flux(const AmrUpdArgs& a, const AmrLevel& lv, const DevConsts& c,
                                const AmrConsts& ac, const AmrLevel* pend,
                                const double* pend_dt, hipStream_t st) {
    using Sh = AmrFluxShape<DIM, M, TB>;
    const unsigned nb = (unsigned)((lv.nact + Sh::CPB - 1) / Sh::CPB);
    const bool with_pend = DIM == 2 && pend && pend->nact > 0;
    const AmrUpdArgs ua = with_pend ? upd_args(*pend, nullptr, nullptr, pend_dt, 0, ac)
                                    : AmrUpdArgs{};
    const unsigned nab =
        with_pend ? (unsigned)((pend->nact + Sh::BLOCK - 1) / Sh::BLOCK) : 0u;
    const MeshParams ump = with_pend ? pend->mp : lv.mp;
    const double* ufbuf = with_pend ? (const double*)pend->fbuf : nullptr;
    WsHeader* uhdr = with_pend ? pend->hdr : lv.hdr;
    // one instantiation per flux (only Euler has the Osher-type flux); the
    // listed coarse-fine faces in the first ncb blocks of the same launch
    constexpr int GPB = Sh::GPB;  // coarse-fine faces per block
    const unsigned ncb = (unsigned)((lv.ncf + GPB - 1) / GPB);
    const int32_t* cfl = (const int32_t*)lv.cf;
    const dim3 grid(ncb + nab + nb);
    if (SYS == 1 && lv.mp.flux == 1)
      hipLaunchKernelGGL((k_amr_flux<DIM, M, SYS, R, TB, 1>), grid, dim3(Sh::BLOCK), 0, st, a,
                         lv.mp, c, ac, lv.fbuf, lv.hdr, cfl, (int64_t)lv.ncf, ncb, ua, ump, ufbuf,
                         uhdr, nab);
    else
      hipLaunchKernelGGL((k_amr_flux<DIM, M, SYS, R, TB, 0>), grid, dim3(Sh::BLOCK), 0, st, a,
                         lv.mp, c, ac, lv.fbuf, lv.hdr, cfl, (int64_t)lv.ncf, ncb, ua, ump, ufbuf,
                         uhdr, nab);
    return hipGetLastError();
  }

  hipError_t cf_faces(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                      const AmrConsts& ac, int* count, hipStream_t st) const override {
    if (lv.nact == 0) return hipSuccess;
    const AmrUpdArgs a = upd_args(lv, coarse, fine, nullptr, 0, ac);
    hipLaunchKernelGGL((k_amr_cf_faces<DIM>), dim3(amr_blocks(lv.nact * 2 * DIM)), dim3(kBlock),
                       0, st, a, lv.mp, lv.cf, count, lv.fc);
    return hipGetLastError();
  }

  hipError_t flux_pend(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                       const double* dt, int sub, const DevConsts& c, const AmrConsts& ac,
                       int flux_block, const AmrLevel* pend, const double* pend_dt,
                       hipStream_t st) const {
    const AmrUpdArgs a = upd_args(lv, coarse, fine, dt, sub, ac);
    switch (flux_block) {
      case 128: return launch_flux<128>(a, lv, c, ac, pend, pend_dt, st);
      case 512: return launch_flux<512>(a, lv, c, ac, pend, pend_dt, st);
      default: return launch_flux<256>(a, lv, c, ac, pend, pend_dt, st);
    }
  }

  hipError_t flux_only(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                       const double* dt, int sub, const DevConsts& c, const AmrConsts& ac,
                       int flux_block, hipStream_t st) const override {
    if (lv.nact == 0) return hipSuccess;
    return flux_pend(lv, coarse, fine, dt, sub, c, ac, flux_block, nullptr, nullptr, st);
  }

  hipError_t update(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                    const double* dt, int sub, const DevConsts& c, const AmrConsts& ac,
                    const AmrShape& sh, bool apply, const AmrLevel* pend,
                    const double* pend_dt, hipStream_t st) const override {
    // the finer level's update in a launch of its own where the face launch
    // does not carry it (3D, or no faces on this level)
    if (pend && pend->nact > 0 && (DIM == 3 || lv.nact == 0)) {
      const AmrUpdArgs ua = upd_args(*pend, nullptr, nullptr, pend_dt, 0, ac);
      hipLaunchKernelGGL((k_amr_apply<DIM, SYS>), dim3(amr_blocks(pend->nact)), dim3(kBlock), 0,
                         st, ua, pend->mp, (const double*)pend->fbuf, pend->hdr);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (lv.nact == 0) return hipSuccess;
    hipError_t e = flux_pend(lv, coarse, fine, dt, sub, c, ac, sh.flux_block, pend, pend_dt, st);
    if (e != hipSuccess || !apply) return e;
    const AmrUpdArgs a = upd_args(lv, coarse, fine, dt, sub, ac);
    hipLaunchKernelGGL((k_amr_apply<DIM, SYS>), dim3(amr_blocks(lv.nact)), dim3(kBlock), 0, st,
                       a, lv.mp, (const double*)lv.fbuf, lv.hdr);
    return hipGetLastError();
  }
};

template <int DIM, int M>
const AmrImplBase* pick_amr(int sys, int prec) {
  static const AmrImpl<DIM, M, 0, double> a;
  static const AmrImpl<DIM, M, 0, float> b;
  static const AmrImpl<DIM, M, 1, double> c;
  static const AmrImpl<DIM, M, 1, float> d;
  static const AmrImpl<DIM, M, 2, double> e;
  static const AmrImpl<DIM, M, 2, float> f;
  if (sys == 0) return prec == 0 ? (const AmrImplBase*)&a : (const AmrImplBase*)&b;
  if (sys == 1) return prec == 0 ? (const AmrImplBase*)&c : (const AmrImplBase*)&d;
  return prec == 0 ? (const AmrImplBase*)&e : (const AmrImplBase*)&f;
}

}  // namespace ader
