// Templated launcher set for one (dim, M, system, predictor precision).
#pragma once

#include <type_traits>

#include "plan.hpp"
#include "cell2d_launch.hpp"
#include "fused2d.hpp"
#include "level.hpp"
#include "predict_mfma.hpp"
#include "predict_wave.hpp"
#include "weno3d.hpp"

namespace ader {

// out[i] = (double)in[i]
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_to_double(const T* __restrict__ in, double* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (double)in[i];
}

inline unsigned int blocks_for(int64_t threads, int per_block = kBlock) {
  return (unsigned int)((threads + per_block - 1) / per_block);
}

template <int DIM, int M, int SYS, typename R>
LevelLayout level_layout_for(const PlanData& p, int64_t npred);

template <int DIM, int M, int SYS, typename R>
struct Impl final : ImplBase {
  static constexpr int n = M + 1;
  static constexpr int NS = Pow<n, DIM>::v;
  static constexpr int NV = NVars<SYS, DIM>::v;

  size_t qh_elem_size() const override { return sizeof(R); }

  hipError_t clear_status(char* ws, hipStream_t st) const override {
    hipLaunchKernelGGL(k_clear_status<DIM>, dim3(1), dim3(kCounterSlots), 0, st,
                       reinterpret_cast<WsHeader*>(ws));
    return hipGetLastError();
  }

  static MeshParams params(const PlanData& p, int64_t ld) {
    MeshParams mp = p.mp;
    mp.ld = ld;
    return mp;
  }

  hipError_t compute_dt(const PlanData& p, const double* u, int64_t ld, double t, double t_end,
                        double* dt, char* ws, hipStream_t st) const override {
    WsHeader* hdr = reinterpret_cast<WsHeader*>(ws);
    const MeshParams mp = params(p, ld);
    StageTimer timer(&p.prof, ADER_STAGE_DT, st);
    unsigned int nb = blocks_for(p.ncells);
    if (nb > (unsigned)kDtUniformBlocks) nb = kDtUniformBlocks;
    double* partial = reinterpret_cast<double*>(ws + p.off_dtp);
    hipLaunchKernelGGL((k_dt<DIM, SYS>), dim3(nb), dim3(kBlock), 0, st, u, mp, hdr, partial,
                       p.prob.cfl, t, t_end, dt);
    return hipGetLastError();
  }

  // WENO passes: averages -> w_h (per-cell blocks) written to wh
  hipError_t weno(const PlanData& p, const double* u, int64_t ld, double* wh, char* ws,
                  hipStream_t st) const {
    const MeshParams mp = params(p, ld);
    const int64_t C = p.ncells;
    StageTimer timer(&p.prof, ADER_STAGE_WENO, st);
    double* wx = reinterpret_cast<double*>(ws + p.off_wx);
    hipLaunchKernelGGL((k_weno_pass<DIM, M, NV, 0, false>), dim3(blocks_for(C * NV)),
                       dim3(kBlock), 0, st, u, ld, 1, wx, mp, p.dc);
    if constexpr (DIM == 2) {
      hipLaunchKernelGGL((k_weno_pass<DIM, M, NV, 1, true>), dim3(blocks_for(C * NV * n)),
                         dim3(kBlock), 0, st, (const double*)wx, C, n, wh, mp, p.dc);
    } else {
      double* wxy = reinterpret_cast<double*>(ws + p.off_wxy);
      hipLaunchKernelGGL((k_weno_pass<DIM, M, NV, 1, false>), dim3(blocks_for(C * NV * n)),
                         dim3(kBlock), 0, st, (const double*)wx, C, n, wxy, mp, p.dc);
      // z pass through LDS: each block writes its cells' w_h contiguously
      hipLaunchKernelGGL((k_weno_z_aos<M, NV>), dim3(blocks_for(C, ZPassCells<M>::v)),
                         dim3(kBlock), 0, st, (const double*)wxy, C, (const int32_t*)nullptr,
                         C, mp, wh, p.dc);
    }
    return hipGetLastError();
  }

  hipError_t reconstruct(const PlanData& p, const double* u, int64_t ld, double* wh, char* ws,
                         hipStream_t st) const override {
    return weno(p, u, ld, wh, ws, st);
  }

  template <typename OUT>
  hipError_t predict(const PlanData& p, const double* wh, int64_t ncells, OUT* qh,
                     const double* dt, char* ws, hipStream_t st) const {
    constexpr int CPB = kBlock / NS;
    WsHeader* hdr = reinterpret_cast<WsHeader*>(ws);
    MeshParams mp = p.mp;
    StageTimer timer(&p.prof, ADER_STAGE_PREDICT, st);
    if constexpr (DIM == 2 && std::is_same<R, double>::value) {
      // fp64 matrix cores: 4 cells per wavefront, 16 per block
      hipLaunchKernelGGL((k_predict_mfma2d<M, SYS, OUT>),
                         dim3(blocks_for(ncells, 4 * (kBlock / 64))), dim3(kBlock), 0, st, wh,
                         qh, ncells, dt, mp, p.dc, hdr);
    } else if constexpr (DIM == 3) {
      // wavefront-local exchanges (no LDS round trips, no block barriers)
      constexpr int WCPB = (64 / WaveGroup<NS>::G) * (kBlock / 64);
      hipLaunchKernelGGL((k_predict_wave<DIM, M, SYS, R, OUT>), dim3(blocks_for(ncells, WCPB)),
                         dim3(kBlock), 0, st, wh, qh, ncells, dt, mp, p.dc, hdr);
    } else {
      hipLaunchKernelGGL((k_predict<DIM, M, SYS, R, OUT>), dim3(blocks_for(ncells, CPB)),
                         dim3(kBlock), 0, st, wh, qh, ncells, dt, mp, p.dc, hdr);
    }
    return hipGetLastError();
  }

  hipError_t predict_debug(const PlanData& p, const double* wh, int64_t ncells, double* qh,
                           const double* dt, char* ws, hipStream_t st) const override {
    if (ncells == 0) return hipSuccess;
    return predict<double>(p, wh, ncells, qh, dt, ws, st);
  }

  hipError_t step(const PlanData& p, const double* u_in, double* u_out, int64_t ld,
                  const double* dt, char* ws, hipStream_t st) const override {
    if constexpr (DIM == 2) return step_fused2d(p, u_in, u_out, ld, dt, ws, st);
    return step_stages(p, u_in, u_out, ld, dt, ws, st);
  }

  LevelLayout level_layout(const PlanData& p, int64_t npred) const override {
    return level_layout_for<DIM, M, SYS, R>(p, npred);
  }

  // one step over a level's cell lists (patch WENO, predictor, update)
  hipError_t step_level(const PlanData& p, const LevelArgs& L, const double* u_in,
                        double* u_out, int64_t ld, const double* dt, char* ws,
                        hipStream_t st) const override {
    constexpr int S = 2 * M + 1;
    constexpr int NS = Pow<n, DIM>::v;
    const LevelLayout lay = level_layout(p, L.npred);
    WsHeader* hdr = reinterpret_cast<WsHeader*>(ws);
    double* A = reinterpret_cast<double*>(ws + lay.off_a);
    double* B = reinterpret_cast<double*>(ws + lay.off_b);
    double* wh = reinterpret_cast<double*>(ws + lay.off_wh);
    R* qh = reinterpret_cast<R*>(ws + lay.off_qh);
    MeshParams mp = p.mp;
    for (int k = 0; k < 3; ++k) mp.dx[k] = L.dx[k];
    mp.ld = ld;
    unsigned int* flags = &hdr->status;
    if (L.npred > 0) {
      StageTimer timer(&p.prof, ADER_STAGE_WENO, st);
      const int64_t l0 = L.npred * NV * Pow<S, DIM - 1>::v;
      // pass 0 -> A; pass 1 -> w_h (2D) or B (3D); pass 2 (3D) -> w_h
      hipLaunchKernelGGL((k_level_weno_pass<DIM, M, NV, 0>), dim3(blocks_for(l0)), dim3(kBlock),
                         0, st, u_in, ld, L.pred_patch, (const double*)nullptr, A, L.npred,
                         p.dc, flags);
      const int64_t l1 = L.npred * NV * n * Pow<S, DIM - 2>::v;
      hipLaunchKernelGGL((k_level_weno_pass<DIM, M, NV, 1>), dim3(blocks_for(l1)), dim3(kBlock),
                         0, st, u_in, ld, L.pred_patch, (const double*)A, DIM == 2 ? wh : B,
                         L.npred, p.dc, flags);
      if constexpr (DIM == 3) {
        const int64_t l2 = L.npred * NV * n * n;
        hipLaunchKernelGGL((k_level_weno_pass<DIM, M, NV, 2>), dim3(blocks_for(l2)),
                           dim3(kBlock), 0, st, u_in, ld, L.pred_patch, (const double*)B, wh,
                           L.npred, p.dc, flags);
      }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.npred > 0) {
      StageTimer timer(&p.prof, ADER_STAGE_PREDICT, st);
      if constexpr (DIM == 2 && std::is_same<R, double>::value) {
        hipLaunchKernelGGL((k_predict_mfma2d<M, SYS, R>),
                           dim3(blocks_for(L.npred, 4 * (kBlock / 64))), dim3(kBlock), 0, st,
                           (const double*)wh, qh, L.npred, dt, mp, p.dc, hdr);
      } else if constexpr (DIM == 3) {
        constexpr int WCPB = (64 / WaveGroup<NS>::G) * (kBlock / 64);
        hipLaunchKernelGGL((k_predict_wave<DIM, M, SYS, R, R>),
                           dim3(blocks_for(L.npred, WCPB)), dim3(kBlock), 0, st,
                           (const double*)wh, qh, L.npred, dt, mp, p.dc, hdr);
      } else {
        hipLaunchKernelGGL((k_predict<DIM, M, SYS, R, R>),
                           dim3(blocks_for(L.npred, kBlock / NS)), dim3(kBlock), 0, st,
                           (const double*)wh, qh, L.npred, dt, mp, p.dc, hdr);
      }
    }
    if (L.nupd > 0) {
      StageTimer timer(&p.prof, ADER_STAGE_UPDATE, st);
      hipLaunchKernelGGL((k_level_update<DIM, M, SYS, R>), dim3(blocks_for(L.nupd)),
                         dim3(kBlock), 0, st, (const R*)qh, L.pred_cells, L.upd, L.upd_nbr,
                         L.nupd, L.npred, u_in, u_out, ld, dt, L.dx[0], L.dx[1], L.dx[2], mp,
                         p.dc, hdr);
    }
    return hipGetLastError();
  }

  // 2D: cell kernel (WENO + predictor + traces) and face kernel
  hipError_t cell2d(const PlanData& p, const double* u_in, int64_t ld, const double* dt,
                    char* ws, int rows, hipStream_t st) const override {
    if constexpr (DIM != 2) {
      return hipErrorInvalidConfiguration;
    } else {
      Cell2dArgs a;
      a.u = u_in;
      a.ld = ld;
      a.traces = ws + p.off_tr;
      a.dt = dt;
      a.mp = params(p, ld);
      a.n0 = p.mp.n[0];
      a.n1 = p.mp.n[1];
      return launch_cell2d(rows, M, SYS, std::is_same<R, double>::value ? 0 : 1, a, p.dc,
                           reinterpret_cast<WsHeader*>(ws), st);
    }
  }

  hipError_t traces_debug(const PlanData& p, const double* u_in, int64_t ld, const double* dt,
                          double* out, char* ws, hipStream_t st) const override {
    if constexpr (DIM != 2) {
      return hipErrorInvalidConfiguration;
    } else {
      hipError_t e = cell2d(p, u_in, ld, dt, ws, p.cell_rows, st);
      if (e != hipSuccess) return e;
      const int64_t count = 4 * p.ncells * NV * n * n;
      hipLaunchKernelGGL((k_to_double<R>), dim3(blocks_for(count)), dim3(kBlock), 0, st,
                         reinterpret_cast<const R*>(ws + p.off_tr), out, count);
      return hipGetLastError();
    }
  }

  hipError_t step_fused2d(const PlanData& p, const double* u_in, double* u_out, int64_t ld,
                          const double* dt, char* ws, hipStream_t st) const {
    const MeshParams mp = params(p, ld);
    WsHeader* hdr = reinterpret_cast<WsHeader*>(ws);
    R* tr = reinterpret_cast<R*>(ws + p.off_tr);
    {
      StageTimer timer(&p.prof, ADER_STAGE_PREDICT, st);
      hipError_t e = cell2d(p, u_in, ld, dt, ws, p.cell_rows, st);
      if (e != hipSuccess) return e;
    }
    {
      StageTimer timer(&p.prof, ADER_STAGE_FLUX, st);
      dim3 grid((p.mp.n[0] + kFaceTX - 1) / kFaceTX, (p.mp.n[1] + kFaceTY - 1) / kFaceTY);
      // one instantiation per flux (only Euler has the Osher-type flux)
      if (SYS == 1 && p.mp.flux == 1)
        hipLaunchKernelGGL((k_face2d<M, SYS, R, 1>), grid, dim3(kBlock), 0, st, (const R*)tr,
                           u_in, u_out, ld, dt, mp, p.dc, hdr);
      else
        hipLaunchKernelGGL((k_face2d<M, SYS, R, 0>), grid, dim3(kBlock), 0, st, (const R*)tr,
                           u_in, u_out, ld, dt, mp, p.dc, hdr);
    }
    return hipGetLastError();
  }

  hipError_t step_stages(const PlanData& p, const double* u_in, double* u_out, int64_t ld,
                         const double* dt, char* ws, hipStream_t st) const {
    hipError_t e;
    double* wh = reinterpret_cast<double*>(ws + p.off_wh);
    R* qh = reinterpret_cast<R*>(ws + p.off_qh);
    if ((e = weno(p, u_in, ld, wh, ws, st)) != hipSuccess) return e;
    if ((e = predict<R>(p, wh, p.ncells, qh, dt, ws, st)) != hipSuccess) return e;
    const MeshParams mp = params(p, ld);
    double* F[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < DIM; ++k) F[k] = reinterpret_cast<double*>(ws + p.off_f[k]);
    constexpr int FPB = kBlock / NS;
    {
    StageTimer timer(&p.prof, ADER_STAGE_FLUX, st);
    hipLaunchKernelGGL((k_face_flux<DIM, M, SYS, R, 0>), dim3(blocks_for(p.nfaces[0], FPB)),
                       dim3(kBlock), 0, st, (const R*)qh, F[0], p.nfaces[0], mp, p.dc);
    hipLaunchKernelGGL((k_face_flux<DIM, M, SYS, R, 1>), dim3(blocks_for(p.nfaces[1], FPB)),
                       dim3(kBlock), 0, st, (const R*)qh, F[1], p.nfaces[1], mp, p.dc);
    if constexpr (DIM == 3)
      hipLaunchKernelGGL((k_face_flux<DIM, M, SYS, R, 2>), dim3(blocks_for(p.nfaces[2], FPB)),
                         dim3(kBlock), 0, st, (const R*)qh, F[2], p.nfaces[2], mp, p.dc);
    }
    StageTimer timer(&p.prof, ADER_STAGE_UPDATE, st);
    WsHeader* hdr = reinterpret_cast<WsHeader*>(ws);
    hipLaunchKernelGGL((k_update<DIM, SYS>), dim3(blocks_for(p.ncells)), dim3(kBlock), 0, st,
                       u_in, u_out, (const double*)F[0], (const double*)F[1],
                       (const double*)F[2], p.nfaces[0], p.nfaces[1], p.nfaces[2], dt, mp,
                       hdr);
    return hipGetLastError();
  }
};

template <int DIM, int M, int SYS, typename R>
LevelLayout level_layout_for(const PlanData& p, int64_t npred) {
  constexpr int n = M + 1, S = 2 * M + 1, NV = NVars<SYS, DIM>::v;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t np = (size_t)(npred > 0 ? npred : 1);
  LevelLayout L;
  size_t off = kHeaderBytes;
  L.off_a = off;
  off = al(off + sizeof(double) * np * NV * n * Pow<S, DIM - 1>::v);
  L.off_b = off;
  off = al(off + (DIM == 3 ? sizeof(double) * np * NV * n * n * S : 0));
  L.off_wh = off;
  off = al(off + sizeof(double) * np * NV * Pow<n, DIM>::v);
  L.off_qh = off;
  off = al(off + sizeof(R) * np * NV * Pow<n, DIM + 1>::v);
  L.bytes = off;
  (void)p;
  return L;
}

template <int DIM, int M>
const ImplBase* pick_impl(int sys, int prec) {
  static const Impl<DIM, M, 0, double> a;
  static const Impl<DIM, M, 0, float> b;
  static const Impl<DIM, M, 1, double> c;
  static const Impl<DIM, M, 1, float> d;
  static const Impl<DIM, M, 2, double> e;
  static const Impl<DIM, M, 2, float> f;
  if (sys == 0) return prec == 0 ? (const ImplBase*)&a : (const ImplBase*)&b;
  if (sys == 1) return prec == 0 ? (const ImplBase*)&c : (const ImplBase*)&d;
  return prec == 0 ? (const ImplBase*)&e : (const ImplBase*)&f;
}

}  // namespace ader
