// Plan data shared by the C ABI and the templated launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ader.h"
#include "consts.hpp"
#include "kernels.hpp"

namespace ader {

// Optional per-stage timing with HIP events (see ader_profile_begin).
struct Profiler {
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipError_t mark(int stage, hipStream_t st, hipEvent_t* a) {
    if (!on) return hipSuccess;
    hipError_t e = hipEventCreate(a);
    if (e == hipSuccess) e = hipEventRecord(*a, st);
    (void)stage;
    return e;
  }
  hipError_t close(int stage, hipStream_t st, hipEvent_t a) {
    if (!on) return hipSuccess;
    hipEvent_t b;
    hipError_t e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) recs.push_back({stage, a, b});
    return e;
  }
};

// RAII bracket of one stage
struct StageTimer {
  Profiler* prof;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(Profiler* p, int s, hipStream_t stream) : prof(p), stage(s), st(stream) {
    if (prof && prof->on) (void)prof->mark(stage, st, &a);
  }
  ~StageTimer() {
    if (prof && prof->on && a) (void)prof->close(stage, st, a);
  }
};

struct PlanData {
  ader_problem prob;
  int dim = 2, M = 0, n = 1, nv = 1, ns = 1, nst = 1;
  int64_t ncells = 0;
  int64_t nfaces[3] = {0, 0, 0};
  MeshParams mp;
  DevConsts dc;
  RefConstants ref;
  // workspace layout (byte offsets; every section 256-byte aligned)
  size_t off_wx = 0, off_wxy = 0, off_wh = 0, off_qh = 0, off_f[3] = {0, 0, 0};
  size_t off_dtp = 0;  // per-block partial maxima of the time-step reduction
  size_t off_tr = 0;   // face traces of the fused 2D path
  size_t ws_bytes = 0;
  size_t step_bytes = 0;  // leading part of the workspace that ader_step uses
  int cell_rows = 8;   // tile height of the fused 2D cell kernel (ader_tune)
  mutable Profiler prof;
};

// Shared by the C ABI entry points (capi.cpp, server.cpp).
ader_status fail(ader_status st, const std::string& msg);  // records ader_last_error
ader_status hip_status(hipError_t e, const char* where);
// Checks a problem description; on success *ncells_out is the cell count.
ader_status validate_problem(const ader_problem& pr, int64_t* ncells_out);
void fill_dev_consts(const RefConstants& r, int M, DevConsts* out);
void fill_mesh_params(const ader_problem& pr, int64_t ncells, MeshParams* out);

// A level view after validation (device pointers).
struct LevelArgs {
  double dx[3];
  int64_t npred, nupd;
  const int32_t* pred_cells;
  const int32_t* pred_patch;
  const int32_t* upd;
  const int32_t* upd_nbr;
};

// Level workspace: header | pass scratch A | pass scratch B | w_h | q_h
struct LevelLayout {
  size_t off_a, off_b, off_wh, off_qh, bytes;
};

// Per-(dim, M, system, precision) launcher set.
struct ImplBase {
  virtual ~ImplBase() = default;
  virtual size_t qh_elem_size() const = 0;
  virtual hipError_t clear_status(char* ws, hipStream_t st) const = 0;
  virtual hipError_t compute_dt(const PlanData& p, const double* u, int64_t ld, double t,
                                double t_end, double* dt, char* ws, hipStream_t st) const = 0;
  virtual hipError_t reconstruct(const PlanData& p, const double* u, int64_t ld, double* wh,
                                 char* ws, hipStream_t st) const = 0;
  virtual hipError_t predict_debug(const PlanData& p, const double* wh, int64_t ncells,
                                   double* qh, const double* dt, char* ws,
                                   hipStream_t st) const = 0;
  virtual hipError_t step(const PlanData& p, const double* u_in, double* u_out, int64_t ld,
                          const double* dt, char* ws, hipStream_t st) const = 0;
  // the fused 2D cell kernel alone with tile height 'rows' (2D plans)
  virtual hipError_t cell2d(const PlanData& p, const double* u_in, int64_t ld, const double* dt,
                            char* ws, int rows, hipStream_t st) const = 0;
  // the cell kernel at the plan's height, then its traces upcast to fp64 (2D plans)
  virtual hipError_t traces_debug(const PlanData& p, const double* u_in, int64_t ld,
                                  const double* dt, double* out, char* ws,
                                  hipStream_t st) const = 0;
  virtual LevelLayout level_layout(const PlanData& p, int64_t npred) const = 0;
  virtual hipError_t step_level(const PlanData& p, const LevelArgs& L, const double* u_in,
                                double* u_out, int64_t ld, const double* dt, char* ws,
                                hipStream_t st) const = 0;
};

const ImplBase* make_impl_2d(int M, int sys, int prec);
const ImplBase* make_impl_3d(int M, int sys, int prec);

}  // namespace ader

// The opaque plan of the C ABI.
struct ader_plan_s {
  ader::PlanData data;
  const ader::ImplBase* impl = nullptr;
};
