// C ABI of the ADER-WENO hot path: argument validation, plan construction,
// workspace layout and dispatch to the templated launchers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "plan.hpp"
#include "cell2d_launch.hpp"

namespace {
thread_local std::string g_last_error;
bool is_finite(double x) { return std::isfinite(x); }
}  // namespace

namespace ader {

ader_status fail(ader_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ader_status hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return ADER_OK;
  return fail(ADER_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

ader_status validate_problem(const ader_problem& pr, int64_t* ncells_out) {
  if (pr.dim != 2 && pr.dim != 3) return fail(ADER_EUNSUPPORTED, "dim must be 2 or 3");
  if (pr.M < 0 || pr.M > 3) return fail(ADER_EUNSUPPORTED, "M must be in 0..3");
  if (pr.system != ADER_SYS_LINADV && pr.system != ADER_SYS_EULER &&
      pr.system != ADER_SYS_MHD_GLM)
    return fail(ADER_EUNSUPPORTED, "unknown system");
  if (pr.precision != ADER_PREC_FP64 && pr.precision != ADER_PREC_FP32_PREDICTOR)
    return fail(ADER_EINVAL, "unknown precision");
  int64_t ncells = 1;
  for (int k = 0; k < pr.dim; ++k) {
    if (pr.n[k] < 1) return fail(ADER_EINVAL, "cells per axis must be >= 1");
    if (!is_finite(pr.lo[k]) || !is_finite(pr.hi[k]) || !(pr.hi[k] > pr.lo[k]))
      return fail(ADER_EINVAL, "domain bounds must be finite with hi > lo");
    if (pr.bc[k] != ADER_BC_PERIODIC && pr.bc[k] != ADER_BC_TRANSMISSIVE)
      return fail(ADER_EINVAL, "unknown boundary condition");
    ncells *= pr.n[k];
  }
  if (ncells > (int64_t(1) << 28)) return fail(ADER_EUNSUPPORTED, "more than 2^28 cells");
  if (!is_finite(pr.cfl) || !(pr.cfl > 0.0) || pr.cfl > 1.0)
    return fail(ADER_EINVAL, "cfl must be in (0, 1]");
  if (pr.system != ADER_SYS_LINADV && (!is_finite(pr.gamma) || !(pr.gamma > 1.0)))
    return fail(ADER_EINVAL, "gamma must be > 1");
  if (pr.system == ADER_SYS_MHD_GLM && (!is_finite(pr.ch) || !(pr.ch > 0.0)))
    return fail(ADER_EINVAL, "the cleaning speed ch must be > 0");
  if (pr.system == ADER_SYS_LINADV)
    for (int k = 0; k < 3; ++k)
      if (!is_finite(pr.adv[k])) return fail(ADER_EINVAL, "advection velocity must be finite");
  if (pr.flux != ADER_FLUX_RUSANOV && pr.flux != ADER_FLUX_OSHER)
    return fail(ADER_EINVAL, "unknown numerical flux");
  if (pr.flux == ADER_FLUX_OSHER && pr.system == ADER_SYS_MHD_GLM)
    return fail(ADER_EUNSUPPORTED, "the Osher-type flux is built for Euler and advection");
  if (!is_finite(pr.picard_tol) || !(pr.picard_tol > 0.0))
    return fail(ADER_EINVAL, "picard_tol must be > 0");
  if (pr.picard_max < 1 || pr.picard_max > 1000)
    return fail(ADER_EINVAL, "picard_max must be in 1..1000");

  *ncells_out = ncells;
  return ADER_OK;
}

void fill_dev_consts(const RefConstants& r, int M, DevConsts* out) {
  DevConsts& c = *out;
  std::memset(&c, 0, sizeof(c));
  const int n = M + 1;
  for (int a = 0; a < n; ++a) {
    c.psi0[a] = (double)r.psi0[a];
    c.psi1[a] = (double)r.psi1[a];
    c.w[a] = (double)r.weights[a];
    c.psi0_f[a] = (float)r.psi0[a];
    c.psi1_f[a] = (float)r.psi1[a];
    for (int b = 0; b < n; ++b) {
      c.dmat[a][b] = (double)r.dmat[a][b];
      c.tinvw[a][b] = (double)r.time_inv_w[a][b];
      c.dmat_f[a][b] = (float)r.dmat[a][b];
      c.tinvw_f[a][b] = (float)r.time_inv_w[a][b];
    }
  }
  for (int j = 0; j < kOsherNodes; ++j) {
    c.path_s[j] = (double)r.path_s[j];
    c.path_w[j] = (double)r.path_w[j];
  }
  for (int s = 0; s < r.nstencils; ++s) {
    c.lam[s] = (double)r.lambda[s];
    for (int pp = 0; pp < n; ++pp)
      for (int e = 0; e < n; ++e) c.rec_inv[s][pp][e] = (double)r.rec_inv[s][pp][e];
    for (int k = 0; k < r.nsig_rows; ++k)
      for (int e = 0; e < n; ++e) c.sig_rows[s][k][e] = (double)r.sig_rows[s][k][e];
  }
}

void fill_mesh_params(const ader_problem& pr, int64_t ncells, MeshParams* out) {
  MeshParams& mp = *out;
  std::memset(&mp, 0, sizeof(mp));
  for (int k = 0; k < 3; ++k) {
    const bool used = k < pr.dim;
    mp.n[k] = used ? pr.n[k] : 1;
    mp.bc[k] = used ? pr.bc[k] : 0;
    mp.dx[k] = used ? (pr.hi[k] - pr.lo[k]) / pr.n[k] : 1.0;
    mp.adv[k] = pr.system == ADER_SYS_LINADV ? pr.adv[k] : 0.0;
  }
  mp.gamma = pr.gamma;
  mp.ch = pr.system == ADER_SYS_MHD_GLM ? pr.ch : 0.0;
  mp.flux = pr.system == ADER_SYS_EULER ? pr.flux : ADER_FLUX_RUSANOV;
  mp.tol = pr.picard_tol;
  mp.maxit = pr.picard_max;
  mp.ncells = ncells;
  mp.ld = ncells;
}

}  // namespace ader

using ader::fail;
using ader::hip_status;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

ader_status check_ws(const ader_plan p, const void* ws) {
  if (!ws) return fail(ADER_EWORKSPACE, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(ADER_EWORKSPACE, "workspace must be 256-byte aligned");
  (void)p;
  return ADER_OK;
}

ader_status check_state(const ader_plan p, const void* u, int64_t ld) {
  if (!u) return fail(ADER_EINVAL, "state pointer is null");
  if (ld < p->data.ncells) return fail(ADER_EINVAL, "ld is smaller than the number of cells");
  return ADER_OK;
}

}  // namespace

extern "C" {

const char* ader_status_string(ader_status s) {
  switch (s) {
    case ADER_OK: return "ok";
    case ADER_EINVAL: return "invalid argument";
    case ADER_EUNSUPPORTED: return "unsupported problem";
    case ADER_EHIP: return "HIP runtime error";
    case ADER_EWORKSPACE: return "bad workspace";
  }
  return "unknown status";
}

const char* ader_last_error(void) { return g_last_error.c_str(); }

ader_status ader_plan_create(const ader_problem* prob, ader_plan* out) {
  if (!prob || !out) return fail(ADER_EINVAL, "null argument");
  *out = nullptr;
  const ader_problem& pr = *prob;
  int64_t ncells = 0;
  if (ader_status st = ader::validate_problem(pr, &ncells)) return st;

  ader_plan p = new (std::nothrow) ader_plan_s();
  if (!p) return fail(ADER_EINVAL, "out of host memory");
  ader::PlanData& d = p->data;
  d.prob = pr;
  if (pr.dim == 2) d.prob.n[2] = 1;
  d.dim = pr.dim;
  d.M = pr.M;
  d.n = pr.M + 1;
  d.nv = pr.system == ADER_SYS_LINADV ? 1 : (pr.system == ADER_SYS_EULER ? pr.dim + 2 : 9);
  d.ns = 1;
  for (int k = 0; k < pr.dim; ++k) d.ns *= d.n;
  d.nst = d.ns * d.n;
  d.ncells = ncells;

  if (!ader::build_ref_constants(pr.M, &d.ref)) {
    delete p;
    return fail(ADER_EINVAL, "singular reference matrix");
  }
  ader::fill_dev_consts(d.ref, d.M, &d.dc);
  ader::fill_mesh_params(pr, ncells, &d.mp);
  const ader::MeshParams& mp = d.mp;

  p->impl = pr.dim == 2 ? ader::make_impl_2d(pr.M, pr.system, pr.precision)
                        : ader::make_impl_3d(pr.M, pr.system, pr.precision);
  if (!p->impl) {
    delete p;
    return fail(ADER_EUNSUPPORTED, "no kernels for this configuration");
  }

  // faces along axis k on the mesh extended by one cell along k
  for (int k = 0; k < pr.dim; ++k) {
    int64_t nf = 1;
    for (int m = 0; m < pr.dim; ++m) nf *= mp.n[m] + (m == k ? 1 : 0);
    d.nfaces[k] = nf;
  }

  // workspace: header | CFL partial maxima | what ader_step uses | the rest.
  //   2D: face traces (the fused step) | Wx | w_h | q_h (stage entry points)
  //   3D: Wx | Wxy | w_h | q_h | face fluxes (all used by the step)
  size_t off = ader::kHeaderBytes;
  const size_t C = (size_t)ncells;
  d.off_dtp = off;
  off = align256(off + sizeof(double) * ader::kDtUniformBlocks);
  d.off_tr = off;
  if (pr.dim == 2) {  // four face traces per cell: nv x n (transverse) x n (time) each
    off = align256(off + p->impl->qh_elem_size() * 4 * (size_t)d.nv * d.n * d.n * C);
    d.step_bytes = off;
  }
  d.off_wx = off;
  off = align256(off + sizeof(double) * d.nv * d.n * C);
  d.off_wxy = off;
  if (pr.dim == 3) off = align256(off + sizeof(double) * d.nv * d.n * d.n * C);
  d.off_wh = off;
  off = align256(off + sizeof(double) * d.nv * d.ns * C);
  d.off_qh = off;
  off = align256(off + p->impl->qh_elem_size() * d.nv * d.nst * C);
  if (pr.dim == 3) {
    for (int k = 0; k < pr.dim; ++k) {
      d.off_f[k] = off;
      off = align256(off + sizeof(double) * d.nv * (size_t)d.nfaces[k]);
    }
    d.step_bytes = off;
  }
  d.ws_bytes = off;
  *out = p;
  return ADER_OK;
}

ader_status ader_plan_destroy(ader_plan plan) {
  delete plan;
  return ADER_OK;
}

ader_status ader_plan_nvar(ader_plan plan, int* nvar) {
  if (!plan || !nvar) return fail(ADER_EINVAL, "null argument");
  *nvar = plan->data.nv;
  return ADER_OK;
}

ader_status ader_workspace_bytes(ader_plan plan, size_t* bytes) {
  if (!plan || !bytes) return fail(ADER_EINVAL, "null argument");
  *bytes = plan->data.ws_bytes;
  return ADER_OK;
}

ader_status ader_clear_status(ader_plan plan, void* ws, void* stream) {
  if (!plan) return fail(ADER_EINVAL, "null plan");
  if (ader_status s = check_ws(plan, ws)) return s;
  return hip_status(plan->impl->clear_status((char*)ws, (hipStream_t)stream),
                    "ader_clear_status");
}

ader_status ader_compute_dt(ader_plan plan, const double* u, int64_t ld, double t,
                            double t_end, double* dt_dev, void* ws, void* stream) {
  if (!plan || !dt_dev) return fail(ADER_EINVAL, "null argument");
  if (ader_status s = check_state(plan, u, ld)) return s;
  if (ader_status s = check_ws(plan, ws)) return s;
  if (!is_finite(t) || std::isnan(t_end) || !(t_end > t))
    return fail(ADER_EINVAL, "need finite t and t_end > t");
  return hip_status(plan->impl->compute_dt(plan->data, u, ld, t, t_end, dt_dev, (char*)ws,
                                           (hipStream_t)stream),
                    "ader_compute_dt");
}

ader_status ader_step(ader_plan plan, const double* u_in, double* u_out, int64_t ld,
                      const double* dt_dev, void* ws, void* stream) {
  if (!plan || !dt_dev) return fail(ADER_EINVAL, "null argument");
  if (ader_status s = check_state(plan, u_in, ld)) return s;
  if (ader_status s = check_state(plan, u_out, ld)) return s;
  if (ader_status s = check_ws(plan, ws)) return s;
  const uintptr_t a0 = (uintptr_t)u_in, b0 = (uintptr_t)u_out;
  const uintptr_t len = sizeof(double) * (uintptr_t)plan->data.nv * (uintptr_t)ld;
  if (a0 < b0 + len && b0 < a0 + len) return fail(ADER_EINVAL, "u_in and u_out overlap");
  return hip_status(plan->impl->step(plan->data, u_in, u_out, ld, dt_dev, (char*)ws,
                                     (hipStream_t)stream),
                    "ader_step");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free step: the workspace is a file-scope device array of
// ADER_STATIC_SCRATCH_BYTES that every GPU the library runs on holds until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol): each device's address comes
// from hipGetSymbolAddress, taken once per device with that device current on
// the first call there, and is kept in g_scratch_dev.
namespace {

static __device__ __align__(256) unsigned char scratch[ADER_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

ader_status static_scratch(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "ader_step_static: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ADER_EUNSUPPORTED, "ader_step_static: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "ader_step_static: hipGetSymbolAddress");
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
      return fail(ADER_EHIP, "ader_step_static: static workspace address is not 256-byte aligned");
    g_scratch_dev[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return ADER_OK;
}

// status[0] = the header's status bits, status[1] = its Picard sweeps summed
// over the counter slots (saturated to 32 bits).
__global__ void k_static_status(const ader::WsHeader* __restrict__ hdr, uint32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  unsigned long long total = 0;
  for (int i = 0; i < ader::kCounterSlots; ++i) total += hdr->iters[i];
  out[0] = hdr->status;
  out[1] = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
}

}  // namespace

extern "C" {

ader_status ader_step_static(ader_plan plan, const double* u_in, double* u_out, int64_t ld,
                             const double* dt_dev, uint32_t* status, void* stream) {
  if (!plan || !dt_dev) return fail(ADER_EINVAL, "null argument");
  if (ader_status s = check_state(plan, u_in, ld)) return s;
  if (ader_status s = check_state(plan, u_out, ld)) return s;
  const uintptr_t a0 = (uintptr_t)u_in, b0 = (uintptr_t)u_out;
  const uintptr_t len = sizeof(double) * (uintptr_t)plan->data.nv * (uintptr_t)ld;
  if (a0 < b0 + len && b0 < a0 + len) return fail(ADER_EINVAL, "u_in and u_out overlap");
  if (plan->data.step_bytes > (size_t)ADER_STATIC_SCRATCH_BYTES)
    return fail(ADER_EWORKSPACE,
                "ader_step_static: this plan's step needs " +
                    std::to_string(plan->data.step_bytes) + " bytes of workspace, the static "
                    "workspace holds " + std::to_string((size_t)ADER_STATIC_SCRATCH_BYTES) +
                    "; use ader_step with a caller-allocated workspace");
  char* ws = nullptr;
  if (ader_status s = static_scratch(&ws)) return s;
  const hipStream_t st = (hipStream_t)stream;
  // the array keeps the previous call's contents: start from a zero header
  hipError_t e = plan->impl->clear_status(ws, st);
  if (e == hipSuccess) e = plan->impl->step(plan->data, u_in, u_out, ld, dt_dev, ws, st);
  if (e == hipSuccess && status) {
    hipLaunchKernelGGL(k_static_status, dim3(1), dim3(64), 0, st,
                       reinterpret_cast<const ader::WsHeader*>(ws), status);
    e = hipGetLastError();
  }
  return hip_status(e, "ader_step_static");
}

ader_status ader_debug_reconstruct(ader_plan plan, const double* u, int64_t ld, double* w_h,
                                   void* ws, void* stream) {
  if (!plan || !w_h) return fail(ADER_EINVAL, "null argument");
  if (ader_status s = check_state(plan, u, ld)) return s;
  if (ader_status s = check_ws(plan, ws)) return s;
  return hip_status(plan->impl->reconstruct(plan->data, u, ld, w_h, (char*)ws,
                                            (hipStream_t)stream),
                    "ader_debug_reconstruct");
}

ader_status ader_debug_predict(ader_plan plan, const double* w_h, int64_t ncells, double* q_h,
                               const double* dt_dev, void* ws, void* stream) {
  if (!plan || !dt_dev) return fail(ADER_EINVAL, "null argument");
  if (ncells < 0 || ncells > (int64_t(1) << 28)) return fail(ADER_EINVAL, "bad ncells");
  if (ncells > 0 && (!w_h || !q_h)) return fail(ADER_EINVAL, "null argument");
  if (ader_status s = check_ws(plan, ws)) return s;
  return hip_status(plan->impl->predict_debug(plan->data, w_h, ncells, q_h, dt_dev, (char*)ws,
                                              (hipStream_t)stream),
                    "ader_debug_predict");
}

ader_status ader_debug_traces(ader_plan plan, const double* u, int64_t ld, const double* dt_dev,
                              double* traces, void* ws, void* stream) {
  if (!plan || !dt_dev || !traces) return fail(ADER_EINVAL, "null argument");
  if (plan->data.dim != 2) return fail(ADER_EUNSUPPORTED, "face traces are exposed for 2D plans");
  if (ader_status s = check_state(plan, u, ld)) return s;
  if (ader_status s = check_ws(plan, ws)) return s;
  return hip_status(plan->impl->traces_debug(plan->data, u, ld, dt_dev, traces, (char*)ws,
                                             (hipStream_t)stream),
                    "ader_debug_traces");
}

ader_status ader_level_workspace_bytes(ader_plan plan, int64_t npred, size_t* bytes) {
  if (!plan || !bytes) return fail(ADER_EINVAL, "null argument");
  if (npred < 0 || npred > (int64_t(1) << 28)) return fail(ADER_EINVAL, "bad npred");
  *bytes = plan->impl->level_layout(plan->data, npred).bytes;
  return ADER_OK;
}

ader_status ader_step_level(ader_plan plan, const ader_level_view* view, const double* u_in,
                            double* u_out, int64_t ld, const double* dt_dev, void* ws,
                            void* stream) {
  if (!plan || !view || !dt_dev) return fail(ADER_EINVAL, "null argument");
  if (!u_in || !u_out) return fail(ADER_EINVAL, "state pointer is null");
  if (ld < 1 || ld > (int64_t(1) << 31) - 1) return fail(ADER_EINVAL, "bad ld");
  if (ader_status s = check_ws(plan, ws)) return s;
  const ader_level_view& v = *view;
  if (v.npred < 0 || v.npred > (int64_t(1) << 28) || v.nupd < 0 || v.nupd > v.npred)
    return fail(ADER_EINVAL, "need 0 <= nupd <= npred <= 2^28");
  if (v.npred > 0 && (!v.pred_cells || !v.pred_patch))
    return fail(ADER_EINVAL, "null predicted-cell arrays");
  if (v.nupd > 0 && (!v.upd || !v.upd_nbr)) return fail(ADER_EINVAL, "null update arrays");
  for (int k = 0; k < plan->data.dim; ++k)
    if (!is_finite(v.dx[k]) || !(v.dx[k] > 0.0)) return fail(ADER_EINVAL, "dx must be > 0");
  const uintptr_t a0 = (uintptr_t)u_in, b0 = (uintptr_t)u_out;
  const uintptr_t len = sizeof(double) * (uintptr_t)plan->data.nv * (uintptr_t)ld;
  if (a0 < b0 + len && b0 < a0 + len) return fail(ADER_EINVAL, "u_in and u_out overlap");
  ader::LevelArgs L;
  for (int k = 0; k < 3; ++k) L.dx[k] = k < plan->data.dim ? v.dx[k] : 1.0;
  L.npred = v.npred;
  L.nupd = v.nupd;
  L.pred_cells = v.pred_cells;
  L.pred_patch = v.pred_patch;
  L.upd = v.upd;
  L.upd_nbr = v.upd_nbr;
  return hip_status(plan->impl->step_level(plan->data, L, u_in, u_out, ld, dt_dev, (char*)ws,
                                           (hipStream_t)stream),
                    "ader_step_level");
}

ader_status ader_read_status(ader_plan plan, const void* ws, uint32_t* flags,
                             uint64_t* picard_iterations, void* stream) {
  if (!plan || !flags) return fail(ADER_EINVAL, "null argument");
  if (ader_status s = check_ws(plan, ws)) return s;
  ader::WsHeader h;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_status(e, "ader_read_status");
  *flags = h.status;
  if (picard_iterations) {
    uint64_t total = 0;
    for (int i = 0; i < ader::kCounterSlots; ++i) total += h.iters[i];
    *picard_iterations = total;
  }
  return ADER_OK;
}

ader_status ader_debug_constants(ader_plan plan, double* nodes, double* weights, double* dmat,
                                 double* time_inv_w) {
  if (!plan || !nodes || !weights || !dmat || !time_inv_w)
    return fail(ADER_EINVAL, "null argument");
  const ader::RefConstants& r = plan->data.ref;
  const int n = r.n;
  for (int a = 0; a < n; ++a) {
    nodes[a] = (double)r.nodes[a];
    weights[a] = (double)r.weights[a];
    for (int b = 0; b < n; ++b) {
      dmat[a * n + b] = (double)r.dmat[a][b];
      time_inv_w[a * n + b] = (double)r.time_inv_w[a][b];
    }
  }
  return ADER_OK;
}

ader_status ader_set_tile_rows(ader_plan plan, int rows) {
  if (!plan) return fail(ADER_EINVAL, "null argument");
  if (plan->data.dim != 2) return fail(ADER_EUNSUPPORTED, "tile heights apply to 2D plans");
  if (rows == 0) rows = ader::kCellRowsDefault;
  bool known = false;
  for (int r : ader::kCellRowChoices) known = known || r == rows;
  const int top = ader::max_cell_rows(plan->data.prob.system, plan->data.prob.precision);
  if (!known || rows > top)
    return fail(ADER_EINVAL, "tile rows must be 2, 4, 8 or 16, at most " + std::to_string(top) +
                                 " for this system and precision");
  plan->data.cell_rows = rows;
  return ADER_OK;
}

ader_status ader_tune(ader_plan plan, const double* u, int64_t ld, const double* dt_dev,
                      void* ws, void* stream, int reps, int* rows, double* ms_out) {
  if (!plan || !dt_dev) return fail(ADER_EINVAL, "null argument");
  if (plan->data.dim != 2) return fail(ADER_EUNSUPPORTED, "tile heights apply to 2D plans");
  if (reps < 1 || reps > 1000) return fail(ADER_EINVAL, "reps must be in 1..1000");
  if (ader_status s = check_state(plan, u, ld)) return s;
  if (ader_status s = check_ws(plan, ws)) return s;
  hipStream_t st = (hipStream_t)stream;
  const int top = ader::max_cell_rows(plan->data.prob.system, plan->data.prob.precision);
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  int best = plan->data.cell_rows;
  float best_ms = 0.0f;
  for (int i = 0; i < 4 && e == hipSuccess; ++i) {
    const int r = ader::kCellRowChoices[i];
    if (ms_out) ms_out[i] = -1.0;
    if (r > top) continue;
    // one untimed launch, then 'reps' timed launches of this height
    e = plan->impl->cell2d(plan->data, u, ld, dt_dev, (char*)ws, r, st);
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    for (int k = 0; k < reps && e == hipSuccess; ++k)
      e = plan->impl->cell2d(plan->data, u, ld, dt_dev, (char*)ws, r, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e != hipSuccess) break;
    ms /= (float)reps;
    if (ms_out) ms_out[i] = ms;
    if (best_ms == 0.0f || ms < best_ms) {
      best_ms = ms;
      best = r;
    }
  }
  if (e == hipSuccess) e = plan->impl->clear_status((char*)ws, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_status(e, "ader_tune");
  plan->data.cell_rows = best;
  if (rows) *rows = best;
  return ADER_OK;
}

ader_status ader_profile_begin(ader_plan plan) {
  if (!plan) return fail(ADER_EINVAL, "null plan");
  plan->data.prof.on = true;
  return ADER_OK;
}

ader_status ader_profile_end(ader_plan plan, double* stage_ms, int64_t* stage_launches) {
  if (!plan || !stage_ms || !stage_launches) return fail(ADER_EINVAL, "null argument");
  ader::Profiler& pr = plan->data.prof;
  for (int i = 0; i < ADER_NSTAGES; ++i) {
    stage_ms[i] = 0.0;
    stage_launches[i] = 0;
  }
  hipError_t err = hipSuccess;
  for (auto& r : pr.recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && err == hipSuccess) err = e;
    if (e == hipSuccess && r.stage >= 0 && r.stage < ADER_NSTAGES) {
      stage_ms[r.stage] += ms;
      stage_launches[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  pr.recs.clear();
  pr.on = false;
  return hip_status(err, "ader_profile_end");
}

}  // extern "C"
