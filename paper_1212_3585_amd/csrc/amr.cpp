// AMR driver: mesh construction on the host, per-level device data, the
// device-side regrid, and the
// local-time-stepping schedule of one level-0 step (Section 3), optionally
// recorded once as a HIP graph and replayed.
//
// Mesh construction (ader_amr_build), from the initial averages of every
// level's full index space:
//   1. flags: Loehner indicator (eq. indicator) > chi_ref on levels 0..L-1,
//      widened by 'buffer' Voronoi layers (or flags given by the caller);
//   2. closure: the mother of every cell in the Voronoi neighbourhood of a
//      flagged level-l cell is flagged on level l-1 (Voronoi neighbours
//      differ by at most one level; refined cells have all their Voronoi
//      neighbours on the finer level); flags nest;
//   3. status: children of flagged cells are active (virtual mothers if
//      flagged themselves); children of the active Voronoi neighbours of
//      flagged cells are virtual children;
//   4. every active cell's (2M+1)^d stencil must lie in the mesh (r >= M).
// The indicator is evaluated in plain double arithmetic, term by term, so the
// integer refinement decisions are reproducible.
//
// After the build, the status arrays and level lists live on the device only.
//
// Regrid (ader_amr_regrid), at a common time of all levels, on the device
// (kernels in amr_regrid.hip; only counts and a changed flag come back):
//   1. virtual mothers averaged; virtual children take the sub-cell averages
//      of their mothers' reconstruction, coarse to fine;
//   2. flags from the indicator variable: an active cell is refined when
//      chi > chi_ref, a virtual mother stays refined unless chi < chi_rec;
//      buffer layers, closure and status as in the build;
//   3. new level lists (stream compaction) and scratch; cells that did not
//      exist take the sub-cell averages of their mothers' reconstruction,
//      coarse to fine; removed cells are set to NaN.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "amr_plan.hpp"
#include "plan.hpp"

using ader::fail;
using ader::hip_status;

// Device buffer with a capacity; grows (never shrinks) on demand.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    if (p) {
      hipError_t e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) return e;
    }
    const size_t want = bytes + bytes / 4 + 256;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

struct ader_amr_s {
  ader_problem prob{};
  ader_amr_config cfg{};
  int d = 2, M = 0, nv = 1, r = 2, L = 0;
  ader::DevConsts dc{};
  ader::AmrConsts ac{};
  const ader::AmrImplBase* impl = nullptr;
  std::vector<ader::AmrLevel> lv;
  std::vector<std::vector<double>> h_init;
  std::vector<std::vector<uint8_t>> h_flags;
  std::vector<std::vector<int8_t>> h_status;  // during the build only
  std::vector<void*> dev_allocs;
  // per-level scratch of the active cells (wa, wh, qh, fbuf, coarse-fine
  // face list), grown on demand, and the level's dense pass buffers (3D;
  // sized by the index space)
  std::vector<std::array<DevBuf, 7>> lvl_bufs;
  // per-level dense regrid arrays: flags, dilation scratch, previous status,
  // mother slots (list capacity = the level's cells)
  struct RegridLevel {
    uint8_t* F = nullptr;
    uint8_t* T = nullptr;
    int8_t* old = nullptr;
    int32_t* slot = nullptr;
    int32_t* list = nullptr;   // second list (new cells)
    int32_t* tslot = nullptr;  // their mother slots
  };
  std::vector<RegridLevel> rg;
  // temporaries of the regrid's reconstruction of mothers (wa, wh)
  std::array<DevBuf, 2> tmp;
  void* sel_temp = nullptr;   // stream-compaction scratch
  size_t sel_bytes = 0;
  int* d_count = nullptr;     // device counters of the compactions
  unsigned int* d_changed = nullptr;
  double* partial = nullptr;
  ader::AmrClock* clock = nullptr;
  ader::AmrClock* h_clock = nullptr;  // pinned staging
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  bool built = false;
  double t_end_set = -1.0;
  uint64_t cell_updates = 0, updates_per_step = 0, regrids = 0;
  ader::AmrShape shape;  // launch shapes of the tuned kernels (ader_amr_tune)
  ader::AmrDtArgs dtargs{};
};

namespace {

int64_t ipow(int b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

struct Grid {
  int d;
  int n[3];
  int64_t cells() const { return (int64_t)n[0] * n[1] * n[2]; }
  int64_t idx(const int* c) const { return c[0] + (int64_t)n[0] * (c[1] + (int64_t)n[1] * c[2]); }
  void coords(int64_t i, int* c) const {
    c[0] = (int)(i % n[0]);
    c[1] = (int)((i / n[0]) % n[1]);
    c[2] = (int)(i / ((int64_t)n[0] * n[1]));
  }
};

int map_bc(int i, int n, int bc) {
  if (bc == ADER_BC_PERIODIC) return ((i % n) + n) % n;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Loehner indicator on a dense level grid (index units), as the oracle
// defines it term by term.
std::vector<double> lohner(const Grid& g, const double* Phi, const int* bc, double eps) {
  const int64_t N = g.cells();
  std::vector<double> chi(N, 0.0);
  auto at = [&](const int* c, const int* o) {
    int cc[3] = {c[0], c[1], c[2]};
    for (int k = 0; k < g.d; ++k) cc[k] = map_bc(c[k] + o[k], g.n[k], bc[k]);
    return Phi[g.idx(cc)];
  };
  for (int64_t i = 0; i < N; ++i) {
    int c[3];
    g.coords(i, c);
    const double P = Phi[i];
    double num = 0.0, den = 0.0;
    for (int k = 0; k < g.d; ++k) {
      for (int m = 0; m < g.d; ++m) {
        double D, De;
        if (k == m) {
          int e[3] = {0, 0, 0}, f[3] = {0, 0, 0};
          e[k] = 1;
          f[k] = -1;
          const double p = at(c, e), q = at(c, f);
          D = p - 2.0 * P + q;
          De = std::fabs(p - P) + std::fabs(P - q) +
               eps * (std::fabs(p) + 2.0 * std::fabs(P) + std::fabs(q));
        } else {
          int o[3] = {0, 0, 0};
          auto s = [&](int a, int b) {
            o[0] = o[1] = o[2] = 0;
            o[k] = a;
            o[m] = b;
            return at(c, o);
          };
          const double pp = s(1, 1), pm = s(1, -1), mp = s(-1, 1), mm = s(-1, -1);
          const double A = pp - mp, B = pm - mm;
          D = 0.25 * (A - B);
          De = 0.25 * (std::fabs(A) + std::fabs(B)) +
               0.25 * eps * (std::fabs(pp) + std::fabs(pm) + std::fabs(mp) + std::fabs(mm));
        }
        num += D * D;
        den += De * De;
      }
    }
    chi[i] = den > 0.0 ? std::sqrt(num / den) : 0.0;
  }
  return chi;
}

std::vector<uint8_t> dilate(const Grid& g, const std::vector<uint8_t>& F, const int* bc) {
  std::vector<uint8_t> out(F);
  const int64_t N = g.cells();
  const int span[3] = {1, g.d > 1 ? 1 : 0, g.d > 2 ? 1 : 0};
  for (int64_t i = 0; i < N; ++i) {
    if (!F[i]) continue;
    int c[3];
    g.coords(i, c);
    for (int dz = -span[2]; dz <= span[2]; ++dz)
      for (int dy = -span[1]; dy <= span[1]; ++dy)
        for (int dx = -span[0]; dx <= span[0]; ++dx) {
          const int o[3] = {dx, dy, dz};
          int cc[3] = {0, 0, 0};
          bool ok = true;
          for (int k = 0; k < g.d; ++k) {
            const int raw = c[k] + o[k];
            if (bc[k] != ADER_BC_PERIODIC && (raw < 0 || raw >= g.n[k])) ok = false;
            cc[k] = map_bc(raw, g.n[k], bc[k]);
          }
          if (ok) out[g.idx(cc)] = 1;
        }
  }
  return out;
}

std::vector<uint8_t> mothers(const Grid& fine, const Grid& coarse, const std::vector<uint8_t>& F,
                             int r) {
  std::vector<uint8_t> out(coarse.cells(), 0);
  for (int64_t i = 0; i < fine.cells(); ++i) {
    if (!F[i]) continue;
    int c[3];
    fine.coords(i, c);
    for (int k = 0; k < fine.d; ++k) c[k] /= r;
    out[coarse.idx(c)] = 1;
  }
  return out;
}

// Calls fn(fine index) for the r^d children of coarse cell c.
template <typename Fn>
void for_children(const Grid& coarse, const Grid& fine, int64_t c, int r, Fn fn) {
  int cc[3];
  coarse.coords(c, cc);
  const int rz = fine.d > 2 ? r : 1, ry = fine.d > 1 ? r : 1;
  for (int z = 0; z < rz; ++z)
    for (int y = 0; y < ry; ++y) {
      const int f[3] = {cc[0] * r, cc[1] * ry + y, cc[2] * rz + z};
      const int64_t row = fine.idx(f);
      for (int x = 0; x < r; ++x) fn(row + x);
    }
}

std::vector<uint8_t> children(const Grid& coarse, const Grid& fine, const std::vector<uint8_t>& F,
                              int r) {
  std::vector<uint8_t> out(fine.cells(), 0);
  for (int64_t c = 0; c < coarse.cells(); ++c)
    if (F[c]) for_children(coarse, fine, c, r, [&](int64_t i) { out[i] = 1; });
  return out;
}

using Flags = std::vector<std::vector<uint8_t>>;
using Status = std::vector<std::vector<int8_t>>;

// Rules 4 and 5: the mother of every cell in the Voronoi neighbourhood of a
// flagged level-l cell is flagged on level l-1; flags nest.
void close_flags(const std::vector<Grid>& g, Flags& F, const int* bc, int r, int L) {
  for (int l = L - 1; l >= 1; --l) {
    std::vector<uint8_t> m = mothers(g[l], g[l - 1], dilate(g[l], F[l], bc), r);
    for (size_t i = 0; i < m.size(); ++i) F[l - 1][i] |= m[i];
  }
  for (int l = 1; l < L; ++l) {
    std::vector<uint8_t> c = children(g[l - 1], g[l], F[l - 1], r);
    for (size_t i = 0; i < c.size(); ++i) F[l][i] &= c[i];
  }
}

// Status of every level from closed flags: children of flagged cells are
// active (virtual mothers if flagged themselves), children of the unflagged
// Voronoi neighbours of flagged cells are virtual children, the rest of
// levels >= 1 is absent.  Written block by block over the coarser level.
Status status_from_flags(const std::vector<Grid>& g, const Flags& F, const int* bc, int r,
                         int L) {
  Status S(L + 1);
  S[0].assign(g[0].cells(), ader::kActive);
  if (L > 0)
    for (int64_t i = 0; i < g[0].cells(); ++i)
      if (F[0][i]) S[0][i] = ader::kVMother;
  for (int l = 1; l <= L; ++l) {
    const std::vector<uint8_t> near = dilate(g[l - 1], F[l - 1], bc);
    const std::vector<uint8_t>& fl = F[l - 1];
    std::vector<int8_t>& s = S[l];
    s.assign(g[l].cells(), ader::kAbsent);
    for (int64_t c = 0; c < g[l - 1].cells(); ++c) {
      if (fl[c]) {
        if (l < L) {
          const std::vector<uint8_t>& ff = F[l];
          for_children(g[l - 1], g[l], c, r,
                       [&](int64_t i) { s[i] = ff[i] ? ader::kVMother : ader::kActive; });
        } else {
          for_children(g[l - 1], g[l], c, r, [&](int64_t i) { s[i] = ader::kActive; });
        }
      } else if (near[c]) {
        for_children(g[l - 1], g[l], c, r, [&](int64_t i) { s[i] = ader::kVChild; });
      }
    }
  }
  return S;
}

// Every active cell's (2M+1)^d stencil lies in the mesh.
bool stencils_in_mesh(const std::vector<Grid>& g, const Status& S, const int* bc, int M) {
  for (size_t l = 0; l < S.size(); ++l) {
    const std::vector<int8_t>& s = S[l];
    const int d = g[l].d;
    for (int64_t i = 0; i < g[l].cells(); ++i) {
      if (s[i] != ader::kActive) continue;
      int c[3];
      g[l].coords(i, c);
      const int spanz = d > 2 ? M : 0;
      for (int oz = -spanz; oz <= spanz; ++oz)
        for (int oy = -M; oy <= M; ++oy)
          for (int ox = -M; ox <= M; ++ox) {
            const int o[3] = {ox, oy, oz};
            int cc[3] = {0, 0, 0};
            for (int k = 0; k < d; ++k) cc[k] = map_bc(c[k] + o[k], g[l].n[k], bc[k]);
            if (s[g[l].idx(cc)] == ader::kAbsent) return false;
          }
    }
  }
  return true;
}

template <typename T>
ader_status upload(ader_amr a, T** dst, const void* src, size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 256);
  if (e != hipSuccess) return hip_status(e, "ader_amr_build (allocation)");
  a->dev_allocs.push_back(p);
  if (src && bytes) {
    e = hipMemcpy(p, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_status(e, "ader_amr_build (upload)");
  }
  *dst = static_cast<T*>(p);
  return ADER_OK;
}

// Copy 'bytes' from host 'src' (may be null) into a grown buffer.
template <typename T>
hipError_t fill_buf(DevBuf& b, T** dst, const void* src, size_t bytes) {
  hipError_t e = b.ensure(bytes);
  if (e == hipSuccess && src && bytes) e = hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
  *dst = static_cast<T*>(b.p);
  return e;
}

ader::RgGrid rg_grid(const ader_amr_s* a, int l) {
  ader::RgGrid g;
  g.dim = a->d;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = a->lv[l].n[k];
    g.bc[k] = k < a->d ? a->prob.bc[k] : ADER_BC_PERIODIC;
  }
  g.N = a->lv[l].ncells;
  return g;
}

// Number selected by a compaction (synchronous read of the device counter).
hipError_t select_count(ader_amr a, int mode, const int8_t* st, const int8_t* old, int64_t N,
                        int32_t* out, int64_t* count) {
  size_t bytes = a->sel_bytes;
  hipError_t e = ader::rg_select(mode, st, old, N, out, a->d_count, a->sel_temp, &bytes,
                                 a->stream);
  int c = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&c, a->d_count, sizeof(int), hipMemcpyDeviceToHost, a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  *count = c;
  return e;
}

// The coarse-fine face lists of every level (after all levels' lists are
// set: a level's faces depend on its neighbours in level l - 1 and l + 1).
ader_status set_cf_lists(ader_amr a) {
  hipError_t e = hipSuccess;
  for (int l = 0; l <= a->L && e == hipSuccess; ++l) {
    ader::AmrLevel& v = a->lv[l];
    int c = 0;
    e = hipMemsetAsync(a->d_count, 0, sizeof(int), a->stream);
    if (e == hipSuccess)
      e = a->impl->cf_faces(v, l > 0 ? &a->lv[l - 1] : nullptr,
                            l < a->L ? &a->lv[l + 1] : nullptr, a->ac, a->d_count, a->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&c, a->d_count, sizeof(int), hipMemcpyDeviceToHost, a->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
    v.ncf = c;
  }
  if (e != hipSuccess) return hip_status(e, "AMR coarse-fine face lists");
  return ADER_OK;
}

// Lists, positions and scratch of level l from its device status.
ader_status set_level_lists(ader_amr a, int l) {
  ader::AmrLevel& v = a->lv[l];
  const int64_t N = v.ncells;
  const int M = a->M, d = a->d;
  hipError_t e = select_count(a, ader::kSelActive, v.st, nullptr, N, v.act, &v.nact);
  if (e == hipSuccess) e = select_count(a, ader::kSelVChild, v.st, nullptr, N, v.vc, &v.nvc);
  if (e == hipSuccess) e = select_count(a, ader::kSelVMother, v.st, nullptr, N, v.vm, &v.nvm);
  if (e == hipSuccess) e = ader::rg_positions(v.pos, N, v.act, v.nact, a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  std::array<DevBuf, 7>& B = a->lvl_bufs[l];
  const size_t na = (size_t)v.nact;
  const size_t dense = sizeof(double) * a->impl->dense_weno_per_cell() * (size_t)N;
  if (e == hipSuccess && dense > 0 && !v.dwx) {
    // allocated once (the index space is fixed) and zeroed, so that lines no
    // reconstruction reads never hold uninitialised memory
    e = fill_buf(B[4], &v.dwx, nullptr, dense);
    if (e == hipSuccess) e = hipMemsetAsync(v.dwx, 0, dense, a->stream);
  }
  if (e == hipSuccess)
    e = fill_buf(B[0], &v.wa, nullptr, sizeof(double) * a->impl->weno_scratch_per_cell() * na);
  if (e == hipSuccess)
    e = fill_buf(B[1], &v.wh, nullptr, sizeof(double) * a->impl->wh_per_cell() * na);
  if (e == hipSuccess)
    e = fill_buf(B[2], &v.qh, nullptr, a->impl->qh_elem_size() * a->nv * ipow(M + 1, d + 1) * na);
  if (e == hipSuccess)
    e = fill_buf(B[3], &v.fbuf, nullptr, sizeof(double) * a->impl->fbuf_per_cell() * na);
  if (e == hipSuccess)
    e = fill_buf(B[5], &v.cf, nullptr, sizeof(int32_t) * ader::kAmrCfRecord * 2 * d * na);
  if (e == hipSuccess) e = fill_buf(B[6], &v.fc, nullptr, sizeof(int32_t) * 2 * d * na);
  if (e != hipSuccess) return hip_status(e, "AMR level lists");
  v.wb = v.wa + (size_t)a->nv * (M + 1) * ipow(2 * M + 1, d - 1) * na;
  a->dtargs.nb[l] = v.nact == 0 ? 0
                    : (int)std::min<int64_t>((v.nact + ader::kBlock - 1) / ader::kBlock,
                                             ader::kDtMaxBlocks);
  a->updates_per_step = 0;
  for (int k = 0; k <= a->L; ++k)
    a->updates_per_step += (uint64_t)a->lv[k].nact * (uint64_t)ipow(a->r, k);
  return ADER_OK;
}

// Level-l cells 'targets' (device list, nt of them) from the reconstruction of
// their mothers on level l-1, listed in 'moth' (nm cells, the slot of each
// level-(l-1) cell in slot_c); wa, wb, wh hold the mothers' scratch.
hipError_t children_from(ader_amr a, int l, const int32_t* moth, int64_t nm, const int32_t* slot_c,
                         double* wa, double* wb, double* wh, const int32_t* targets, int64_t nt) {
  if (nt == 0 || nm == 0) return hipSuccess;
  int32_t* tslot = a->rg[l].tslot;
  hipError_t e = ader::rg_slots(rg_grid(a, l), rg_grid(a, l - 1), a->r, targets, nt, slot_c,
                                tslot, a->stream);
  if (e == hipSuccess)
    e = a->impl->children(a->lv[l - 1], moth, nm, wa, wb, wh, a->lv[l], targets, tslot, nt,
                          a->dc, a->ac, a->stream);
  return e;
}

// Records level l's substep 'sub': the finer levels' substeps recursively
// between its predictor and its update.  A finer level's substep (defer_apply)
// computes its face fluxes and leaves the update of its cells to the next
// launch that can carry it: the next substep's preparation (prepare with
// apply_dt), or after the last substep of the run the coarser level's face
// launch (update with pend).  They write disjoint cells and read none of the
// deferred update's.
ader_status record_advance(ader_amr a, int l, int sub, bool defer_apply, bool pending_apply,
                           hipStream_t st) {
  const ader::AmrImplBase* im = a->impl;
  hipError_t e = hipSuccess;
  // virtual mothers of the finer levels, finest first (they read finer
  // levels only, so they may precede the pending update); then this level's
  // averaging, projection, the finer level's memory and the pending update
  // in one launch
  for (int lev = a->L - 1; lev > l && e == hipSuccess; --lev)
    e = im->average(a->lv[lev], a->lv[lev + 1], a->r, st);
  if (e == hipSuccess)
    e = im->prepare(a->lv[l], l > 0 ? &a->lv[l - 1] : nullptr,
                    l < a->L ? &a->lv[l + 1] : nullptr, a->ac, sub,
                    pending_apply ? &a->clock->dt[l] : nullptr, st);
  if (e == hipSuccess) e = im->predict(a->lv[l], &a->clock->dt[l], a->dc, a->shape, st);
  if (e != hipSuccess) return hip_status(e, "ader_amr_step");
  if (l < a->L)
    for (int s = 0; s < a->r; ++s)
      if (ader_status stt = record_advance(a, l + 1, s, true, s > 0, st)) return stt;
  e = im->update(a->lv[l], l > 0 ? &a->lv[l - 1] : nullptr, l < a->L ? &a->lv[l + 1] : nullptr,
                 &a->clock->dt[l], sub, a->dc, a->ac, a->shape, !defer_apply,
                 l < a->L ? &a->lv[l + 1] : nullptr, l < a->L ? &a->clock->dt[l + 1] : nullptr,
                 st);
  return hip_status(e, "ader_amr_step");
}

ader_status record_step(ader_amr a, hipStream_t st) {
  hipError_t e = hipSuccess;
  e = a->impl->cfl(a->lv.data(), a->L + 1, a->partial, a->dtargs.nb, st);
  if (e == hipSuccess) e = ader::launch_amr_dt(a->partial, a->dtargs, a->clock, a->lv[0].hdr, st);
  if (e != hipSuccess) return hip_status(e, "ader_amr_step");
  if (ader_status s = record_advance(a, 0, 0, false, false, st)) return s;
  for (int lev = a->L - 1; lev >= 0 && e == hipSuccess; --lev)
    e = a->impl->average(a->lv[lev], a->lv[lev + 1], a->r, st);
  return hip_status(e, "ader_amr_step");
}

}  // namespace

extern "C" {

ader_status ader_amr_create(const ader_problem* prob, const ader_amr_config* cfg, ader_amr* out) {
  if (!prob || !cfg || !out) return fail(ADER_EINVAL, "null argument");
  *out = nullptr;
  int64_t ncells = 0;
  if (ader_status s = ader::validate_problem(*prob, &ncells)) return s;
  if (cfg->max_level < 0 || cfg->max_level >= ader::kAmrMaxLevels)
    return fail(ADER_EINVAL, "max_level must be in 0..5");
  const int rmin = prob->M > 2 ? prob->M : 2;
  if (cfg->r < rmin || cfg->r > ader::kAmrMaxR)
    return fail(ADER_EINVAL, "the refinement factor must satisfy max(M, 2) <= r <= 4");
  const int nv = prob->system == ADER_SYS_LINADV ? 1
                 : (prob->system == ADER_SYS_EULER ? prob->dim + 2 : 9);
  if (cfg->indicator_var < 0 || cfg->indicator_var >= nv)
    return fail(ADER_EINVAL, "indicator_var out of range");
  if (!std::isfinite(cfg->chi_ref) || !std::isfinite(cfg->eps) || cfg->eps < 0.0)
    return fail(ADER_EINVAL, "chi_ref and eps must be finite, eps >= 0");
  if (!std::isfinite(cfg->chi_rec) || cfg->chi_rec > cfg->chi_ref)
    return fail(ADER_EINVAL, "chi_rec must be finite and at most chi_ref");
  if (cfg->buffer < 0 || cfg->buffer > 4) return fail(ADER_EINVAL, "buffer must be in 0..4");
  // every level's cell count and the indices of the finest level must fit
  int64_t fine = ncells * ipow(cfg->r, cfg->max_level * prob->dim);
  if (fine > (int64_t(1) << 30)) return fail(ADER_EUNSUPPORTED, "more than 2^30 cells on a level");
  ader_amr a = new (std::nothrow) ader_amr_s();
  if (!a) return fail(ADER_EINVAL, "out of host memory");
  a->prob = *prob;
  if (prob->dim == 2) a->prob.n[2] = 1;
  a->cfg = *cfg;
  a->d = prob->dim;
  a->M = prob->M;
  a->nv = nv;
  a->r = cfg->r;
  a->L = cfg->max_level;
  a->impl = a->d == 2 ? ader::make_amr_impl_2d(a->M, prob->system, prob->precision)
                      : ader::make_amr_impl_3d(a->M, prob->system, prob->precision);
  ader::RefConstants ref;
  ader::AmrTables tab;
  if (!a->impl || !ader::build_ref_constants(a->M, &ref) ||
      !ader::build_amr_tables(a->M, a->r, &tab)) {
    delete a;
    return fail(ADER_EUNSUPPORTED, "no AMR kernels or tables for this configuration");
  }
  ader::fill_dev_consts(ref, a->M, &a->dc);
  std::memset(&a->ac, 0, sizeof(a->ac));
  a->ac.r = a->r;
  for (int i = 0; i < a->r; ++i)
    for (int p = 0; p <= a->M; ++p) {
      a->ac.sub_avg[i][p] = (double)tab.sub_avg[i][p];
      a->ac.at_sub[i][p] = (double)tab.at_sub[i][p];
      a->ac.at_face[i][0][p] = (double)tab.at_face[i][0][p];
      a->ac.at_face[i][1][p] = (double)tab.at_face[i][1][p];
      for (int b = 0; b <= a->M; ++b) a->ac.at_nodes[i][b][p] = (double)tab.at_nodes[i][b][p];
    }
  a->lv.resize(a->L + 1);
  a->h_init.resize(a->L + 1);
  a->h_flags.resize(a->L + 1);
  for (int l = 0; l <= a->L; ++l) {
    ader::AmrLevel& v = a->lv[l];
    const int64_t f = ipow(a->r, l);
    for (int k = 0; k < 3; ++k) v.n[k] = k < a->d ? (int)(a->prob.n[k] * f) : 1;
    v.ncells = (int64_t)v.n[0] * v.n[1] * v.n[2];
  }
  *out = a;
  return ADER_OK;
}

ader_status ader_amr_destroy(ader_amr a) {
  if (!a) return ADER_OK;
  if (a->stream) (void)hipStreamSynchronize(a->stream);
  if (a->exec) (void)hipGraphExecDestroy(a->exec);
  for (void* p : a->dev_allocs) (void)hipFree(p);
  for (auto& v : a->lvl_bufs)
    for (DevBuf& b : v) b.release();
  for (DevBuf& b : a->tmp) b.release();
  if (a->h_clock) (void)hipHostFree(a->h_clock);
  if (a->stream) (void)hipStreamDestroy(a->stream);
  delete a;
  return ADER_OK;
}

ader_status ader_amr_level_cells(ader_amr a, int level, int n[3]) {
  if (!a || !n || level < 0 || level > a->L) return fail(ADER_EINVAL, "bad level");
  for (int k = 0; k < 3; ++k) n[k] = a->lv[level].n[k];
  return ADER_OK;
}

ader_status ader_amr_set_level(ader_amr a, int level, const double* u) {
  if (!a || !u || level < 0 || level > a->L) return fail(ADER_EINVAL, "bad level or pointer");
  if (a->built) return fail(ADER_EINVAL, "the mesh is already built");
  const int64_t N = a->lv[level].ncells;
  a->h_init[level].assign(u, u + (size_t)a->nv * N);
  return ADER_OK;
}

ader_status ader_amr_set_flags(ader_amr a, int level, const uint8_t* flags) {
  if (!a || !flags || level < 0 || level >= a->L) return fail(ADER_EINVAL, "bad level or pointer");
  const int64_t N = a->lv[level].ncells;
  a->h_flags[level].assign(flags, flags + N);
  for (auto& x : a->h_flags[level]) x = x ? 1 : 0;
  return ADER_OK;
}

ader_status ader_amr_build(ader_amr a) {
  if (!a) return fail(ADER_EINVAL, "null argument");
  if (a->built) return fail(ADER_EINVAL, "the mesh is already built");
  const int d = a->d, r = a->r, L = a->L, nv = a->nv;
  const int* bc = a->prob.bc;
  std::vector<Grid> g(L + 1);
  for (int l = 0; l <= L; ++l) {
    g[l].d = d;
    for (int k = 0; k < 3; ++k) g[l].n[k] = a->lv[l].n[k];
    if (a->h_init[l].size() != (size_t)nv * g[l].cells())
      return fail(ADER_EINVAL, "initial averages missing for level " + std::to_string(l));
  }
  // 1. flags
  std::vector<std::vector<uint8_t>> F(L);
  for (int l = 0; l < L; ++l) {
    if (!a->h_flags[l].empty()) {
      F[l] = a->h_flags[l];
    } else {
      const double* Phi = a->h_init[l].data() + (size_t)a->cfg.indicator_var * g[l].cells();
      std::vector<double> chi = lohner(g[l], Phi, bc, a->cfg.eps);
      F[l].resize(chi.size());
      for (size_t i = 0; i < chi.size(); ++i) F[l][i] = chi[i] > a->cfg.chi_ref ? 1 : 0;
      for (int b = 0; b < a->cfg.buffer; ++b) F[l] = dilate(g[l], F[l], bc);
    }
  }
  // 2. closure and nesting, 3. status, 4. every active stencil lies in the mesh
  close_flags(g, F, bc, r, L);
  a->h_status = status_from_flags(g, F, bc, r, L);
  if (!stencils_in_mesh(g, a->h_status, bc, a->M))
    return fail(ADER_EINVAL, "an active cell's stencil leaves the mesh");
  for (auto& f : a->h_flags) f.clear();
  // 5. device data
  hipError_t e = hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_status(e, "ader_amr_build");
  const double dx0[3] = {(a->prob.hi[0] - a->prob.lo[0]) / a->prob.n[0],
                         (a->prob.hi[1] - a->prob.lo[1]) / a->prob.n[1],
                         d > 2 ? (a->prob.hi[2] - a->prob.lo[2]) / a->prob.n[2] : 1.0};
  a->lvl_bufs.resize(L + 1);
  a->rg.assign(L + 1, {});
  {
    // compaction scratch for the largest level, device counters
    int64_t nmax = 0;
    for (int l = 0; l <= L; ++l) nmax = std::max<int64_t>(nmax, a->lv[l].ncells);
    size_t bytes = 0;
    e = ader::rg_select(ader::kSelActive, nullptr, nullptr, nmax, nullptr, nullptr, nullptr,
                        &bytes, a->stream);
    if (e != hipSuccess) return hip_status(e, "ader_amr_build (compaction scratch)");
    a->sel_bytes = bytes;
    if (ader_status st = upload(a, &a->sel_temp, nullptr, bytes)) return st;
    if (ader_status st = upload(a, &a->d_count, nullptr, sizeof(int) * 4)) return st;
    if (ader_status st = upload(a, &a->d_changed, nullptr, sizeof(unsigned int))) return st;
  }
  for (int l = 0; l <= L; ++l) {
    ader::AmrLevel& v = a->lv[l];
    const int64_t N = v.ncells;
    const std::vector<int8_t>& s = a->h_status[l];
    std::vector<double> u0(a->h_init[l]);
    for (int64_t i = 0; i < N; ++i)
      if (s[i] == ader::kAbsent)
        for (int q = 0; q < nv; ++q) u0[(size_t)q * N + i] = std::nan("");
    ader_status st = ADER_OK;
    if (!st) st = upload(a, &v.u, u0.data(), sizeof(double) * nv * N);
    if (!st) st = upload(a, &v.st, s.data(), N);
    if (!st) st = upload(a, &v.pos, nullptr, sizeof(int32_t) * N);
    if (!st) st = upload(a, &v.act, nullptr, sizeof(int32_t) * N);
    if (!st) st = upload(a, &v.vc, nullptr, sizeof(int32_t) * N);
    if (!st) st = upload(a, &v.vm, nullptr, sizeof(int32_t) * N);
    if (!st && l > 0) st = upload(a, &v.mem, nullptr, sizeof(double) * d * 2 * nv * N);
    std::vector<char> zero(ader::kHeaderBytes, 0);
    if (!st) st = upload(a, &v.hdr, zero.data(), ader::kHeaderBytes);
    auto& R = a->rg[l];
    if (!st && l < L) st = upload(a, &R.F, nullptr, N);
    if (!st) st = upload(a, &R.T, nullptr, N);
    if (!st) st = upload(a, &R.old, nullptr, N);
    if (!st && l < L) st = upload(a, &R.slot, nullptr, sizeof(int32_t) * N);
    if (!st) st = upload(a, &R.list, nullptr, sizeof(int32_t) * N);
    if (!st) st = upload(a, &R.tslot, nullptr, sizeof(int32_t) * N);
    if (st) return st;
    ader_problem pl = a->prob;
    for (int k = 0; k < d; ++k) pl.n[k] = v.n[k];
    ader::fill_mesh_params(pl, N, &v.mp);
    for (int k = 0; k < d; ++k) v.dx[k] = v.mp.dx[k] = dx0[k] / (double)ipow(r, l);
    v.mp.ld = N;
  }
  for (int l = 0; l <= L; ++l)
    if (ader_status st = set_level_lists(a, l)) return st;
  if (ader_status st = set_cf_lists(a)) return st;
  a->h_status.clear();
  a->h_status.shrink_to_fit();
  a->dtargs.nlev = L + 1;
  a->dtargs.r = r;
  a->dtargs.cfl = a->prob.cfl;
  if (ader_status st = upload(a, &a->partial, nullptr,
                              sizeof(double) * ader::kDtMaxBlocks * (L + 1)))
    return st;
  std::vector<char> clk(sizeof(ader::AmrClock), 0);
  if (ader_status st = upload(a, &a->clock, clk.data(), clk.size())) return st;
  e = hipHostMalloc(&a->h_clock, sizeof(ader::AmrClock), hipHostMallocDefault);
  if (e != hipSuccess) return hip_status(e, "ader_amr_build");
  std::memset(a->h_clock, 0, sizeof(ader::AmrClock));
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_status(e, "ader_amr_build");
  a->built = true;
  return ADER_OK;
}

ader_status ader_amr_step(ader_amr a, double t_end, void* stream) {
  if (!a) return fail(ADER_EINVAL, "null argument");
  if (!a->built) return fail(ADER_EINVAL, "build the mesh first");
  if (!std::isfinite(t_end)) return fail(ADER_EINVAL, "t_end must be finite");
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : a->stream;
  hipError_t e = hipSuccess;
  if (t_end != a->t_end_set) {
    // the end time lives in the device clock (the recorded step reads it)
    e = hipStreamSynchronize(st);
    if (e == hipSuccess)
      e = hipMemcpy(&a->clock->t_end, &t_end, sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_status(e, "ader_amr_step");
    a->t_end_set = t_end;
  }
  if (a->cfg.use_graph) {
    if (!a->exec) {
      hipGraph_t graph = nullptr;
      e = hipStreamBeginCapture(a->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_status(e, "ader_amr_step (capture)");
      ader_status rs = record_step(a, a->stream);
      e = hipStreamEndCapture(a->stream, &graph);
      if (rs) {
        if (graph) (void)hipGraphDestroy(graph);
        return rs;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&a->exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_status(e, "ader_amr_step (graph)");
    }
    e = hipGraphLaunch(a->exec, st);
    if (e != hipSuccess) return hip_status(e, "ader_amr_step (graph launch)");
  } else {
    if (ader_status rs = record_step(a, st)) return rs;
  }
  a->cell_updates += a->updates_per_step;
  return ADER_OK;
}

ader_status ader_amr_regrid(ader_amr a, int* changed) {
  if (changed) *changed = 0;
  if (!a || !a->built) return fail(ADER_EINVAL, "mesh not built");
  const int r = a->r, L = a->L;
  if (L == 0) return ADER_OK;
  hipStream_t st = a->stream;
  std::vector<ader::RgGrid> g(L + 1);
  for (int l = 0; l <= L; ++l) g[l] = rg_grid(a, l);
  hipError_t e = hipDeviceSynchronize();
  // 1. virtual mothers, then virtual children from their mothers (the level's
  //    reconstruction of its active cells), coarse to fine
  for (int lev = L - 1; lev >= 0 && e == hipSuccess; --lev)
    e = a->impl->average(a->lv[lev], a->lv[lev + 1], r, st);
  for (int l = 1; l <= L && e == hipSuccess; ++l) {
    const ader::AmrLevel& c = a->lv[l - 1];
    e = children_from(a, l, c.act, c.nact, c.pos, c.wa, c.wb, c.wh, a->lv[l].vc, a->lv[l].nvc);
  }
  // 2. flags: refine active cells above chi_ref, keep virtual mothers down to
  //    chi_rec (or the caller's flags), buffer layers
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    auto& R = a->rg[l];
    const int64_t N = g[l].N;
    if (!a->h_flags[l].empty()) {
      e = hipMemcpyAsync(R.F, a->h_flags[l].data(), N, hipMemcpyHostToDevice, st);
      continue;
    }
    e = ader::rg_lohner(g[l], a->lv[l].u + (size_t)a->cfg.indicator_var * N, a->lv[l].st,
                        a->cfg.eps, a->cfg.chi_ref, a->cfg.chi_rec, R.F, st);
    for (int b = 0; b < a->cfg.buffer && e == hipSuccess; ++b) {
      e = ader::rg_dilate(g[l], R.F, R.T, st);
      if (e == hipSuccess) e = hipMemcpyAsync(R.F, R.T, N, hipMemcpyDeviceToDevice, st);
    }
  }
  //    closure (rules 4, 5) and nesting
  for (int l = L - 1; l >= 1 && e == hipSuccess; --l) {
    e = ader::rg_dilate(g[l], a->rg[l].F, a->rg[l].T, st);
    if (e == hipSuccess) e = ader::rg_mothers_or(g[l], g[l - 1], r, a->rg[l].T, a->rg[l - 1].F, st);
  }
  for (int l = 1; l < L && e == hipSuccess; ++l)
    e = ader::rg_nest(g[l], g[l - 1], r, a->rg[l - 1].F, a->rg[l].F, st);
  // 3. status of every level (the previous one kept), changed?
  for (int l = 0; l <= L && e == hipSuccess; ++l)
    e = hipMemcpyAsync(a->rg[l].old, a->lv[l].st, g[l].N, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = ader::rg_status0(g[0].N, a->rg[0].F, a->lv[0].st, st);
  for (int l = 1; l <= L && e == hipSuccess; ++l) {
    e = ader::rg_dilate(g[l - 1], a->rg[l - 1].F, a->rg[l - 1].T, st);
    if (e == hipSuccess)
      e = ader::rg_status(g[l], g[l - 1], r, a->rg[l - 1].F, a->rg[l - 1].T,
                          l < L ? a->rg[l].F : nullptr, a->lv[l].st, st);
  }
  unsigned int ch = 0;
  if (e == hipSuccess) e = hipMemsetAsync(a->d_changed, 0, sizeof(unsigned int), st);
  for (int l = 0; l <= L && e == hipSuccess; ++l)
    e = ader::rg_diff(g[l].N, a->lv[l].st, a->rg[l].old, a->d_changed, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&ch, a->d_changed, sizeof(unsigned int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (auto& f : a->h_flags) f.clear();
  if (e != hipSuccess) return hip_status(e, "ader_amr_regrid");
  if (!ch) return ADER_OK;
  // (the stencil check of the build holds by construction here: an active
  // cell's stencil, M <= r cells wide, lies in the children of its mother's
  // Voronoi neighbours, which are flagged or near-flagged)
  // 4. new lists; new cells from their mothers' reconstruction, coarse to
  //    fine (a new cell's mother may be new itself); removed cells NaN
  for (int l = 0; l <= L; ++l)
    if (ader_status s = set_level_lists(a, l)) return s;
  if (ader_status s = set_cf_lists(a)) return s;
  for (int l = 1; l <= L && e == hipSuccess; ++l) {
    const int64_t Nc = g[l - 1].N, Nf = g[l].N;
    auto& Rc = a->rg[l - 1];
    auto& Rf = a->rg[l];
    int64_t nm = 0, nt = 0;
    e = select_count(a, ader::kSelMothers, a->lv[l - 1].st, nullptr, Nc, Rc.list, &nm);
    if (e == hipSuccess) e = select_count(a, ader::kSelBorn, a->lv[l].st, Rf.old, Nf, Rf.list, &nt);
    if (e != hipSuccess || nt == 0) continue;
    if (e == hipSuccess) e = ader::rg_positions(Rc.slot, Nc, Rc.list, nm, st);
    double *wa = nullptr, *wh = nullptr;
    if (e == hipSuccess)
      e = fill_buf(a->tmp[0], &wa, nullptr,
                   sizeof(double) * a->impl->weno_scratch_per_cell() * (size_t)nm);
    if (e == hipSuccess)
      e = fill_buf(a->tmp[1], &wh, nullptr, sizeof(double) * a->impl->wh_per_cell() * (size_t)nm);
    if (e != hipSuccess) break;
    double* wb = wa + (size_t)a->nv * (a->M + 1) * ipow(2 * a->M + 1, a->d - 1) * nm;
    e = children_from(a, l, Rc.list, nm, Rc.slot, wa, wb, wh, Rf.list, nt);
  }
  for (int l = 1; l <= L && e == hipSuccess; ++l)
    e = ader::rg_gone(g[l].N, a->nv, a->lv[l].u, a->lv[l].st, a->rg[l].old, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_status(e, "ader_amr_regrid");
  // the recorded step holds the old lists: record again at the next step
  if (a->exec) {
    (void)hipGraphExecDestroy(a->exec);
    a->exec = nullptr;
  }
  a->regrids += 1;
  if (changed) *changed = 1;
  return ADER_OK;
}

ader_status ader_amr_tune(ader_amr a, int reps, int* pred_block, int* flux_block,
                          double* ms_out) {
  if (!a || !a->built) return fail(ADER_EINVAL, "mesh not built");
  if (reps < 1 || reps > 1000) return fail(ADER_EINVAL, "reps must be in 1..1000");
  if (a->cell_updates == 0) return fail(ADER_EINVAL, "take a step first (the level steps)");
  hipStream_t st = a->stream;
  hipError_t e = hipDeviceSynchronize();
  // the level with the most active cells
  int lt = 0;
  for (int l = 1; l <= a->L; ++l)
    if (a->lv[l].nact > a->lv[lt].nact) lt = l;
  const ader::AmrLevel& v = a->lv[lt];
  const ader::AmrLevel* coarse = lt > 0 ? &a->lv[lt - 1] : nullptr;
  const ader::AmrLevel* fine = lt < a->L ? &a->lv[lt + 1] : nullptr;
  // the tuning launches must not count in the statistics
  std::vector<ader::WsHeader> saved(a->L + 1);
  for (int l = 0; l <= a->L && e == hipSuccess; ++l)
    e = hipMemcpy(&saved[l], a->lv[l].hdr, sizeof(ader::WsHeader), hipMemcpyDeviceToHost);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  ader::AmrShape best = a->shape;
  float best_ms[2] = {0.0f, 0.0f};
  for (int which = 0; which < 2 && e == hipSuccess; ++which) {
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
      const int b = ader::kAmrBlockChoices[i];
      double* slot = ms_out ? &ms_out[which * 3 + i] : nullptr;
      if (slot) *slot = -1.0;
      if (v.nact == 0 || (which == 0 && !a->impl->pred_block_ok(b))) continue;
      ader::AmrShape sh = a->shape;
      sh.pred_block = b;
      auto run = [&]() {
        return which == 0 ? a->impl->predict(v, &a->clock->dt[lt], a->dc, sh, st)
                          : a->impl->flux_only(v, coarse, fine, &a->clock->dt[lt], 0, a->dc,
                                               a->ac, b, st);
      };
      e = run();  // untimed
      if (e == hipSuccess) e = hipEventRecord(ev[0], st);
      for (int k = 0; k < reps && e == hipSuccess; ++k) e = run();
      if (e == hipSuccess) e = hipEventRecord(ev[1], st);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e != hipSuccess) break;
      ms /= (float)reps;
      if (slot) *slot = ms;
      if (best_ms[which] == 0.0f || ms < best_ms[which]) {
        best_ms[which] = ms;
        if (which == 0)
          best.pred_block = b;
        else
          best.flux_block = b;
      }
    }
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  for (int l = 0; l <= a->L && e == hipSuccess; ++l)
    e = hipMemcpy(a->lv[l].hdr, &saved[l], sizeof(ader::WsHeader), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_status(e, "ader_amr_tune");
  a->shape = best;
  if (a->exec) {  // the recorded step holds the old shapes
    (void)hipGraphExecDestroy(a->exec);
    a->exec = nullptr;
  }
  if (pred_block) *pred_block = best.pred_block;
  if (flux_block) *flux_block = best.flux_block;
  return ADER_OK;
}

ader_status ader_amr_clock(ader_amr a, double* t, int64_t* steps, double* dt0) {
  if (!a || !a->built) return fail(ADER_EINVAL, "mesh not built");
  hipError_t e = hipStreamSynchronize(a->stream);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(a->h_clock, a->clock, sizeof(ader::AmrClock), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e, "ader_amr_clock");
  if (t) *t = a->h_clock->t;
  if (steps) *steps = (int64_t)a->h_clock->steps;
  if (dt0) *dt0 = a->h_clock->dt[0];
  return ADER_OK;
}

ader_status ader_amr_get_level(ader_amr a, int level, double* u, int8_t* status) {
  if (!a || !a->built || level < 0 || level > a->L) return fail(ADER_EINVAL, "bad level");
  hipError_t e = hipDeviceSynchronize();
  const ader::AmrLevel& v = a->lv[level];
  if (e == hipSuccess && u)
    e = hipMemcpy(u, v.u, sizeof(double) * a->nv * v.ncells, hipMemcpyDeviceToHost);
  if (e == hipSuccess && status) e = hipMemcpy(status, v.st, v.ncells, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e, "ader_amr_get_level");
  return ADER_OK;
}

ader_status ader_amr_counts(ader_amr a, int level, int64_t counts[3]) {
  if (!a || !a->built || !counts || level < 0 || level > a->L)
    return fail(ADER_EINVAL, "bad level");
  counts[0] = a->lv[level].nact;
  counts[1] = a->lv[level].nvc;
  counts[2] = a->lv[level].nvm;
  return ADER_OK;
}

ader_status ader_amr_stats(ader_amr a, uint32_t* flags, uint64_t* picard_iterations,
                           uint64_t* cell_updates) {
  if (!a || !a->built) return fail(ADER_EINVAL, "mesh not built");
  hipError_t e = hipDeviceSynchronize();
  uint32_t f = 0;
  uint64_t it = 0;
  for (int l = 0; l <= a->L && e == hipSuccess; ++l) {
    ader::WsHeader h;
    e = hipMemcpy(&h, a->lv[l].hdr, sizeof(h), hipMemcpyDeviceToHost);
    f |= h.status;
    for (int k = 0; k < ader::kCounterSlots; ++k) it += h.iters[k];
  }
  if (e != hipSuccess) return hip_status(e, "ader_amr_stats");
  if (flags) *flags = f;
  if (picard_iterations) *picard_iterations = it;
  if (cell_updates) *cell_updates = a->cell_updates;
  return ADER_OK;
}

}  // extern "C"
