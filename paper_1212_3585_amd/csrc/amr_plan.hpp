// Device-side data of an AMR mesh (Section 3) shared by the driver
// (amr.cpp) and the templated launchers (amr_impl.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace ader {

constexpr int kAmrMaxR = 4;       // refinement factors 2..4
constexpr int kAmrMaxLevels = 6;  // levels 0..5
constexpr int8_t kAbsent = -2, kVMother = -1, kActive = 0, kVChild = 1;

// Basis tables of the AMR operators (fp64 copies of AmrTables).
struct AmrConsts {
  int r;
  double sub_avg[kAmrMaxR][4];      // [a][p]
  double at_sub[kAmrMaxR][4];       // [substep][p]
  double at_face[kAmrMaxR][2][4];   // [a][side][p]
  double at_nodes[kAmrMaxR][4][4];  // [a][node][p]
};

// Device clock of an AMR run: time, end time and the level steps of the
// current level-0 step (dt[l] = dt[l-1] / r).
struct AmrClock {
  double t;
  double t_end;
  double dt[kAmrMaxLevels];
  unsigned long long steps;
};

// int32 per coarse-fine face record (k_amr_cf_faces)
constexpr int kAmrCfRecord = 4;

// One level of the dense per-level representation.
struct AmrLevel {
  int n[3] = {1, 1, 1};  // cells per axis of the level's index space
  int64_t ncells = 0;    // n[0] n[1] n[2] (= ld of u)
  double dx[3] = {1, 1, 1};
  double* u = nullptr;        // [nv][ncells] cell averages
  int8_t* st = nullptr;       // [ncells] status
  int32_t* pos = nullptr;     // [ncells] position in the active list, -1 otherwise
  int32_t* act = nullptr;     // active cells (dense indices, ascending)
  int64_t nact = 0;
  int32_t* vc = nullptr;      // virtual children
  int64_t nvc = 0;
  int32_t* vm = nullptr;      // virtual mothers
  int64_t nvm = 0;
  double* mem = nullptr;      // [dim][2][nv][ncells] fine-coarse flux memory (level >= 1)
  double* wa = nullptr;       // WENO pass buffers of the active cells
  double* wb = nullptr;
  double* wh = nullptr;       // reconstruction w_h of the active cells
  double* dwx = nullptr;      // 3D: dense x- and y-pass lines [nv][n + n^2][ncells]
  void* qh = nullptr;         // predictor of the active cells (predictor precision)
  double* fbuf = nullptr;     // face fluxes of the active cells [cell][2 dim][nv]
  int32_t* cf = nullptr;      // coarse-fine face records of the active cells (k_amr_cf_faces)
  int32_t* fc = nullptr;      // kind of every face of the active cells (k_amr_cf_faces)
  int64_t ncf = 0;
  WsHeader* hdr = nullptr;    // status bits and Picard counters of the level
  MeshParams mp{};            // the level's mesh (n, dx, ld = ncells)
};

// Launch shapes of the tuned AMR kernels (ader_amr_tune): threads per block
// of the generic predictor and about-threads per block of the face-flux
// kernel, each 128, 256 or 512.
struct AmrShape {
  int pred_block = 256;
  int flux_block = 256;
};
constexpr int kAmrBlockChoices[3] = {128, 256, 512};

class AmrImplBase {
 public:
  virtual ~AmrImplBase() = default;
  virtual size_t qh_elem_size() const = 0;
  // WENO scratch doubles per active cell (two pass buffers) and w_h doubles
  virtual size_t weno_scratch_per_cell() const = 0;
  virtual size_t wh_per_cell() const = 0;
  // doubles per cell of the level's index space of the dense pass buffers
  virtual size_t dense_weno_per_cell() const = 0;
  // face-flux doubles per active cell
  virtual size_t fbuf_per_cell() const = 0;
  // block maxima of sum_k speed_k / dx_k over the active cells of levels
  // 0..nlev-1 -> partial[l kDtMaxBlocks + 0..nb[l]), one launch
  virtual hipError_t cfl(const AmrLevel* lv, int nlev, double* partial, const int* nb,
                         hipStream_t st) const = 0;
  // virtual mothers of 'coarse' from their children on 'fine'
  virtual hipError_t average(const AmrLevel& coarse, const AmrLevel& fine, int r,
                             hipStream_t st) const = 0;
  // one level substep's averaging (from 'fine'), projection (from 'coarse'
  // at substep 'sub') and the clearing of fine's memory at its virtual
  // children; coarse / fine may be null at the ends.  With apply_dt, the
  // same launch also applies the level's update of its previous substep
  // (deferred by update(..., apply = false)) with step *apply_dt.
  virtual hipError_t prepare(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                             const AmrConsts& ac, int sub, const double* apply_dt,
                             hipStream_t st) const = 0;
  // reconstruction + predictor of the active cells of 'lv' with step *dt
  virtual hipError_t predict(const AmrLevel& lv, const double* dt, const DevConsts& c,
                             const AmrShape& sh, hipStream_t st) const = 0;
  // whether the predictor of this configuration has a tunable block (the 2D
  // fp64 matrix-core predictor has a fixed layout), and whether a block size
  // fits (LDS)
  virtual bool pred_block_ok(int block) const = 0;
  // finite-volume update of the active cells of 'lv' (substep 'sub' of the
  // coarser level's step); coarse / fine may be null at the ends.  With
  // apply false only the face fluxes are computed, and the update is left
  // to the level's next prepare (its apply_dt) or to the coarser level's
  // update (its pend).  pend (or null): a finer level whose deferred update,
  // with step *pend_dt, rides in this update's face launch
  virtual hipError_t update(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                            const double* dt, int sub, const DevConsts& c, const AmrConsts& ac,
                            const AmrShape& sh, bool apply, const AmrLevel* pend,
                            const double* pend_dt, hipStream_t st) const = 0;
  // the list of the level's coarse-fine faces into lv.cf; *count (device)
  // must be zero on entry and holds the count on exit
  virtual hipError_t cf_faces(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                              const AmrConsts& ac, int* count, hipStream_t st) const = 0;
  // the face-flux kernel alone (for tuning; its fluxes go to the scratch)
  virtual hipError_t flux_only(const AmrLevel& lv, const AmrLevel* coarse, const AmrLevel* fine,
                               const double* dt, int sub, const DevConsts& c,
                               const AmrConsts& ac, int flux_block, hipStream_t st) const = 0;
  // regrid: reconstruction of the listed cells 'moth' (nm of them) of
  // 'coarse' into wh (scratch wa, wb as for predict), then targets[i] of
  // 'fine' = sub-cell average of w_h of slot tslot[i]
  virtual hipError_t children(const AmrLevel& coarse, const int32_t* moth, int64_t nm,
                              double* wa, double* wb, double* wh, const AmrLevel& fine,
                              const int32_t* targets, const int32_t* tslot, int64_t nt,
                              const DevConsts& c, const AmrConsts& ac, hipStream_t st) const = 0;
};

const AmrImplBase* make_amr_impl_2d(int M, int system, int precision);
const AmrImplBase* make_amr_impl_3d(int M, int system, int precision);

// CFL step of the AMR run (one block): dt0 = min over levels with active
// cells of r^l cfl / max_l, clipped to t_end - t; dt[l] = dt[l-1] / r;
// t += dt0.  partial holds kDtMaxBlocks maxima per level, nb[l] of them used.
struct AmrDtArgs {
  int nlev;
  int r;
  double cfl;
  int nb[kAmrMaxLevels];
};
hipError_t launch_amr_dt(const double* partial, AmrDtArgs a, AmrClock* clock, WsHeader* hdr,
                         hipStream_t st);
// u[v * ld + list[i]] = value for every variable v < nv and i < n
hipError_t launch_fill_list(double* u, int64_t ld, int nv, const int32_t* list, int64_t n,
                            double value, hipStream_t st);

// ----- device-side mesh change (amr_regrid.hip) -----
struct RgGrid {
  int dim;
  int n[3];   // cells per axis of the level
  int bc[3];  // boundary kinds per axis
  int64_t N;  // n0 n1 n2
};
enum { kSelActive = 0, kSelVChild = 1, kSelVMother = 2, kSelMothers = 3, kSelBorn = 4 };

// F = refine / keep flags from the Loehner indicator of phi (see k_rg_lohner)
hipError_t rg_lohner(const RgGrid& g, const double* phi, const int8_t* st, double eps,
                     double chi_ref, double chi_rec, uint8_t* F, hipStream_t s);
// out = Voronoi neighbourhood of the flagged cells of in
hipError_t rg_dilate(const RgGrid& g, const uint8_t* in, uint8_t* out, hipStream_t s);
// Fc |= some child flagged in Ff
hipError_t rg_mothers_or(const RgGrid& fine, const RgGrid& coarse, int r, const uint8_t* Ff,
                         uint8_t* Fc, hipStream_t s);
// Ff &= Fc[mother]
hipError_t rg_nest(const RgGrid& fine, const RgGrid& coarse, int r, const uint8_t* Fc,
                   uint8_t* Ff, hipStream_t s);
// status of a level >= 1 from the coarser level's flags and near flags
hipError_t rg_status(const RgGrid& fine, const RgGrid& coarse, int r, const uint8_t* Fc,
                     const uint8_t* near_c, const uint8_t* Ff, int8_t* st, hipStream_t s);
hipError_t rg_status0(int64_t N, const uint8_t* F0, int8_t* st, hipStream_t s);
// *changed |= 1 where a and b differ
hipError_t rg_diff(int64_t N, const int8_t* a, const int8_t* b, unsigned int* changed,
                   hipStream_t s);
// NaN in every variable of the cells absent in st_new and not in st_old
hipError_t rg_gone(int64_t N, int nv, double* u, const int8_t* st_new, const int8_t* st_old,
                   hipStream_t s);
// pos = -1, then pos[list[j]] = j
hipError_t rg_positions(int32_t* pos, int64_t N, const int32_t* list, int64_t n, hipStream_t s);
// tslot[i] = slot_c[mother of targets[i]]
hipError_t rg_slots(const RgGrid& fine, const RgGrid& coarse, int r, const int32_t* targets,
                    int64_t nt, const int32_t* slot_c, int32_t* tslot, hipStream_t s);
// ascending dense indices i with the selection 'mode' (kSel*) into out,
// their number into *d_count (device); temp == nullptr queries *temp_bytes
hipError_t rg_select(int mode, const int8_t* st, const int8_t* old, int64_t N, int32_t* out,
                     int* d_count, void* temp, size_t* temp_bytes, hipStream_t s);

}  // namespace ader
