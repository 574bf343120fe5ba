/*
 * ader.h -- C ABI of the MI355X (gfx950) one-step ADER-WENO hot path.
 *
 * The library advances the cell averages of a hyperbolic conservation law
 *     u_t + f(u)_x + g(u)_y + h(u)_z = 0                 (Section 2.1, S = 0)
 * on a uniform Cartesian mesh by one step of the one-step ADER-WENO finite
 * volume scheme (Section 2): dimension-by-dimension polynomial WENO
 * reconstruction (Section 2.2), element-local space-time DG predictor solved
 * by Picard iteration (Section 2.3, eq. stdg.final), Rusanov fluxes at the
 * space-time Gauss-Legendre points of every face (eqs. flux:F-H, rusanov; or
 * the Osher-type flux of eq. osher) and
 * the conservative update (eq. finite_vol).
 *
 * Conventions shared by every call:
 *   - Every function returns ader_status: ADER_OK (0) or a negative code.
 *     Argument errors are detected on the host and returned synchronously;
 *     nothing is launched in that case.  ader_last_error() returns a message
 *     for the most recent failure of the calling thread.
 *   - Numerical faults found on the device (NaN, non-positive density or
 *     pressure, predictor iteration not converged) set bits in a status word
 *     inside the workspace; ader_read_status() fetches it.
 *   - State arrays are structure-of-arrays in device memory, fp64:
 *         u[v * ld + cell],  cell = i + nx * (j + ny * k)   (x fastest),
 *     v = 0..nvar-1, ld >= number of cells.  The caller owns all device
 *     buffers (inputs, outputs, workspace); the plan owns only host memory.
 *   - 'stream' is a hipStream_t passed as void* (NULL = the null stream).
 *     Every compute call is asynchronous on that stream and never
 *     synchronises, allocates or frees device memory.
 *   - The time step lives in device memory (dt_dev, one double) so that a
 *     sequence of steps needs no host round trip.
 *   - Calls that share one workspace must be ordered (same stream or
 *     synchronised); two concurrent calls on one workspace race.
 */
#ifndef ADER_H
#define ADER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADER_OK = 0,
  ADER_EINVAL = -1,        /* invalid argument (null pointer, bad size ...) */
  ADER_EUNSUPPORTED = -2,  /* valid problem outside what the library supports */
  ADER_EHIP = -3,          /* a HIP runtime call failed */
  ADER_EWORKSPACE = -4     /* workspace pointer null or misaligned */
} ader_status;

/* Balance law: scalar linear advection with constant velocity adv[]; the
 * Euler equations of an ideal gas (Section 4.1, eq. Euler-system) with
 * conserved variables (rho, rho v_x, rho v_y, [rho v_z,] E): nvar = dim + 2;
 * or ideal MHD with hyperbolic GLM divergence cleaning (Section 4.2) with
 * (rho, rho v_x, rho v_y, rho v_z, E, B_x, B_y, B_z, psi): nvar = 9 in 2D and
 * 3D, magnetic terms in the paper's units (|B|^2 / 8 pi, B B / 4 pi), cleaning
 * speed ch; Rusanov and CFL use max(|v_n| + c_f, ch) with the fast
 * magnetosonic speed c_f. */
typedef enum { ADER_SYS_LINADV = 0, ADER_SYS_EULER = 1, ADER_SYS_MHD_GLM = 2 } ader_system;

/* FP64: every stage in double precision.  FP32_PREDICTOR: the Picard
 * iteration of the predictor and its face traces in single precision with
 * single-precision accumulation; reconstruction (smoothness indicators and
 * nonlinear weights), Rusanov flux, flux quadrature and update stay fp64. */
typedef enum { ADER_PREC_FP64 = 0, ADER_PREC_FP32_PREDICTOR = 1 } ader_precision;

/* Numerical flux at the space-time Gauss points of a face: Rusanov (eq.
 * rusanov, local Lax-Friedrichs) or the Osher-type flux (eq. osher): the
 * path integral of |A| = R |Lambda| R^-1 of the flux Jacobian along the
 * straight segment between the two traces by 3-point Gauss-Legendre
 * quadrature, with the analytic Euler eigenvectors.  Osher is available
 * for the Euler equations; for linear advection both fluxes are the upwind
 * flux; GLM-MHD takes Rusanov only (EUNSUPPORTED otherwise). */
typedef enum { ADER_FLUX_RUSANOV = 0, ADER_FLUX_OSHER = 1 } ader_flux;

/* Periodic, or transmissive: zero-gradient ghost averages for the WENO
 * stencils and, on a boundary face, outer predictor trace = inner trace. */
typedef enum { ADER_BC_PERIODIC = 0, ADER_BC_TRANSMISSIVE = 1 } ader_bc;

typedef struct {
  int dim;            /* 2 or 3 */
  int M;              /* polynomial degree 0..3 (order of accuracy M+1) */
  int system;         /* ader_system */
  double gamma;       /* ratio of specific heats (Euler, MHD) */
  double ch;          /* GLM divergence-cleaning speed (MHD), > 0 */
  double adv[3];      /* advection velocity (linear advection) */
  int n[3];           /* cells per axis (n[2] ignored for dim 2); each >= 1 */
  double lo[3];       /* domain lower corner */
  double hi[3];       /* domain upper corner */
  int bc[3];          /* ader_bc per axis (both sides of an axis alike) */
  double cfl;         /* Courant number of the time-step rule, in (0, 1] */
  int flux;           /* ader_flux */
  int precision;      /* ader_precision */
  double picard_tol;  /* relative stop tolerance of the predictor iteration */
  int picard_max;     /* iteration cap (1..1000); reaching it sets a flag */
} ader_problem;

typedef struct ader_plan_s* ader_plan;

/* Device status bits (ader_read_status). */
#define ADER_FLAG_NAN 1u          /* a NaN appeared in the new averages or dt */
#define ADER_FLAG_NONPHYSICAL 2u  /* rho <= 0 or p <= 0 (gas pressure) in the new averages */
#define ADER_FLAG_NOCONV 4u       /* predictor reached picard_max */
#define ADER_FLAG_BADINDEX 8u     /* a level view held an index out of range */

/* Validate the problem and build the reference-element constants (Gauss-
 * Legendre nodes and weights, Lagrange basis values and derivatives,
 * per-stencil inverse reconstruction matrices, oscillation matrix, and the
 * time matrix of K^1 with its inverse; Sections 2.2 and 2.3) on the host.
 * *out receives a plan owned by the caller; release with ader_plan_destroy.
 * Errors: EINVAL (null pointers, non-finite or out-of-range fields),
 * EUNSUPPORTED (dim/M/system outside what the library supports). */
ader_status ader_plan_create(const ader_problem* prob, ader_plan* out);

/* Release a plan (NULL is accepted). */
ader_status ader_plan_destroy(ader_plan plan);

/* Number of conserved variables of the plan's system (1; 4 or 5; 9). */
ader_status ader_plan_nvar(ader_plan plan, int* nvar);

/* Bytes of device workspace every compute call of this plan needs.  The
 * workspace is caller-allocated device memory, 256-byte aligned, reusable
 * across calls of the same plan; its status word survives between calls. */
ader_status ader_workspace_bytes(ader_plan plan, size_t* bytes);

/* Zero the workspace's status word and iteration counters (a fill kernel on
 * 'stream', no hipMemset). */
ader_status ader_clear_status(ader_plan plan, void* ws, void* stream);

/* Time step from the CFL rule on the averages u at time t:
 *   dt = cfl / max_cells sum_k (|v_k| + c) / dx_k     (|a_k| for advection,
 *   max(|v_k| + c_f, ch) for MHD),
 * then dt = min(dt, t_end - t).  Written to dt_dev (one device double).
 * The paper states no formula for dt; this is the rule the library uses. */
ader_status ader_compute_dt(ader_plan plan, const double* u, int64_t ld,
                            double t, double t_end, double* dt_dev, void* ws,
                            void* stream);

/* One step of the scheme on every cell: u_out = u_in advanced by *dt_dev
 * (eq. finite_vol with the fluxes of eqs. flux:F-H).  u_in and u_out are
 * distinct nvar x ld device arrays (EINVAL if they overlap). */
ader_status ader_step(ader_plan plan, const double* u_in, double* u_out,
                      int64_t ld, const double* dt_dev, void* ws, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ader_step
 * with its workspace taken from a device array inside the library instead of
 * a caller-allocated one.  The array holds ADER_STATIC_SCRATCH_BYTES; each GPU
 * the library runs on holds its own copy until the process ends.  Same
 * arguments, layouts and results as ader_step (the same kernels, bit for
 * bit), minus 'ws':
 *   status  NULL, or caller-owned device memory for two uint32 written at the
 *           end of the call: [0] the status bits of this call (ADER_FLAG_*),
 *           [1] its Picard sweeps summed over the cells (saturated at
 *           2^32 - 1).  Each call starts from a zero status.
 * The call makes no hipMalloc, hipFree or other allocating call; its first
 * call on a device looks the array up there (hipGetSymbolAddress).
 * Errors: as ader_step; EWORKSPACE (before any launch) when the plan's step
 * needs more than ADER_STATIC_SCRATCH_BYTES (2D Euler, M = 3, fp64: 2 KiB per
 * cell, so up to about 32,000 cells; ader_workspace_bytes gives the whole
 * workspace, of which the step uses the leading part).
 * All calls on one GPU share that GPU's array and it keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
#define ADER_STATIC_SCRATCH_BYTES (64ull << 20)
ader_status ader_step_static(ader_plan plan, const double* u_in, double* u_out,
                             int64_t ld, const double* dt_dev, uint32_t* status,
                             void* stream);

/* Stage entry points (for stage-by-stage checks):
 *
 * ader_debug_reconstruct: WENO polynomial of every cell (Section 2.2),
 *   w_h[(cell * nvar + v) * n^d + a], a = p_x + n p_y (+ n^2 p_z), n = M+1:
 *   nodal values at the tensor Gauss-Legendre nodes of the reference cell.
 *
 * ader_debug_predict: space-time predictor (Section 2.3) of 'ncells'
 *   independent cells from their nodal reconstructions w_h (layout above),
 *   q_h[(cell * nvar + v) * n^(d+1) + a + n^d s] (s = time node), with
 *   dt/dx_k of the plan's mesh and *dt_dev.  ncells is free (not tied to the
 *   mesh); the workspace must still be the plan's. */
ader_status ader_debug_reconstruct(ader_plan plan, const double* u, int64_t ld,
                                   double* w_h, void* ws, void* stream);
ader_status ader_debug_predict(ader_plan plan, const double* w_h,
                               int64_t ncells, double* q_h,
                               const double* dt_dev, void* ws, void* stream);

/* ader_debug_traces (2D plans; EUNSUPPORTED for 3D): the fused 2D cell kernel
 *   of ader_step alone, at the plan's tile height, on the averages u with
 *   *dt_dev: reconstruction (Section 2.2), predictor (Section 2.3, eq.
 *   stdg.final, in the plan's precision) and the predictor's values on the
 *   four faces of every cell at the face's space-time Gauss points (the
 *   operands of eqs. flux:F and flux:G), written as fp64 to
 *     traces[((f * ncells + cell) * nvar + v) * n * n + s * n + b],
 *   f = 0 x-low, 1 x-high, 2 y-low, 3 y-high face, s the time node, b the
 *   transverse node; 4 ncells nvar n^2 doubles, caller-owned device memory.
 *   The averages are not updated.  The workspace's status bits and counters
 *   accumulate as in ader_step. */
ader_status ader_debug_traces(ader_plan plan, const double* u, int64_t ld,
                              const double* dt_dev, double* traces, void* ws,
                              void* stream);

/* Autotuning of the fused 2D cell kernel (2D plans; EUNSUPPORTED for 3D).
 * The cell kernel works on tiles of 4 x rows cells, one wavefront per tile
 * row; rows is 2, 4, 8 or 16 (at most 8 for GLM-MHD, whose kernel needs more
 * registers).  Results do not depend on the height: every wavefront holds one
 * tile row whatever the height, so the arithmetic per cell is the same.
 *   ader_tune       times one untimed and 'reps' (1..1000) timed launches of
 *                   the cell kernel per candidate height on the caller's
 *                   state u (read only) with *dt_dev, on 'stream'.  It keeps
 *                   the fastest height in the plan, writes it to *rows (may be
 *                   NULL), and writes the mean ms of each of the four heights
 *                   to ms_out[4] (may be NULL; -1 for a height that is not a
 *                   candidate).  The workspace's traces are overwritten and
 *                   its status bits and counters cleared.  Synchronous.
 *   ader_set_tile_rows  forces a height (0 = the default, 8). */
ader_status ader_tune(ader_plan plan, const double* u, int64_t ld, const double* dt_dev,
                      void* ws, void* stream, int reps, int* rows, double* ms_out);
ader_status ader_set_tile_rows(ader_plan plan, int rows);

/* One step over the cell lists of one refinement level (or any subset of a
 * uniform mesh).  On a cell-by-cell AMR mesh the predictor is element-local
 * and identical to the uniform one; the reconstruction of every cell reads a
 * layer of at least M same-level cells, real or virtual (Section 3), which
 * the caller names explicitly:
 *   level       refinement level (informational)
 *   dx          mesh widths of the level
 *   npred       cells whose predictor is computed: the cells updated and the
 *               face neighbours their fluxes need
 *   pred_cells  [npred] state index of each of them
 *   pred_patch  [npred * (2M+1)^d] state indices of the (2M+1)^d cells around
 *               each (offsets -M..M per axis, x fastest); virtual and ghost
 *               cells are ordinary entries of the state arrays
 *   nupd        cells updated
 *   upd         [nupd] positions (0..npred-1) in pred_cells of those cells
 *   upd_nbr     [nupd * 2d] positions in pred_cells of their face neighbours,
 *               order x-low, x-high, y-low, y-high[, z-low, z-high]; -1 marks
 *               an outflow face (outer trace = inner trace)
 * u_out receives the new averages of the updated cells only; u_in and u_out
 * must not overlap.  All arrays are device memory.  The plan's M, dim,
 * system, precision and Picard settings apply; its mesh sizes do not.  The
 * workspace is ader_level_workspace_bytes(plan, npred) bytes.  Indices out
 * of range are not dereferenced: they set ADER_FLAG_BADINDEX (an outflow
 * face for a bad neighbour, no update for a bad cell). */
typedef struct {
  int level;
  double dx[3];
  int64_t npred;
  const int32_t* pred_cells;
  const int32_t* pred_patch;
  int64_t nupd;
  const int32_t* upd;
  const int32_t* upd_nbr;
} ader_level_view;

ader_status ader_level_workspace_bytes(ader_plan plan, int64_t npred, size_t* bytes);
ader_status ader_step_level(ader_plan plan, const ader_level_view* view,
                            const double* u_in, double* u_out, int64_t ld,
                            const double* dt_dev, void* ws, void* stream);

/* Synchronise 'stream' and read the status bits (ADER_FLAG_*) and the sum of
 * predictor iterations over all cells since the last clear. */
ader_status ader_read_status(ader_plan plan, const void* ws, uint32_t* flags,
                             uint64_t* picard_iterations, void* stream);

/* Reference-element constants as the device path uses them, for checks:
 * nodes[n], weights[n], dmat[n*n] (dmat[a*n+b] = psi_b'(node_a)),
 * time_inv_w[n*n] = (time matrix of K^1)^-1 diag(weights). */
ader_status ader_debug_constants(ader_plan plan, double* nodes, double* weights,
                                 double* dmat, double* time_inv_w);

/* Stage timing with HIP events recorded on the launch stream.
 * ader_profile_begin: from now on every compute call of this plan brackets
 *   each stage (ADER_STAGE_*) with a pair of events on its stream.
 * ader_profile_end: synchronise those events, write the summed milliseconds
 *   and launch counts per stage (arrays of ADER_NSTAGES), stop recording.
 * Host-side events only; device memory is untouched. */
#define ADER_STAGE_DT 0
#define ADER_STAGE_WENO 1
#define ADER_STAGE_PREDICT 2
#define ADER_STAGE_FLUX 3
#define ADER_STAGE_UPDATE 4
#define ADER_NSTAGES 5
ader_status ader_profile_begin(ader_plan plan);
ader_status ader_profile_end(ader_plan plan, double* stage_ms, int64_t* stage_launches);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching of independent 2D solves.
 *
 * A server keeps many independent solves (problem + initial averages + end
 * time, each advanced with the CFL step of ader_compute_dt until t_end, as
 * ader_step does) resident on one GPU and advances them together.
 *   - Admission by HBM footprint: the server owns one device arena of
 *     hbm_bytes; a submitted solve waits in a FIFO queue until a slot and
 *     arena space for its two state buffers and its workspace are free
 *     (ader_server_footprint gives the bytes).  It is then uploaded and joins
 *     the next round of its kernel group.
 *   - Rounds: all resident solves with the same (M, system, precision) form a
 *     group; one round advances every solve of the group by one step with
 *     three launches whose grids cover all of them (CFL step, cell kernel,
 *     face kernel).  Each solve's time lives on the device: a round computes
 *     its dt = min(CFL / max, t_end - t) and t += dt, and a solve that has
 *     reached t_end costs nothing further.  Groups are spread over the
 *     server's streams (default priority) and overlap on the device.
 *   - The host reads a small table of solve clocks after each round (pinned
 *     memory, asynchronous) to retire finished solves: their averages are
 *     copied to the caller's output buffer and their slot and memory freed.
 * The per-solve arithmetic is that of ader_step: a result is bitwise the
 * same whichever other solves share its rounds.
 *
 * Threading: a server is driven from one host thread.  u0 and u_out are host
 * arrays [nvar][cells] (x fastest); u0 is copied at submit, u_out must stay
 * valid until the request is done.  Only dim = 2 problems are served. */
typedef struct ader_server_s* ader_server;

typedef struct {
  size_t hbm_bytes;  /* device arena for resident solves (>= 1 MiB) */
  int max_slots;     /* solves resident at once, 1..4096 */
  int streams;       /* HIP streams the groups are spread over, 1..16 */
  int rounds_ahead;  /* rounds a group may have in flight, 1..8 */
} ader_server_config;

typedef struct {
  int state;                   /* 0 queued, 1 resident, 2 done, 3 failed */
  uint32_t flags;              /* ADER_FLAG_* of the solve (when done) */
  uint64_t steps;              /* steps taken */
  uint64_t picard_iterations;  /* predictor iterations summed over cells and steps */
  double t;                    /* time reached */
  double submit_s, admit_s, done_s;  /* host monotonic clock, seconds */
} ader_request_info;

typedef struct {
  size_t arena_bytes, bytes_in_use, peak_bytes_in_use;
  int resident, peak_resident, queued;
  int64_t rounds, launches, completed;
} ader_server_stats;

ader_status ader_server_create(const ader_server_config* config, ader_server* out);
/* Waits for the device work of the server, then frees everything it owns.
 * Requests not done by then stay not done. */
ader_status ader_server_destroy(ader_server server);
/* Device bytes a problem occupies while resident. */
ader_status ader_server_footprint(const ader_problem* prob, size_t* bytes);
/* Queue one solve: EINVAL / EUNSUPPORTED for a bad problem, t_end <= 0 or
 * non-finite, or a footprint above the arena (it could never be admitted). */
ader_status ader_server_submit(ader_server server, const ader_problem* prob,
                               const double* u0, double t_end, double* u_out,
                               int64_t* id);
/* One scheduling pass: retire finished solves, admit queued ones, launch the
 * next round of every group with room.  wait != 0 blocks until at least one
 * in-flight round or retirement completes (if there is any). */
ader_status ader_server_progress(ader_server server, int wait, int* resident, int* queued);
ader_status ader_server_request(ader_server server, int64_t id, ader_request_info* info);
ader_status ader_server_stats_get(ader_server server, ader_server_stats* stats);

/* ------------------------------------------------------------------------
 * Cell-by-cell AMR with time-accurate local time stepping (Section 3).
 *
 * Mesh: level 0 is the problem's uniform mesh; level l refines it by r^l per
 * axis (eq. refine-factor, max(M, 2) <= r <= 4, levels 0..max_level <= 5).
 * Every level is held on the device as a dense array over its whole index
 * space ([nvar][cells], x fastest, the layout of ader_step) with a status per
 * cell: active (updated by the scheme), virtual child (projection of the
 * mother's space-time predictor, Section 3.1.3), virtual mother (average of
 * its children, eq. average) or absent.  Children of a cell are the r^d
 * consecutive-index blocks i*r + a; the mother of i is i / r.
 *
 * ader_amr_build constructs the mesh once from the initial averages of
 * every level: the Loehner indicator (eq. indicator, index units; filter
 * eps (|P+| + 2|P| + |P-|) on the diagonal pairs, the mean of the four
 * diagonal neighbours on the cross pairs) of variable indicator_var above
 * chi_ref flags cells of levels 0..max_level-1, plus 'buffer' layers of
 * their Voronoi neighbours (ader_amr_set_flags replaces the indicator for a
 * level; such flags are taken as given).  Flags are closed so that Voronoi neighbours differ by at
 * most one level and a refined cell's Voronoi neighbours exist on the finer
 * level; children of flagged cells are active, children of their active
 * Voronoi neighbours are virtual.  EINVAL if an active cell's (2M+1)^d
 * stencil would leave the mesh.
 *
 * ader_amr_regrid refines and recoarsens between steps (Section 3.1, rules
 * 1-7; thresholds of Section 3.1.1).  All levels are at one time after a
 * step.  Virtual mothers are averaged, then virtual children take the
 * average of their mother's reconstruction (Section 2.2) over their
 * sub-cell, coarse to fine.  The indicator then flags active cells with
 * chi > chi_ref and keeps virtual mothers with chi >= chi_rec.  Flags set by
 * ader_amr_set_flags after the build replace the indicator for one regrid.
 * Buffer layers, closure and status follow the build.  Cells that did not
 * exist take the sub-cell averages of their mother's reconstruction, coarse
 * to fine.  Recoarsened cells keep the average of their children (eq.
 * average), so a regrid is conservative.  Removed cells become NaN.
 * Synchronous; *changed (may be NULL) is 1 when the mesh changed.  A
 * recorded step graph is recorded again at the next ader_amr_step.
 *
 * ader_amr_step: one level-0 step, Delta t_0 = min over levels of
 * r^l CFL / max over active cells of sum_k speed_k / dx_(l,k), clipped to
 * t_end (an empty step once t_end is reached); level l takes r^l substeps of
 * Delta t_0 / r^l, finest first (Section 3.1.2): averaging, projection,
 * reconstruction and predictor, the finer level's substeps, then the update.
 * A face between a fine active cell and a coarser active cell takes the
 * coarse predictor at the fine face's space-time Gauss points; the fine
 * fluxes are kept in memory variables and their average is the coarse
 * cell's flux (eq. memory.sum): the scheme is conservative.  Time, end time
 * and level steps live on the device; use_graph records one step as a HIP
 * graph once and replays it.  Asynchronous on 'stream' (NULL: the object's
 * own stream); ader_amr_clock synchronises and reads the time.
 *
 * The object owns its device memory (allocated by ader_amr_build). */
typedef struct ader_amr_s* ader_amr;

typedef struct {
  int r;              /* refinement factor */
  int max_level;      /* finest level L */
  int indicator_var;  /* conserved variable fed to the indicator */
  double chi_ref;     /* refine where chi > chi_ref */
  double chi_rec;     /* regrid: a refined cell is recoarsened where chi < chi_rec
                         (chi_rec <= chi_ref; equal values: no hysteresis) */
  double eps;         /* indicator filter (0.01 in the paper) */
  int buffer;         /* Voronoi layers added around indicator flags (0..4) */
  int use_graph;      /* replay one recorded step per ader_amr_step */
} ader_amr_config;

ader_status ader_amr_create(const ader_problem* prob, const ader_amr_config* config,
                            ader_amr* out);
ader_status ader_amr_destroy(ader_amr amr);
/* Dense cells per axis of a level. */
ader_status ader_amr_level_cells(ader_amr amr, int level, int n[3]);
/* Initial averages of a level's whole index space (host, [nvar][cells]). */
ader_status ader_amr_set_level(ader_amr amr, int level, const double* u);
/* Refinement flags of a level < max_level (host, [cells], nonzero = refine),
 * taken as given by the next ader_amr_build or ader_amr_regrid. */
ader_status ader_amr_set_flags(ader_amr amr, int level, const uint8_t* flags);
ader_status ader_amr_build(ader_amr amr);
ader_status ader_amr_regrid(ader_amr amr, int* changed);
ader_status ader_amr_step(ader_amr amr, double t_end, void* stream);
/* Autotuning of the AMR kernels' launch shapes, after at least one step
 * (the level steps must be set).  On the level with the most active cells,
 * it times one untimed and 'reps' (1..1000) timed launches of each candidate.
 * Candidates: the predictor's block of 128, 256 or 512 threads (cells of
 * (M+1)^d lanes each; only sizes whose LDS fits; the 2D fp64 matrix-core
 * predictor has its one layout) and the face-flux kernel's block of about
 * 128, 256 or 512 threads.  It keeps the fastest of each, writes them to
 * *pred_block and *flux_block (may be NULL), and writes the mean ms of the
 * six candidates to ms_out[6] (predictor 128/256/512, then flux; -1 where
 * not a candidate; may be NULL).  Results do not depend on the shapes.  The
 * level's scratch is overwritten; the averages, the clock and the
 * statistics are kept.  Synchronous; the step graph is recorded again. */
ader_status ader_amr_tune(ader_amr amr, int reps, int* pred_block, int* flux_block,
                          double* ms_out);
ader_status ader_amr_clock(ader_amr amr, double* t, int64_t* steps, double* dt0);
/* Level averages (host [nvar][cells]; absent cells NaN) and status (host
 * [cells]: -2 absent, -1 virtual mother, 0 active, 1 virtual child). */
ader_status ader_amr_get_level(ader_amr amr, int level, double* u, int8_t* status);
/* counts[0..2] = active, virtual children, virtual mothers of a level. */
ader_status ader_amr_counts(ader_amr amr, int level, int64_t counts[3]);
/* Status bits, predictor iterations and cell updates (active cells times
 * substeps) since the mesh was built. */
ader_status ader_amr_stats(ader_amr amr, uint32_t* flags, uint64_t* picard_iterations,
                           uint64_t* cell_updates);

const char* ader_status_string(ader_status status);
const char* ader_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADER_H */
