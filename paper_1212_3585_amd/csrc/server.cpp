// Solve server: continuous batching of independent 2D solves on one GPU.
//
// Host side of the server declared in ader.h.  Resources:
//   - one device arena (first-fit, coalescing free list) holding, per
//     resident solve, its two state buffers and its workspace (status
//     header, CFL block maxima, face traces);
//   - a device array of per-slot clocks (SolveClock) and, per kernel group,
//     rings of round tables and clock mirrors (rounds_ahead + 1 entries,
//     device + pinned host), so a ring entry is rewritten only after the
//     round that last used it has completed;
//   - one pinned host buffer per request: the initial averages until upload,
//     then the result and the final status header.
// Scheduling pass (ader_server_progress): harvest completed rounds (their
// clock mirrors name the solves that reached t_end; those are retired with
// an asynchronous copy of their final state), finish completed retirements
// (copy to the caller's array, free slot and memory), admit queued requests
// in FIFO order while slot and arena space allow, then launch one more round
// for every group with fewer than rounds_ahead rounds in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "plan.hpp"
#include "server.hpp"

using ader::fail;
using ader::hip_status;
using ader::SolveClock;
using ader::SolveDesc;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator of byte ranges of [0, size).
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

// Pinned host buffers, reused by size.
class PinnedPool {
 public:
  ~PinnedPool() {
    for (auto& kv : size_) (void)hipHostFree(kv.first);
  }
  void* get(size_t bytes) {
    auto it = free_.lower_bound(bytes);
    if (it != free_.end() && it->first <= 2 * bytes + 65536) {
      void* p = it->second;
      free_.erase(it);
      return p;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    size_[p] = bytes;
    return p;
  }
  void put(void* p) {
    if (p) free_.emplace(size_[p], p);
  }

 private:
  std::multimap<size_t, void*> free_;
  std::unordered_map<void*, size_t> size_;
};

// Sizes of one resident solve.
struct Footprint {
  int nv = 0, n = 0;
  int64_t ncells = 0, ld = 0;
  size_t off_u1 = 0, off_hdr = 0, off_partial = 0, off_traces = 0, bytes = 0;
};

Footprint footprint(const ader_problem& pr, int64_t ncells, size_t trace_elem) {
  Footprint f;
  f.nv = pr.system == ADER_SYS_LINADV ? 1 : (pr.system == ADER_SYS_EULER ? pr.dim + 2 : 9);
  f.n = pr.M + 1;
  f.ncells = ncells;
  f.ld = (ncells + 31) / 32 * 32;  // every variable row 256-byte aligned
  const size_t state = align256(sizeof(double) * f.nv * (size_t)f.ld);
  f.off_u1 = state;
  f.off_hdr = 2 * state;
  f.off_partial = f.off_hdr + ader::kHeaderBytes;
  f.off_traces = align256(f.off_partial + sizeof(double) * ader::kDtMaxBlocks);
  f.bytes = align256(f.off_traces + trace_elem * 4 * (size_t)f.nv * f.n * f.n * (size_t)ncells);
  return f;
}

constexpr int kQueued = 0, kResident = 1, kDone = 2, kFailed = 3;

struct Request {
  int64_t id = 0;
  ader_problem prob{};
  Footprint fp;
  double t_end = 0.0;
  double* u_out = nullptr;
  int state = kQueued;
  double submit_s = 0.0, admit_s = 0.0, done_s = 0.0;
  int group = -1;
  int slot = -1;
  size_t off = 0;
  void* pinned = nullptr;  // [nv][ncells] averages, then the WsHeader
  hipEvent_t done_ev = nullptr;
  bool retiring = false;
  SolveDesc desc{};  // block offsets are filled per table
  long long dt_blocks = 0, cell_blocks = 0, face_blocks = 0;
  uint32_t flags = 0;
  uint64_t steps = 0, iters = 0;
  double t = 0.0;
};

struct InFlight {
  hipEvent_t ev;
  int mirror;
  std::vector<Request*> reqs;
};

struct Group {
  int M = 0, system = 0, precision = 0;
  const ader::BatchImplBase* impl = nullptr;
  ader::DevConsts dc{};
  hipStream_t stream = nullptr;
  std::vector<Request*> table;  // resident solves that still step
  bool dirty = true;
  int table_slot = 0;
  long long dt_blocks = 0, cell_blocks = 0, face_blocks = 0;
  int ns = 0;
  int64_t rounds = 0;
  std::vector<SolveDesc*> h_tab, d_tab;   // rings (rounds_ahead + 1)
  std::vector<SolveClock*> h_mir, d_mir;  // rings (rounds_ahead + 1)
  std::deque<InFlight> inflight;
};

}  // namespace

struct ader_server_s {
  ader_server_config cfg{};
  char* arena_base = nullptr;
  std::unique_ptr<Arena> arena;
  SolveClock* d_clocks = nullptr;
  SolveClock* h_clock_init = nullptr;  // pinned, one per slot
  void* h_zero = nullptr;              // pinned zeros (a workspace header)
  std::vector<hipStream_t> streams;
  std::vector<int> free_slots;
  std::map<int, std::unique_ptr<Group>> groups;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request*> queue;
  std::vector<Request*> retiring;
  std::vector<hipEvent_t> event_pool;
  PinnedPool pinned;
  int64_t next_id = 1;
  size_t in_use = 0, peak_in_use = 0;
  int resident = 0, peak_resident = 0;
  int64_t rounds = 0, launches = 0, completed = 0;

  hipError_t event(hipEvent_t* e) {
    if (!event_pool.empty()) {
      *e = event_pool.back();
      event_pool.pop_back();
      return hipSuccess;
    }
    return hipEventCreateWithFlags(e, hipEventDisableTiming);
  }
  void release_event(hipEvent_t e) { event_pool.push_back(e); }
};

namespace {

int group_key(const ader_problem& p) { return (p.M * 8 + p.system) * 2 + p.precision; }

ader_status get_group(ader_server s, const ader_problem& p, Group** out) {
  const int key = group_key(p);
  auto it = s->groups.find(key);
  if (it != s->groups.end()) {
    *out = it->second.get();
    return ADER_OK;
  }
  auto g = std::make_unique<Group>();
  g->M = p.M;
  g->system = p.system;
  g->precision = p.precision;
  g->impl = ader::make_batch_impl_2d(p.M, p.system, p.precision);
  if (!g->impl) return fail(ADER_EUNSUPPORTED, "no batched kernels for this configuration");
  ader::RefConstants ref;
  if (!ader::build_ref_constants(p.M, &ref)) return fail(ADER_EINVAL, "singular reference matrix");
  ader::fill_dev_consts(ref, p.M, &g->dc);
  g->stream = s->streams[s->groups.size() % s->streams.size()];
  const int ring = s->cfg.rounds_ahead + 1;
  const size_t tab = sizeof(SolveDesc) * s->cfg.max_slots;
  const size_t mir = sizeof(SolveClock) * s->cfg.max_slots;
  for (int r = 0; r < ring; ++r) {
    void *ht = nullptr, *dt = nullptr, *hm = nullptr, *dm = nullptr;
    if (hipHostMalloc(&ht, tab, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&dt, tab) != hipSuccess ||
        hipHostMalloc(&hm, mir, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&dm, mir) != hipSuccess) {
      if (ht) (void)hipHostFree(ht);
      if (dt) (void)hipFree(dt);
      if (hm) (void)hipHostFree(hm);
      if (dm) (void)hipFree(dm);
      for (auto p2 : g->h_tab) (void)hipHostFree(p2);
      for (auto p2 : g->d_tab) (void)hipFree(p2);
      for (auto p2 : g->h_mir) (void)hipHostFree(p2);
      for (auto p2 : g->d_mir) (void)hipFree(p2);
      return fail(ADER_EHIP, "allocating the round tables of a kernel group");
    }
    g->h_tab.push_back(static_cast<SolveDesc*>(ht));
    g->d_tab.push_back(static_cast<SolveDesc*>(dt));
    g->h_mir.push_back(static_cast<SolveClock*>(hm));
    g->d_mir.push_back(static_cast<SolveClock*>(dm));
  }
  *out = g.get();
  s->groups.emplace(key, std::move(g));
  return ADER_OK;
}

// Admit the head of the queue if a slot and arena space are free.
ader_status try_admit(ader_server s, bool* admitted) {
  *admitted = false;
  if (s->queue.empty() || s->free_slots.empty()) return ADER_OK;
  Request* r = s->queue.front();
  size_t off = 0;
  if (!s->arena->alloc(r->fp.bytes, &off)) return ADER_OK;
  Group* g = nullptr;
  if (ader_status st = get_group(s, r->prob, &g)) {
    s->arena->release(off, r->fp.bytes);
    return st;
  }
  s->queue.pop_front();
  r->off = off;
  r->slot = s->free_slots.back();
  s->free_slots.pop_back();
  r->group = group_key(r->prob);
  const Footprint& f = r->fp;
  char* base = s->arena_base + off;
  SolveDesc& d = r->desc;
  std::memset(&d, 0, sizeof(d));
  d.u[0] = reinterpret_cast<double*>(base);
  d.u[1] = reinterpret_cast<double*>(base + f.off_u1);
  d.hdr = reinterpret_cast<ader::WsHeader*>(base + f.off_hdr);
  d.partial = reinterpret_cast<double*>(base + f.off_partial);
  d.traces = base + f.off_traces;
  d.clock = s->d_clocks + r->slot;
  ader::fill_mesh_params(r->prob, f.ncells, &d.mp);
  d.mp.ld = f.ld;
  d.cfl = r->prob.cfl;
  const int nx = r->prob.n[0], ny = r->prob.n[1];
  d.tiles_x = (nx + 3) / 4;
  d.ftiles_x = (nx + ader::kFaceTX - 1) / ader::kFaceTX;
  const long long dtb = (f.ncells + ader::kBlock - 1) / ader::kBlock;
  d.dt_blocks = (int)std::min<long long>(dtb, ader::kDtMaxBlocks);
  r->dt_blocks = d.dt_blocks;
  r->cell_blocks = (long long)d.tiles_x * ((ny + ader::kBatchTY - 1) / ader::kBatchTY);
  r->face_blocks = (long long)d.ftiles_x * ((ny + ader::kFaceTY - 1) / ader::kFaceTY);

  SolveClock& ci = s->h_clock_init[r->slot];
  std::memset(&ci, 0, sizeof(ci));
  ci.t = 0.0;
  ci.t_end = r->t_end;
  hipError_t e = hipMemcpy2DAsync(d.u[0], sizeof(double) * f.ld, r->pinned,
                                  sizeof(double) * f.ncells, sizeof(double) * f.ncells, f.nv,
                                  hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d.hdr, s->h_zero, ader::kHeaderBytes, hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d.clock, &ci, sizeof(SolveClock), hipMemcpyHostToDevice, g->stream);
  if (e != hipSuccess) return hip_status(e, "ader_server_progress (admission)");
  r->state = kResident;
  r->admit_s = now_s();
  g->table.push_back(r);
  g->dirty = true;
  s->in_use += r->fp.bytes;
  s->peak_in_use = std::max(s->peak_in_use, s->in_use);
  ++s->resident;
  s->peak_resident = std::max(s->peak_resident, s->resident);
  *admitted = true;
  return ADER_OK;
}

// Enqueue the copy of a finished solve's state and header.
ader_status retire(ader_server s, Group* g, Request* r, const SolveClock& c) {
  r->retiring = true;
  r->steps = c.step;
  r->t = c.t;
  g->table.erase(std::find(g->table.begin(), g->table.end(), r));
  g->dirty = true;
  const Footprint& f = r->fp;
  char* hdr_dst = static_cast<char*>(r->pinned) + sizeof(double) * f.nv * f.ncells;
  hipError_t e = hipMemcpy2DAsync(r->pinned, sizeof(double) * f.ncells, r->desc.u[c.step & 1],
                                  sizeof(double) * f.ld, sizeof(double) * f.ncells, f.nv,
                                  hipMemcpyDeviceToHost, g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hdr_dst, r->desc.hdr, sizeof(ader::WsHeader), hipMemcpyDeviceToHost,
                       g->stream);
  if (e == hipSuccess) e = s->event(&r->done_ev);
  if (e == hipSuccess) e = hipEventRecord(r->done_ev, g->stream);
  if (e != hipSuccess) return hip_status(e, "ader_server_progress (retirement)");
  s->retiring.push_back(r);
  return ADER_OK;
}

ader_status launch_round(ader_server s, Group* g) {
  const int ring = s->cfg.rounds_ahead + 1;
  hipError_t e = hipSuccess;
  if (g->dirty) {
    // a ring entry is reused only after the round that last read it completed:
    // at most rounds_ahead rounds are in flight and the ring has one more entry
    g->table_slot = (g->table_slot + 1) % ring;
    SolveDesc* h = g->h_tab[g->table_slot];
    long long dtb = 0, cb = 0, fb = 0;
    for (size_t i = 0; i < g->table.size(); ++i) {
      Request* r = g->table[i];
      h[i] = r->desc;
      h[i].dt_block0 = dtb;
      h[i].cell_block0 = cb;
      h[i].face_block0 = fb;
      dtb += r->dt_blocks;
      cb += r->cell_blocks;
      fb += r->face_blocks;
    }
    g->ns = (int)g->table.size();
    g->dt_blocks = dtb;
    g->cell_blocks = cb;
    g->face_blocks = fb;
    e = hipMemcpyAsync(g->d_tab[g->table_slot], h, sizeof(SolveDesc) * g->ns,
                       hipMemcpyHostToDevice, g->stream);
    if (e != hipSuccess) return hip_status(e, "ader_server_progress (round table)");
    g->dirty = false;
  }
  if (g->ns == 0) return ADER_OK;
  const int m = (int)(g->rounds % ring);
  e = g->impl->round(g->d_tab[g->table_slot], g->d_mir[m], g->ns, g->dt_blocks, g->cell_blocks,
                     g->face_blocks, g->dc, g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->h_mir[m], g->d_mir[m], sizeof(SolveClock) * g->ns,
                       hipMemcpyDeviceToHost, g->stream);
  InFlight f;
  if (e == hipSuccess) e = s->event(&f.ev);
  if (e == hipSuccess) e = hipEventRecord(f.ev, g->stream);
  if (e != hipSuccess) return hip_status(e, "ader_server_progress (round)");
  f.mirror = m;
  f.reqs = g->table;
  g->inflight.push_back(std::move(f));
  ++g->rounds;
  ++s->rounds;
  s->launches += 3;
  return ADER_OK;
}

// Harvest completed rounds of a group (oldest first).
ader_status harvest(ader_server s, Group* g, bool* any) {
  while (!g->inflight.empty()) {
    InFlight& f = g->inflight.front();
    const hipError_t q = hipEventQuery(f.ev);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) return hip_status(q, "ader_server_progress (round event)");
    *any = true;
    const SolveClock* mir = g->h_mir[f.mirror];
    for (size_t i = 0; i < f.reqs.size(); ++i) {
      Request* r = f.reqs[i];
      r->t = mir[i].t;
      r->steps = mir[i].step;
      if (!r->retiring && !(mir[i].t < r->t_end))
        if (ader_status st = retire(s, g, r, mir[i])) return st;
    }
    s->release_event(f.ev);
    g->inflight.pop_front();
  }
  return ADER_OK;
}

ader_status finish_retirements(ader_server s, bool* any) {
  for (size_t i = 0; i < s->retiring.size();) {
    Request* r = s->retiring[i];
    const hipError_t q = hipEventQuery(r->done_ev);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (q != hipSuccess) return hip_status(q, "ader_server_progress (retirement event)");
    *any = true;
    const Footprint& f = r->fp;
    std::memcpy(r->u_out, r->pinned, sizeof(double) * f.nv * f.ncells);
    ader::WsHeader h;
    std::memcpy(&h, static_cast<char*>(r->pinned) + sizeof(double) * f.nv * f.ncells, sizeof(h));
    r->flags = h.status;
    r->iters = 0;
    for (int k = 0; k < ader::kCounterSlots; ++k) r->iters += h.iters[k];
    // failed: a NaN (also a NaN time) or a predictor that did not converge;
    // other flags (non-physical states) are reported with a done result
    const bool bad = !std::isfinite(r->t) || (r->flags & (ADER_FLAG_NAN | ADER_FLAG_NOCONV));
    r->state = bad ? kFailed : kDone;
    r->done_s = now_s();
    s->release_event(r->done_ev);
    r->done_ev = nullptr;
    s->arena->release(r->off, f.bytes);
    s->in_use -= f.bytes;
    --s->resident;
    s->free_slots.push_back(r->slot);
    r->slot = -1;
    s->pinned.put(r->pinned);
    r->pinned = nullptr;
    ++s->completed;
    s->retiring[i] = s->retiring.back();
    s->retiring.pop_back();
  }
  return ADER_OK;
}

}  // namespace

extern "C" {

ader_status ader_server_footprint(const ader_problem* prob, size_t* bytes) {
  if (!prob || !bytes) return fail(ADER_EINVAL, "null argument");
  int64_t ncells = 0;
  if (ader_status st = ader::validate_problem(*prob, &ncells)) return st;
  if (prob->dim != 2) return fail(ADER_EUNSUPPORTED, "the server runs 2D problems only");
  const size_t el = prob->precision == ADER_PREC_FP64 ? sizeof(double) : sizeof(float);
  *bytes = footprint(*prob, ncells, el).bytes;
  return ADER_OK;
}

ader_status ader_server_create(const ader_server_config* cfg, ader_server* out) {
  if (!cfg || !out) return fail(ADER_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->hbm_bytes < (size_t(1) << 20)) return fail(ADER_EINVAL, "hbm_bytes must be >= 1 MiB");
  if (cfg->max_slots < 1 || cfg->max_slots > 4096)
    return fail(ADER_EINVAL, "max_slots must be in 1..4096");
  if (cfg->streams < 1 || cfg->streams > 16) return fail(ADER_EINVAL, "streams must be in 1..16");
  if (cfg->rounds_ahead < 1 || cfg->rounds_ahead > 8)
    return fail(ADER_EINVAL, "rounds_ahead must be in 1..8");
  ader_server s = new (std::nothrow) ader_server_s();
  if (!s) return fail(ADER_EINVAL, "out of host memory");
  s->cfg = *cfg;
  hipError_t e = hipMalloc(&s->arena_base, cfg->hbm_bytes);
  if (e == hipSuccess) e = hipMalloc(&s->d_clocks, sizeof(SolveClock) * cfg->max_slots);
  if (e == hipSuccess)
    e = hipHostMalloc(&s->h_clock_init, sizeof(SolveClock) * cfg->max_slots, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&s->h_zero, ader::kHeaderBytes, hipHostMallocDefault);
  for (int i = 0; e == hipSuccess && i < cfg->streams; ++i) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) s->streams.push_back(st);
  }
  if (e != hipSuccess) {
    ader_status st = hip_status(e, "ader_server_create");
    ader_server_destroy(s);
    return st;
  }
  std::memset(s->h_zero, 0, ader::kHeaderBytes);
  s->arena = std::make_unique<Arena>(cfg->hbm_bytes);
  for (int i = cfg->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  *out = s;
  return ADER_OK;
}

ader_status ader_server_destroy(ader_server s) {
  if (!s) return ADER_OK;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& kv : s->groups) {
    Group* g = kv.second.get();
    for (auto& f : g->inflight) (void)hipEventDestroy(f.ev);
    for (auto p : g->h_tab) (void)hipHostFree(p);
    for (auto p : g->d_tab) (void)hipFree(p);
    for (auto p : g->h_mir) (void)hipHostFree(p);
    for (auto p : g->d_mir) (void)hipFree(p);
  }
  for (Request* r : s->retiring)
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (auto& kv : s->reqs) s->pinned.put(kv.second->pinned);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->d_clocks) (void)hipFree(s->d_clocks);
  if (s->h_clock_init) (void)hipHostFree(s->h_clock_init);
  if (s->h_zero) (void)hipHostFree(s->h_zero);
  delete s;
  return ADER_OK;
}

ader_status ader_server_submit(ader_server s, const ader_problem* prob, const double* u0,
                               double t_end, double* u_out, int64_t* id) {
  if (!s || !prob || !u0 || !u_out || !id) return fail(ADER_EINVAL, "null argument");
  int64_t ncells = 0;
  if (ader_status st = ader::validate_problem(*prob, &ncells)) return st;
  if (prob->dim != 2) return fail(ADER_EUNSUPPORTED, "the server runs 2D problems only");
  if (!std::isfinite(t_end) || !(t_end > 0.0)) return fail(ADER_EINVAL, "t_end must be > 0");
  auto r = std::make_unique<Request>();
  r->prob = *prob;
  r->prob.n[2] = 1;
  const size_t el = prob->precision == ADER_PREC_FP64 ? sizeof(double) : sizeof(float);
  r->fp = footprint(r->prob, ncells, el);
  if (r->fp.bytes > s->cfg.hbm_bytes)
    return fail(ADER_EINVAL, "the solve's footprint exceeds the server's arena");
  const size_t state = sizeof(double) * r->fp.nv * ncells;
  r->pinned = s->pinned.get(state + sizeof(ader::WsHeader));
  if (!r->pinned) return fail(ADER_EHIP, "allocating pinned host memory");
  std::memcpy(r->pinned, u0, state);
  r->t_end = t_end;
  r->u_out = u_out;
  r->id = s->next_id++;
  r->submit_s = now_s();
  *id = r->id;
  s->queue.push_back(r.get());
  s->reqs.emplace(r->id, std::move(r));
  return ADER_OK;
}

ader_status ader_server_progress(ader_server s, int wait, int* resident, int* queued) {
  if (!s) return fail(ADER_EINVAL, "null argument");
  bool any = false;
  for (auto& kv : s->groups)
    if (ader_status st = harvest(s, kv.second.get(), &any)) return st;
  if (ader_status st = finish_retirements(s, &any)) return st;
  for (;;) {
    bool admitted = false;
    if (ader_status st = try_admit(s, &admitted)) return st;
    if (!admitted) break;
  }
  for (auto& kv : s->groups) {
    Group* g = kv.second.get();
    if ((int)g->inflight.size() < s->cfg.rounds_ahead && (!g->table.empty() || g->dirty))
      if (ader_status st = launch_round(s, g)) return st;
  }
  if (wait && !any) {
    // block on the oldest outstanding event: a round, else a retirement
    hipEvent_t e = nullptr;
    for (auto& kv : s->groups)
      if (!e && !kv.second->inflight.empty()) e = kv.second->inflight.front().ev;
    if (!e && !s->retiring.empty()) e = s->retiring.front()->done_ev;
    if (e) {
      const hipError_t q = hipEventSynchronize(e);
      if (q != hipSuccess) return hip_status(q, "ader_server_progress (wait)");
    }
  }
  if (resident) *resident = s->resident;
  if (queued) *queued = (int)s->queue.size();
  return ADER_OK;
}

ader_status ader_server_request(ader_server s, int64_t id, ader_request_info* info) {
  if (!s || !info) return fail(ADER_EINVAL, "null argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(ADER_EINVAL, "unknown request id");
  const Request& r = *it->second;
  info->state = r.state;
  info->flags = r.flags;
  info->steps = r.steps;
  info->picard_iterations = r.iters;
  info->t = r.t;
  info->submit_s = r.submit_s;
  info->admit_s = r.admit_s;
  info->done_s = r.done_s;
  return ADER_OK;
}

ader_status ader_server_stats_get(ader_server s, ader_server_stats* st) {
  if (!s || !st) return fail(ADER_EINVAL, "null argument");
  st->arena_bytes = s->cfg.hbm_bytes;
  st->bytes_in_use = s->in_use;
  st->peak_bytes_in_use = s->peak_in_use;
  st->resident = s->resident;
  st->peak_resident = s->peak_resident;
  st->queued = (int)s->queue.size();
  st->rounds = s->rounds;
  st->launches = s->launches;
  st->completed = s->completed;
  return ADER_OK;
}

}  // extern "C"
