// Device side of an AMR mesh change (Section 3.1, rules 1-7; thresholds of
// Section 3.1.1) on the dense per-level representation: indicator flags,
// Voronoi dilations, closure, status, level lists (stream compaction) and the
// slots that tie a level's new cells to their mothers' reconstructions.
// Every kernel is a gather over one level's index space (no atomics on the
// data), so the results do not depend on the launch order of the blocks.
#include <hipcub/hipcub.hpp>

#include "../../include/ader.h"

#include "amr_plan.hpp"

namespace ader {
namespace {

__device__ __forceinline__ void rg_coords(const RgGrid& g, int64_t i, int (&c)[3]) {
  c[0] = (int)(i % g.n[0]);
  c[1] = (int)((i / g.n[0]) % g.n[1]);
  c[2] = (int)(i / ((int64_t)g.n[0] * g.n[1]));
}

__device__ __forceinline__ int64_t rg_index(const RgGrid& g, const int (&c)[3]) {
  return c[0] + (int64_t)g.n[0] * (c[1] + (int64_t)g.n[1] * c[2]);
}

__device__ __forceinline__ int rg_map(int i, int n, int bc) {
  if (bc == ADER_BC_PERIODIC) return ((i % n) + n) % n;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Loehner indicator (eq. indicator) in index units on one variable, term by
// term in the order of the oracle with no fused multiply-adds, then the
// refine / keep decision: active cells with chi > chi_ref, virtual mothers
// with chi >= chi_rec.  Other cells get no flag.
__global__ void __launch_bounds__(kBlock)
k_rg_lohner(RgGrid g, const double* __restrict__ phi, const int8_t* __restrict__ st, double eps,
            double chi_ref, double chi_rec, uint8_t* __restrict__ F) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= g.N) return;
  const int8_t s = st[i];
  if (s != kActive && s != kVMother) {
    F[i] = 0;
    return;
  }
  int c[3];
  rg_coords(g, i, c);
  auto at = [&](int ok, int ov, int k, int m) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[k] = rg_map(cc[k] + ok, g.n[k], g.bc[k]);
    cc[m] = rg_map(cc[m] + ov, g.n[m], g.bc[m]);
    return phi[rg_index(g, cc)];
  };
  const double P = phi[i];
  double num = 0.0, den = 0.0;
  for (int k = 0; k < g.dim; ++k) {
    for (int m = 0; m < g.dim; ++m) {
      double D, De;
      if (k == m) {
        int e[3] = {c[0], c[1], c[2]}, f[3] = {c[0], c[1], c[2]};
        e[k] = rg_map(c[k] + 1, g.n[k], g.bc[k]);
        f[k] = rg_map(c[k] - 1, g.n[k], g.bc[k]);
        const double p = phi[rg_index(g, e)], q = phi[rg_index(g, f)];
        D = p - 2.0 * P + q;
        De = fabs(p - P) + fabs(P - q) + eps * (fabs(p) + 2.0 * fabs(P) + fabs(q));
      } else {
        const double pp = at(1, 1, k, m), pm = at(1, -1, k, m), mp = at(-1, 1, k, m),
                     mm = at(-1, -1, k, m);
        const double A = pp - mp, B = pm - mm;
        D = 0.25 * (A - B);
        De = 0.25 * (fabs(A) + fabs(B)) + 0.25 * eps * (fabs(pp) + fabs(pm) + fabs(mp) + fabs(mm));
      }
      num += D * D;
      den += De * De;
    }
  }
  const double chi = den > 0.0 ? sqrt(num / den) : 0.0;
  F[i] = (s == kActive && chi > chi_ref) || (s == kVMother && chi >= chi_rec) ? 1 : 0;
}

// out = Voronoi (3^d) neighbourhood of the flagged cells of 'in', in gather
// form: no wrap through a transmissive boundary.
__global__ void __launch_bounds__(kBlock)
k_rg_dilate(RgGrid g, const uint8_t* __restrict__ in, uint8_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= g.N) return;
  int c[3];
  rg_coords(g, i, c);
  const int sy = g.dim > 1 ? 1 : 0, sz = g.dim > 2 ? 1 : 0;
  uint8_t v = 0;
  for (int dz = -sz; dz <= sz && !v; ++dz)
    for (int dy = -sy; dy <= sy && !v; ++dy)
      for (int dx = -1; dx <= 1 && !v; ++dx) {
        const int o[3] = {dx, dy, dz};
        int cc[3] = {0, 0, 0};
        bool ok = true;
        for (int k = 0; k < g.dim; ++k) {
          const int raw = c[k] + o[k];
          if (g.bc[k] != ADER_BC_PERIODIC && (raw < 0 || raw >= g.n[k])) ok = false;
          cc[k] = rg_map(raw, g.n[k], g.bc[k]);
        }
        if (ok && in[rg_index(g, cc)]) v = 1;
      }
  out[i] = v;
}

// Fc |= (some child flagged in Ff)
__global__ void __launch_bounds__(kBlock)
k_rg_mothers_or(RgGrid fine, RgGrid coarse, int r, const uint8_t* __restrict__ Ff,
                uint8_t* __restrict__ Fc) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= coarse.N) return;
  int c[3];
  rg_coords(coarse, i, c);
  const int ry = fine.dim > 1 ? r : 1, rz = fine.dim > 2 ? r : 1;
  uint8_t v = Fc[i];
  for (int z = 0; z < rz && !v; ++z)
    for (int y = 0; y < ry && !v; ++y)
      for (int x = 0; x < r && !v; ++x) {
        const int f[3] = {c[0] * r + x, c[1] * ry + y, c[2] * rz + z};
        if (Ff[rg_index(fine, f)]) v = 1;
      }
  Fc[i] = v;
}

// Ff &= Fc[mother]
__global__ void __launch_bounds__(kBlock)
k_rg_nest(RgGrid fine, RgGrid coarse, int r, const uint8_t* __restrict__ Fc,
          uint8_t* __restrict__ Ff) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= fine.N) return;
  int c[3];
  rg_coords(fine, i, c);
  for (int k = 0; k < fine.dim; ++k) c[k] /= r;
  if (!Fc[rg_index(coarse, c)]) Ff[i] = 0;
}

// Status of level l >= 1: children of flagged cells are active (virtual
// mothers when flagged themselves, Ff non-null below the finest level),
// children of unflagged near cells are virtual children, the rest absent.
__global__ void __launch_bounds__(kBlock)
k_rg_status(RgGrid fine, RgGrid coarse, int r, const uint8_t* __restrict__ Fc,
            const uint8_t* __restrict__ near_c, const uint8_t* __restrict__ Ff,
            int8_t* __restrict__ st) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= fine.N) return;
  int c[3];
  rg_coords(fine, i, c);
  for (int k = 0; k < fine.dim; ++k) c[k] /= r;
  const int64_t m = rg_index(coarse, c);
  int8_t s = kAbsent;
  if (Fc[m])
    s = (Ff && Ff[i]) ? kVMother : kActive;
  else if (near_c[m])
    s = kVChild;
  st[i] = s;
}

__global__ void __launch_bounds__(kBlock)
k_rg_status0(int64_t N, const uint8_t* __restrict__ F0, int8_t* __restrict__ st) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  st[i] = (F0 && F0[i]) ? kVMother : kActive;
}

__global__ void __launch_bounds__(kBlock)
k_rg_diff(int64_t N, const int8_t* __restrict__ a, const int8_t* __restrict__ b,
          unsigned int* __restrict__ changed) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool d = i < N && a[i] != b[i];
  if (__ballot(d) && (threadIdx.x & 63) == 0) atomicOr(changed, 1u);
}

// removed cells (absent now, not before) become NaN in every variable
__global__ void __launch_bounds__(kBlock)
k_rg_gone(int64_t N, int nv, double* __restrict__ u, const int8_t* __restrict__ st_new,
          const int8_t* __restrict__ st_old) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N || st_new[i] != kAbsent || st_old[i] == kAbsent) return;
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  for (int v = 0; v < nv; ++v) u[(int64_t)v * N + i] = nan;
}

__global__ void __launch_bounds__(kBlock)
k_rg_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void __launch_bounds__(kBlock)
k_rg_scatter_pos(int32_t* __restrict__ pos, const int32_t* __restrict__ list, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < n) pos[list[j]] = (int32_t)j;
}

// tslot[i] = slot_c[mother of targets[i]]
__global__ void __launch_bounds__(kBlock)
k_rg_slots(RgGrid fine, RgGrid coarse, int r, const int32_t* __restrict__ targets, int64_t nt,
           const int32_t* __restrict__ slot_c, int32_t* __restrict__ tslot) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nt) return;
  int c[3];
  rg_coords(fine, targets[i], c);
  for (int k = 0; k < fine.dim; ++k) c[k] /= r;
  tslot[i] = slot_c[rg_index(coarse, c)];
}

struct RgSelect {
  const int8_t* st;
  const int8_t* old;
  int mode;
  __host__ __device__ bool operator()(const int32_t& i) const {
    const int8_t s = st[i];
    switch (mode) {
      case kSelActive: return s == kActive;
      case kSelVChild: return s == kVChild;
      case kSelVMother: return s == kVMother;
      case kSelMothers: return s == kActive || s == kVMother;
      default: return s != kAbsent && old[i] == kAbsent;  // kSelBorn
    }
  }
};

unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1); }

}  // namespace

hipError_t rg_lohner(const RgGrid& g, const double* phi, const int8_t* st, double eps,
                     double chi_ref, double chi_rec, uint8_t* F, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_lohner, dim3(blocks(g.N)), dim3(kBlock), 0, s, g, phi, st, eps, chi_ref,
                     chi_rec, F);
  return hipGetLastError();
}

hipError_t rg_dilate(const RgGrid& g, const uint8_t* in, uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_dilate, dim3(blocks(g.N)), dim3(kBlock), 0, s, g, in, out);
  return hipGetLastError();
}

hipError_t rg_mothers_or(const RgGrid& fine, const RgGrid& coarse, int r, const uint8_t* Ff,
                         uint8_t* Fc, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_mothers_or, dim3(blocks(coarse.N)), dim3(kBlock), 0, s, fine, coarse,
                     r, Ff, Fc);
  return hipGetLastError();
}

hipError_t rg_nest(const RgGrid& fine, const RgGrid& coarse, int r, const uint8_t* Fc,
                   uint8_t* Ff, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_nest, dim3(blocks(fine.N)), dim3(kBlock), 0, s, fine, coarse, r, Fc,
                     Ff);
  return hipGetLastError();
}

hipError_t rg_status(const RgGrid& fine, const RgGrid& coarse, int r, const uint8_t* Fc,
                     const uint8_t* near_c, const uint8_t* Ff, int8_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_status, dim3(blocks(fine.N)), dim3(kBlock), 0, s, fine, coarse, r, Fc,
                     near_c, Ff, st);
  return hipGetLastError();
}

hipError_t rg_status0(int64_t N, const uint8_t* F0, int8_t* st, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_status0, dim3(blocks(N)), dim3(kBlock), 0, s, N, F0, st);
  return hipGetLastError();
}

hipError_t rg_diff(int64_t N, const int8_t* a, const int8_t* b, unsigned int* changed,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_rg_diff, dim3(blocks(N)), dim3(kBlock), 0, s, N, a, b, changed);
  return hipGetLastError();
}

hipError_t rg_gone(int64_t N, int nv, double* u, const int8_t* st_new, const int8_t* st_old,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_rg_gone, dim3(blocks(N)), dim3(kBlock), 0, s, N, nv, u, st_new, st_old);
  return hipGetLastError();
}

hipError_t rg_positions(int32_t* pos, int64_t N, const int32_t* list, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_rg_fill_i32, dim3(blocks(N)), dim3(kBlock), 0, s, pos, N, (int32_t)-1);
  if (n > 0)
    hipLaunchKernelGGL(k_rg_scatter_pos, dim3(blocks(n)), dim3(kBlock), 0, s, pos, list, n);
  return hipGetLastError();
}

hipError_t rg_slots(const RgGrid& fine, const RgGrid& coarse, int r, const int32_t* targets,
                    int64_t nt, const int32_t* slot_c, int32_t* tslot, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rg_slots, dim3(blocks(nt)), dim3(kBlock), 0, s, fine, coarse, r, targets,
                     nt, slot_c, tslot);
  return hipGetLastError();
}

hipError_t rg_select(int mode, const int8_t* st, const int8_t* old, int64_t N, int32_t* out,
                     int* d_count, void* temp, size_t* temp_bytes, hipStream_t s) {
  hipcub::CountingInputIterator<int32_t> it(0);
  return hipcub::DeviceSelect::If(temp, *temp_bytes, it, out, d_count, (int)N,
                                  RgSelect{st, old, mode}, s);
}

}  // namespace ader
