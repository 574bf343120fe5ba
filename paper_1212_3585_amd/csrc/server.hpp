// Launchers of the batched rounds used by the solve server (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "batch.hpp"

namespace ader {

constexpr int kBatchTY = 8;  // cell kernel tile rows (tile = 4 x kBatchTY cells)

class BatchImplBase {
 public:
  virtual ~BatchImplBase() = default;
  virtual size_t trace_elem_size() const = 0;
  // One round over the table d_desc[0..ns) (device memory); blocks are the
  // totals of the per-solve block counts; d_mirror[0..ns) receives the
  // solves' clocks after the round's time update.
  virtual hipError_t round(const SolveDesc* d_desc, SolveClock* d_mirror, int ns,
                           long long dt_blocks,
                           long long cell_blocks, long long face_blocks, const DevConsts& c,
                           hipStream_t st) const = 0;
};

// nullptr if (M, system, precision) has no kernels (2D only)
const BatchImplBase* make_batch_impl_2d(int M, int system, int precision);

}  // namespace ader
