// Kernels of the library's test hooks: workspace poisoning (opts.flags bit 5)
// and the recursive-residual perturbation (pbcgs_debug_perturb).  Neither runs
// unless its hook is switched on.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pbcgs {

constexpr int kDebugWG = 256;
constexpr int64_t kDebugMaxBlocks = 4096;

inline unsigned debug_blocks(int64_t n) {
  const int64_t g = (n + kDebugWG - 1) / kDebugWG;
  return (unsigned)(g < 1 ? 1 : (g > kDebugMaxBlocks ? kDebugMaxBlocks : g));
}

// Sets n 32-bit words to all-ones bits: a quiet NaN whether the words are read
// as binary32 values or in pairs as binary64 values.  Any result computed from
// a word that a solve reads before writing it becomes NaN.
__global__ __launch_bounds__(kDebugWG) void k_poison(uint32_t* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kDebugWG;
  for (int64_t k = (int64_t)blockIdx.x * kDebugWG + threadIdx.x; k < n; k += stride) p[k] = 0xFFFFFFFFu;
}

// v_k = v_k * c for k < n, one rounding per entry.
__global__ __launch_bounds__(kDebugWG) void k_scale_vec(double* v, int32_t n, double c) {
  const int64_t stride = (int64_t)gridDim.x * kDebugWG;
  for (int64_t k = (int64_t)blockIdx.x * kDebugWG + threadIdx.x; k < n; k += stride) v[k] = v[k] * c;
}

}  // namespace pbcgs
