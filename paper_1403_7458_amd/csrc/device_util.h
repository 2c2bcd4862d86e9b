// Small device helpers shared by the leaf-product kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spamm {

constexpr int kXcds = 8;

// Workgroups are dispatched to the 8 XCDs round-robin; renumber them so
// that each XCD (and its L2) works through one contiguous range of the
// Morton-ordered C blocks, whose A rows and B columns overlap.
__device__ inline int64_t xcd_contiguous_block() {
  const int64_t g = gridDim.x, b = blockIdx.x;
  const int64_t x = b % kXcds, r = b / kXcds;
  const int64_t q = g / kXcds, rem = g % kXcds;
  return x * q + min(x, rem) + r;
}

// Wave-uniform copies (scalar registers), so that loops over a C block's
// tasks compile to scalar branches with exact memory waits.
__device__ inline int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace spamm
