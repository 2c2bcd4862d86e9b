// 16-bit tile formats of the reduced-precision forms.
//
// A slot of a BF16 / FP16 matrix holds 1024 16-bit values of the block
// (part 0), then the same values transposed (part 1), each part in the
// operand order of the leaf kernels (half_idx), so that both the A role
// (rows of A_ik) and the B role (columns of B_kj) of a leaf product read
// 1 KiB contiguously per load of a wave.  The split forms
// (BF16X3, FP16X3) add a low part and its transpose (parts 2 and 3):
//   x = hi + lo * 2^-L,  hi = round16(x),  lo = round16((x - hi) * 2^L),
// L = 0 for BF16 (its exponent range covers the residual) and L = 11 for
// FP16, which keeps the residual of values down to ~1e-4 out of FP16's
// subnormal range.  A leaf product then takes hi*hi + 2^-L (hi*lo + lo*hi),
// three MFMA products with FP32 accumulation, two accumulators.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace spamm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__host__ __device__ constexpr bool is_half(int prec) {
  return prec == SPAMM_BF16 || prec == SPAMM_FP16 || prec == SPAMM_BF16X3 ||
         prec == SPAMM_FP16X3;
}
__host__ __device__ constexpr bool is_split(int prec) {
  return prec == SPAMM_BF16X3 || prec == SPAMM_FP16X3;
}
__host__ __device__ constexpr bool is_bf16(int prec) {
  return prec == SPAMM_BF16 || prec == SPAMM_BF16X3;
}
// Scale of the low part: x = hi + lo * 2^-L.
__host__ __device__ constexpr float lo_scale(int prec) { return prec == SPAMM_FP16X3 ? 2048.0f : 1.0f; }
// Largest magnitude a tile may hold (FP16's finite range; BF16 has FP32's).
__host__ __device__ constexpr double half_max(int prec) {
  return is_bf16(prec) ? 3.0e38 : 65504.0;
}

template <int P>
struct Half;
template <>
struct Half<SPAMM_BF16> {
  typedef __bf16 T;
  typedef bf16x8 V;
};
template <>
struct Half<SPAMM_BF16X3> {
  typedef __bf16 T;
  typedef bf16x8 V;
};
template <>
struct Half<SPAMM_FP16> {
  typedef _Float16 T;
  typedef f16x8 V;
};
template <>
struct Half<SPAMM_FP16X3> {
  typedef _Float16 T;
  typedef f16x8 V;
};

// hi and lo of x (lo = 0 for the non-split forms).
template <int P>
__device__ inline void encode_half(double x, typename Half<P>::T& hi, typename Half<P>::T& lo) {
  typedef typename Half<P>::T T;
  hi = T(float(x));
  if (is_split(P)) {
    const double r = (x - double(float(hi))) * double(lo_scale(P));
    lo = T(float(r));
  } else {
    lo = T(0.0f);
  }
}

template <int P>
__device__ inline double decode_half(typename Half<P>::T hi, typename Half<P>::T lo) {
  double v = double(float(hi));
  if (is_split(P)) v += double(float(lo)) / double(lo_scale(P));
  return v;
}

// The same in FP32, exact for values that FP32 holds: hi + lo * 2^-L spans
// at most 22 significant bits, and v - hi is exact for hi = round16(v).
template <int P>
__device__ inline void encode_half_f(float v, typename Half<P>::T& hi, typename Half<P>::T& lo) {
  typedef typename Half<P>::T T;
  hi = T(v);
  lo = is_split(P) ? T((v - float(hi)) * lo_scale(P)) : T(0.0f);
}

template <int P>
__device__ inline float decode_half_f(typename Half<P>::T hi, typename Half<P>::T lo) {
  float v = float(hi);
  if (is_split(P)) v += float(lo) * (1.0f / lo_scale(P));
  return v;
}

// Element offsets of the parts of a 16-bit tile.
__host__ __device__ constexpr int64_t half_part(int part) { return int64_t(part) * kLeaf2; }

// Position of element (r, c) inside a part: the 16-byte operand of lane
// l = 32 kk + r for MFMA step s (k = 16 kk + 8 s .. + 7) is chunk 64 s + l,
// so each step's operand load of a wave reads 1 KiB contiguously.
__host__ __device__ constexpr int half_idx(int r, int c) {
  return (((c & 15) >> 3) * 64 + (c >> 4) * 32 + r) * 8 + (c & 7);
}
// Whether position x of a part holds a diagonal element (r == c).
__host__ __device__ constexpr bool half_idx_diag(int x) {
  return ((x >> 3) & 31) == (((x >> 8) & 1) << 4) + ((x >> 9) << 3) + (x & 7);
}

}  // namespace spamm
