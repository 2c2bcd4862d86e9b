// Leaf products of SpAMM on the MFMA units (the dense C <- C + A x B on
// N_b x N_b blocks of Sec. 3, here N_b = 32), with the SP2 update fused
// into the epilogue.
//
// Ownership: one 64-lane wave owns one C block and walks its task list in
// ascending k, so every C block is written by exactly one wave, in a fixed
// order, with no atomics (the role of the paper's per-block locks in Alg. 1
// and of the exclusive store phase of Alg. 2).
//
// Operand placement.  The MFMA sums over its k slots; which global k goes
// to which slot is free as long as A and B agree.  Slot kk of step s takes
// k = kk * (32 / #slots) + s, so each lane's A operands are one contiguous
// run of a tile row (vector loads) and each B operand step is one
// coalesced row segment.
//   FP32: v_mfma_f32_32x32x2f32, 16 steps per leaf product.
//         A lane l: row l%32, k = (l/32)*16 + s; B lane l: col l%32.
//         D reg r: row (r/4)*8 + (l/32)*4 + r%4, col l%32.
//   FP64: v_mfma_f64_16x16x4f64 on the 2 x 2 sub-blocks, 8 steps each.
//         A lane l: row l%16, k = (l/16)*8 + s; B lane l: col l%16.
//         D reg r: row l/16 + 4r, col l%16.
#include "internal.h"

namespace spamm {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Epilogue shared by both precisions: value c at (row, col) of C block
// (i, j).  Plain product: store c.  SP2: X_{n+1} = c or 2 x - c, plus the
// block's ||X_{n+1}||^2, ||C - X_n||^2 and diagonal sum.
template <class T>
struct Epi {
  double nrm = 0.0, err = 0.0, tr = 0.0;
  __device__ inline T apply(T c, T x, bool sp2, bool square, bool diag) {
    T v = c;
    if (sp2) {
      v = square ? c : T(2) * x - c;
      const double d = double(c) - double(x);
      err += d * d;
    }
    nrm += double(v) * double(v);
    if (diag) tr += double(v);
    return v;
  }
  __device__ inline void finish(const GemmArgs& g, int64_t node, int32_t ij, int lane) {
    const int i = unpack_i(ij), j = unpack_j(ij);
    const double n2 = wave_sum(nrm);
    const double e2 = g.sp2 ? wave_sum(err) : 0.0;
    const double t = (g.sp2 && i == j) ? wave_sum(tr) : 0.0;
    if (lane == 0) {
      const int64_t cell = int64_t(i) * g.nb + j;
      g.norm_c[cell] = sqrt(n2);
      g.map_c[cell] = int32_t(node);
      g.coords_c[node] = ij;
      if (g.sp2) {
        g.err_part[cell] = e2;
        if (i == j) g.trace_part[i] = t;
      }
    }
  }
};

struct F32Frag {
  v4f a[4];
  float b[16];
};

__device__ inline void load_f32(const float* __restrict__ A, const float* __restrict__ B, int lane,
                                F32Frag& f) {
  const int m = lane & 31, kk = lane >> 5;
  const v4f* pa = reinterpret_cast<const v4f*>(A + m * kLeaf + kk * 16);
#pragma unroll
  for (int q = 0; q < 4; ++q) f.a[q] = pa[q];
  const float* pb = B + (kk * 16) * kLeaf + m;
#pragma unroll
  for (int s = 0; s < 16; ++s) f.b[s] = pb[s * kLeaf];
}

__device__ inline void mma_f32(const F32Frag& f, v16f& acc) {
#pragma unroll
  for (int s = 0; s < 16; ++s)
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[s >> 2][s & 3], f.b[s], acc, 0, 0, 0);
}

__global__ void __launch_bounds__(256) k_leaf_gemm_f32(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int64_t node = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  if (node >= g.n_nodes) return;
  const int32_t ij = g.nodes[node];
  const int i = unpack_i(ij), j = unpack_j(ij);
  const float* pa = static_cast<const float*>(g.pool_a);
  const float* pb = static_cast<const float*>(g.pool_b);
  const int64_t t0 = g.nptr[node], t1 = g.nptr[node + 1];
  v16f acc = {};
  F32Frag cur, nxt;
  auto tile_a = [&](int64_t t) {
    return pa + int64_t(g.map_a[int64_t(i) * g.nb + g.ks[t]]) * kLeaf2;
  };
  auto tile_b = [&](int64_t t) {
    return pb + int64_t(g.map_b[int64_t(g.ks[t]) * g.nb + j]) * kLeaf2;
  };
  if (t0 < t1) load_f32(tile_a(t0), tile_b(t0), lane, cur);
  for (int64_t t = t0; t < t1; ++t) {
    if (t + 1 < t1) load_f32(tile_a(t + 1), tile_b(t + 1), lane, nxt);
    mma_f32(cur, acc);
    cur = nxt;
  }
  float* out = static_cast<float*>(g.pool_c) + node * kLeaf2;
  const float* xt = nullptr;
  if (g.sp2) {
    const int32_t sx = g.map_x[int64_t(i) * g.nb + j];
    if (sx >= 0) xt = static_cast<const float*>(g.pool_x) + int64_t(sx) * kLeaf2;
  }
  const int col = lane & 31, kk = lane >> 5;
  Epi<float> e;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = (r >> 2) * 8 + kk * 4 + (r & 3);
    const float x = xt ? xt[row * kLeaf + col] : 0.0f;
    out[row * kLeaf + col] = e.apply(acc[r], x, g.sp2, g.square, i == j && row == col);
  }
  e.finish(g, node, ij, lane);
}

struct F64Frag {
  double a[2][8];
  double b[2][8];
};

__device__ inline void load_f64(const double* __restrict__ A, const double* __restrict__ B, int lane,
                                F64Frag& f) {
  const int m = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double* pa = A + (p * 16 + m) * kLeaf + kk * 8;
#pragma unroll
    for (int s = 0; s < 8; ++s) f.a[p][s] = pa[s];
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double* pb = B + (kk * 8) * kLeaf + q * 16 + m;
#pragma unroll
    for (int s = 0; s < 8; ++s) f.b[q][s] = pb[s * kLeaf];
  }
}

__device__ inline void mma_f64(const F64Frag& f, v4d (&acc)[2][2]) {
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[p][s], f.b[q][s], acc[p][q], 0, 0, 0);
}

__global__ void __launch_bounds__(256) k_leaf_gemm_f64(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int64_t node = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  if (node >= g.n_nodes) return;
  const int32_t ij = g.nodes[node];
  const int i = unpack_i(ij), j = unpack_j(ij);
  const double* pa = static_cast<const double*>(g.pool_a);
  const double* pb = static_cast<const double*>(g.pool_b);
  const int64_t t0 = g.nptr[node], t1 = g.nptr[node + 1];
  v4d acc[2][2] = {};
  F64Frag cur, nxt;
  auto tile_a = [&](int64_t t) {
    return pa + int64_t(g.map_a[int64_t(i) * g.nb + g.ks[t]]) * kLeaf2;
  };
  auto tile_b = [&](int64_t t) {
    return pb + int64_t(g.map_b[int64_t(g.ks[t]) * g.nb + j]) * kLeaf2;
  };
  if (t0 < t1) load_f64(tile_a(t0), tile_b(t0), lane, cur);
  for (int64_t t = t0; t < t1; ++t) {
    if (t + 1 < t1) load_f64(tile_a(t + 1), tile_b(t + 1), lane, nxt);
    mma_f64(cur, acc);
    cur = nxt;
  }
  double* out = static_cast<double*>(g.pool_c) + node * kLeaf2;
  const double* xt = nullptr;
  if (g.sp2) {
    const int32_t sx = g.map_x[int64_t(i) * g.nb + j];
    if (sx >= 0) xt = static_cast<const double*>(g.pool_x) + int64_t(sx) * kLeaf2;
  }
  const int m = lane & 15, kk = lane >> 4;
  Epi<double> e;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = p * 16 + kk + 4 * r, col = q * 16 + m;
        const double x = xt ? xt[row * kLeaf + col] : 0.0;
        out[row * kLeaf + col] = e.apply(acc[p][q][r], x, g.sp2, g.square, i == j && row == col);
      }
  e.finish(g, node, ij, lane);
}

// SP2 blocks of X_n with no executed product: C = 0 there, so
// ||C - X_n||^2 gains ||X_n||^2, and the 2X - X^2 branch carries 2 X_n.
template <class T>
__global__ void __launch_bounds__(256) k_sp2_rest(RestArgs r) {
  const int lane = threadIdx.x & 63;
  const int64_t s = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  if (s >= r.n_x) return;
  const int32_t ij = r.coords_x[s];
  const int i = unpack_i(ij), j = unpack_j(ij);
  const int64_t cell = int64_t(i) * r.nb + j;
  if (r.map_out[cell] >= 0) return;  // has products: done by the leaf GEMM
  const T* x = static_cast<const T*>(r.pool_x) + s * kLeaf2;
  T v[16];
  double e = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    v[q] = x[q * 64 + lane];
    e += double(v[q]) * double(v[q]);
  }
  e = wave_sum(e);
  if (lane == 0) r.err_part[cell] = e;
  if (r.square) return;
  int64_t slot = 0;
  if (lane == 0) slot = r.base_slot + atomicAdd(reinterpret_cast<unsigned long long*>(r.counter), 1ull);
  slot = __shfl(slot, 0, 64);
  T* out = static_cast<T*>(r.pool_out) + slot * kLeaf2;
  double nrm = 0.0, tr = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e_ = q * 64 + lane;
    const T w = T(2) * v[q];
    out[e_] = w;
    nrm += double(w) * double(w);
    if (i == j && (e_ >> 5) == (e_ & 31)) tr += double(w);
  }
  nrm = wave_sum(nrm);
  if (i == j) tr = wave_sum(tr);
  if (lane == 0) {
    r.map_out[cell] = int32_t(slot);
    r.coords_out[slot] = ij;
    r.norm_out[cell] = sqrt(nrm);
    if (i == j) r.trace_part[i] = tr;
  }
}

__global__ void __launch_bounds__(1024) k_sp2_reduce(int nb, const double* __restrict__ trace_part,
                                                     const double* __restrict__ err_part,
                                                     const double* __restrict__ norm_leaf,
                                                     Control* ctl) {
  __shared__ double st[1024], se[1024], sf[1024];
  double t = 0.0, e = 0.0, f = 0.0;
  const int64_t cells = int64_t(nb) * nb;
  for (int64_t x = threadIdx.x; x < nb; x += blockDim.x) t += trace_part[x];
  if (err_part)
    for (int64_t x = threadIdx.x; x < cells; x += blockDim.x) e += err_part[x];
  if (norm_leaf)
    for (int64_t x = threadIdx.x; x < cells; x += blockDim.x) f += norm_leaf[x] * norm_leaf[x];
  st[threadIdx.x] = t;
  se[threadIdx.x] = e;
  sf[threadIdx.x] = f;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      st[threadIdx.x] += st[threadIdx.x + o];
      se[threadIdx.x] += se[threadIdx.x + o];
      sf[threadIdx.x] += sf[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctl->sp2_trace = st[0];
    ctl->sp2_err2 = se[0];
    ctl->frob2 = sf[0];
    ctl->extra_blocks = ctl->scratch[1];
  }
}

}  // namespace

void launch_leaf_gemm(int prec, const GemmArgs& g, hipStream_t s) {
  if (g.n_nodes <= 0) return;
  const unsigned grid = unsigned((g.n_nodes + kWaves - 1) / kWaves);
  if (prec == SPAMM_FP64)
    k_leaf_gemm_f64<<<grid, 64 * kWaves, 0, s>>>(g);
  else
    k_leaf_gemm_f32<<<grid, 64 * kWaves, 0, s>>>(g);
}

void launch_sp2_rest(int prec, const RestArgs& r, hipStream_t s) {
  if (r.n_x <= 0) return;
  const unsigned grid = unsigned((r.n_x + kWaves - 1) / kWaves);
  if (prec == SPAMM_FP64)
    k_sp2_rest<double><<<grid, 64 * kWaves, 0, s>>>(r);
  else
    k_sp2_rest<float><<<grid, 64 * kWaves, 0, s>>>(r);
}

void launch_sp2_reduce(int nb, const double* trace_part, const double* err_part,
                       const double* norm_leaf, Control* ctl, hipStream_t s) {
  k_sp2_reduce<<<1, 1024, 0, s>>>(nb, trace_part, err_part, norm_leaf, ctl);
}

}  // namespace spamm
