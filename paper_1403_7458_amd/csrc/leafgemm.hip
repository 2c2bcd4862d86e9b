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
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "device_util.h"
#include "internal.h"

namespace spamm {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
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
  // ms: the mirror's slot (symmetric products), or -1.
  __device__ inline void finish(const GemmArgs& g, int64_t node, int32_t ij, int lane,
                                int64_t ms) {
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
      if (ms >= 0) {
        const int64_t mcell = int64_t(j) * g.nb + i;
        g.norm_c[mcell] = sqrt(n2);
        g.map_c[mcell] = int32_t(ms);
        g.coords_c[ms] = pack_ij(j, i);
        if (g.sp2) g.err_part[mcell] = e2;
      }
    }
  }
};

// Tile slots of a C block's tasks, looked up 64 at a time (one task per
// lane) into a per-wave LDS list.  Reading a slot is then an LDS load, so
// the operand loads of the next product never wait behind the index loads
// (k, then the two block maps) or behind the current product's operands.
struct TaskSlots {
  const GemmArgs& g;
  int i, j;
  int64_t t1, base;
  int32_t* lds;  // [2][64] for this wave
  __device__ TaskSlots(const GemmArgs& g_, int i_, int j_, int64_t t0, int64_t t1_, int32_t* lds_,
                       int lane)
      : g(g_), i(i_), j(j_), t1(t1_), lds(lds_) {
    fetch(t0, lane);
  }
  __device__ inline void fetch(int64_t b, int lane) {
    base = b;
    const int64_t t = b + lane;
    int32_t sa = 0, sb = 0;
    if (t < t1) {
      const int k = g.ks[t];
      sa = g.map_a[int64_t(i) * g.nb + k];
      sb = g.map_b[int64_t(k) * g.nb + j];
    }
    lds[lane] = sa;
    lds[64 + lane] = sb;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // Call before a(t) / b(t) when t may have left the current batch.
  __device__ inline void advance(int64_t t, int lane) {
    if (t - base >= 64) fetch(t, lane);
  }
  __device__ inline int64_t a(int64_t t) const {
    return __builtin_amdgcn_readfirstlane(lds[t - base]);
  }
  __device__ inline int64_t b(int64_t t) const {
    return __builtin_amdgcn_readfirstlane(lds[64 + (t - base)]);
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

// One wave per C block over its leaf task list; slots: the wave's [128]
// LDS table.
__device__ __forceinline__ void f32_block(const GemmArgs& g, int64_t node, int lane,
                                          int32_t* slots) {
  const int32_t ij = uniform(g.nodes[node]);
  const int i = unpack_i(ij), j = unpack_j(ij);
  const float* pa = static_cast<const float*>(g.pool_a);
  const float* pb = static_cast<const float*>(g.pool_b);
  const int64_t t0 = uniform(g.nptr[node]), t1 = uniform(g.nptr[node + 1]);
  v16f acc = {};
  F32Frag cur, nxt;
  TaskSlots ts(g, i, j, t0, t1, slots, lane);
  if (t0 < t1) {
    // Two operand sets in alternation: the next product's loads are always
    // in flight while the current product runs on the MFMA unit.  The loop
    // body has no conditional loads, so the waits stay exact.
    auto fetch = [&](int64_t t, F32Frag& f) {
      ts.advance(t, lane);
      load_f32(pa + ts.a(t) * kLeaf2, pb + ts.b(t) * kLeaf2, lane, f);
    };
    fetch(t0, cur);
    int64_t t = t0;
    for (; t + 2 < t1; t += 2) {
      fetch(t + 1, nxt);
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
      mma_f32(cur, acc);
      __builtin_amdgcn_sched_barrier(0);
      fetch(t + 2, cur);
      __builtin_amdgcn_sched_barrier(0);
      mma_f32(nxt, acc);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (t + 1 < t1) {
      fetch(t + 1, nxt);
      mma_f32(cur, acc);
      mma_f32(nxt, acc);
    } else {
      mma_f32(cur, acc);
    }
  }
  float* out = static_cast<float*>(g.pool_c) + node * kLeaf2;
  const int64_t ms = uniform(mirror_slot(g, node, i, j));
  float* outm = ms >= 0 ? static_cast<float*>(g.pool_c) + ms * kLeaf2 : nullptr;
  const float* xt = nullptr;
  if (g.sp2) {
    const int32_t sx = g.map_x[int64_t(i) * g.nb + j];
    if (sx >= 0) xt = static_cast<const float*>(g.pool_x) + int64_t(sx) * kLeaf2;
  }
  const int col = lane & 31, kk = lane >> 5;
  Epi<float> e;
  v4f m4;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = (r >> 2) * 8 + kk * 4 + (r & 3);
    const float x = xt ? xt[row * kLeaf + col] : 0.0f;
    const float v = e.apply(acc[r], x, g.sp2, g.square, i == j && row == col);
    out[row * kLeaf + col] = v;
    // The mirror's row `col` holds this lane's 4 consecutive rows.
    m4[r & 3] = v;
    if ((r & 3) == 3 && outm)
      *reinterpret_cast<v4f*>(outm + col * kLeaf + (r >> 2) * 8 + kk * 4) = m4;
  }
  e.finish(g, node, ij, lane, ms);
}

__global__ void __launch_bounds__(256) k_leaf_gemm_f32(GemmArgs g) {
  __shared__ int32_t s_slots[kWaves][128];
  const int64_t node = uniform(xcd_contiguous_block() * kWaves + (threadIdx.x >> 6));
  if (node >= g.n_nodes) return;
  f32_block(g, node, threadIdx.x & 63, s_slots[threadIdx.x >> 6]);
}

__global__ void __launch_bounds__(256) k_leaf_gemm_f32_batch(GemmBatch b) {
  __shared__ int32_t s_slots[kWaves][128];
  int64_t node = 0;
  const GemmArgs* g = batch_locate(b, threadIdx.x >> 6, node);
  if (!g) return;
  f32_block(*g, node, threadIdx.x & 63, s_slots[threadIdx.x >> 6]);
}

// ---- FP32 leaf products on 2 x 2 groups of C blocks --------------------------
//
// One workgroup of 4 waves owns the 2 x 2 C blocks (2I + a, 2J + b) below a
// tier-(d-1) node (I, J); wave q = 2a + b owns block q.  Its work is the
// node's ascending K list from the occlusion pass, each entry carrying the
// 8 pass bits of (q, leaf k = 2K + c).  For every leaf k in ascending
// order, the tiles A_{2I+a,k} and B_{k,2J+b} that some owner needs are
// loaded once into LDS (double-buffered; the next k's tiles travel through
// registers while the current k's products run) and each owner whose bit is
// set runs its 16 MFMAs from there, so an A or B tile read from memory feeds
// up to two products.  The accumulation order of every C block is its
// ascending k, exactly as with one wave per block.

constexpr int kBatch = 64;             // list entries staged per batch
constexpr int kSteps = 2 * kBatch;     // leaf steps per batch (c = 0, 1)
constexpr int kAStride = kLeaf + 4;    // padded A rows: conflict-free b128 reads

struct StepTable {
  int32_t mask[kSteps];     // bit q: owner q multiplies at this step
  int32_t slot[kSteps][4];  // A_{2I}, A_{2I+1}, B_{,2J}, B_{,2J+1}; -1 if unused
};

__global__ void __launch_bounds__(256) k_leaf_gemm_f32_2x2(GemmArgs g) {
  __shared__ float s_a[2][2][kLeaf * kAStride];
  __shared__ float s_b[2][2][kLeaf2];
  __shared__ StepTable st;
  __shared__ int32_t s_wcnt[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p = uniform(xcd_contiguous_block());
  if (p >= g.n_super) return;
  const int32_t IJ = uniform(g.sup_nodes[p]);
  const int I = unpack_i(IJ), J = unpack_j(IJ);
  const int a_own = wave >> 1, b_own = wave & 1;
  const float* pa = static_cast<const float*>(g.pool_a);
  const float* pb = static_cast<const float*>(g.pool_b);
  const int64_t e0 = uniform(g.sup_nptr[p]), e1 = uniform(g.sup_nptr[p + 1]);
  // Tile element of this thread while staging: row tid / 8, columns 4 (tid % 8) ..
  const int srow = tid >> 3, scol = (tid & 7) * 4;
  v16f acc = {};
  v4f r0[4], r1[4];
  for (int64_t eb = e0; eb < e1; eb += kBatch) {
    // Step table of this batch: thread x < kSteps takes entry x / 2, c = x % 2.
    int32_t mask = 0, sl[4] = {-1, -1, -1, -1};
    if (tid < kSteps) {
      const int64_t e = eb + (tid >> 1);
      if (e < e1) {
        const int c = tid & 1;
        const int bits = g.sup_bits[e];
        for (int q = 0; q < 4; ++q) mask |= ((bits >> (2 * q + c)) & 1) << q;
        const int k = 2 * g.sup_ks[e] + c;
        if (mask & 0x3) sl[0] = g.map_a[int64_t(2 * I) * g.nb + k];
        if (mask & 0xC) sl[1] = g.map_a[int64_t(2 * I + 1) * g.nb + k];
        if (mask & 0x5) sl[2] = g.map_b[int64_t(k) * g.nb + 2 * J];
        if (mask & 0xA) sl[3] = g.map_b[int64_t(k) * g.nb + 2 * J + 1];
      }
    }
    // Compact away the steps nobody needs (same order).
    const uint64_t live = __ballot(mask != 0);
    if (lane == 0) s_wcnt[wave] = __popcll(live);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += s_wcnt[w];
    const int n_steps = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
    if (mask != 0) {
      const int at = before + __popcll(live & ((uint64_t(1) << lane) - 1));
      st.mask[at] = mask;
      for (int u = 0; u < 4; ++u) st.slot[at][u] = sl[u];
    }
    __syncthreads();
    // Two register sets: the tiles of step x + 2 are requested while step x
    // runs, so each load has two steps to arrive before it is stored to LDS.
    auto stage = [&](int x, v4f (&reg)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t sv = st.slot[x][u];
        if (sv >= 0) {
          const float* src = (u < 2 ? pa : pb) + int64_t(sv) * kLeaf2 + srow * kLeaf + scol;
          reg[u] = *reinterpret_cast<const v4f*>(src);
        }
      }
    };
    auto store = [&](int x, int buf, const v4f (&reg)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (st.slot[x][u] < 0) continue;
        float* dst = u < 2 ? &s_a[buf][u][srow * kAStride + scol] : &s_b[buf][u - 2][srow * kLeaf + scol];
        *reinterpret_cast<v4f*>(dst) = reg[u];
      }
    };
    auto compute = [&](int x, int buf) {
      if ((st.mask[x] >> wave) & 1) {
        const int m = lane & 31, kk = lane >> 5;
        F32Frag f;
        const v4f* ar = reinterpret_cast<const v4f*>(&s_a[buf][a_own][m * kAStride + kk * 16]);
#pragma unroll
        for (int u = 0; u < 4; ++u) f.a[u] = ar[u];
        const float* br = &s_b[buf][b_own][(kk * 16) * kLeaf + m];
#pragma unroll
        for (int u = 0; u < 16; ++u) f.b[u] = br[u * kLeaf];
        mma_f32(f, acc);
      }
    };
    // One step: request step x + 2 into `ahead`, multiply step x from LDS,
    // then move step x + 1 (requested a step earlier, in `next`) to LDS.
    auto step = [&](int x, v4f (&ahead)[4], const v4f (&next)[4]) {
      if (x + 2 < n_steps) stage(x + 2, ahead);
      compute(x, x & 1);
      if (x + 1 < n_steps) store(x + 1, (x + 1) & 1, next);
      __syncthreads();
    };
    if (n_steps > 0) {
      stage(0, r0);
      if (n_steps > 1) stage(1, r1);
      store(0, 0, r0);
      __syncthreads();
    }
    for (int x = 0; x < n_steps; x += 2) {
      step(x, r0, r1);
      if (x + 1 < n_steps) step(x + 1, r1, r0);
    }
  }
  // Epilogue: owner q writes its C block if it exists.
  const int q = wave;
  if (uniform(g.sup_cnt4[4 * p + q]) <= 0) return;
  const int64_t node = uniform(g.sup_noff[4 * p + q]);
  const int i = 2 * I + a_own, j = 2 * J + b_own;
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
  e.finish(g, node, pack_ij(i, j), lane, -1);
}

// ---- FP32 leaf products: one wave per 2 x 2 group, no barriers ---------------
//
// The same 2 x 2 groups and pass bits as k_leaf_gemm_f32_2x2, but one wave
// owns all four C blocks (four accumulators) and loads its operands straight
// into registers: per leaf k the (up to) two A tiles and two B tiles feed up
// to four products, the next k's tiles are in flight while the current k's
// products run, and waves never wait for each other.

struct W2x2Frag {
  v4f a[2][4];
  float b[2][16];
};

__device__ inline void load_w2x2(const float* __restrict__ pa, const float* __restrict__ pb,
                                 const int32_t (&sl)[4], int lane, W2x2Frag& f) {
  const int m = lane & 31, kk = lane >> 5;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (sl[u] >= 0) {
      const v4f* ar = reinterpret_cast<const v4f*>(pa + int64_t(sl[u]) * kLeaf2 + m * kLeaf + kk * 16);
#pragma unroll
      for (int q = 0; q < 4; ++q) f.a[u][q] = ar[q];
    }
    if (sl[2 + u] >= 0) {
      const float* br = pb + int64_t(sl[2 + u]) * kLeaf2 + (kk * 16) * kLeaf + m;
#pragma unroll
      for (int q = 0; q < 16; ++q) f.b[u][q] = br[q * kLeaf];
    }
  }
}

// The same operands from the column-quad copies (colq_index): A_ik as the
// columns of its stored transpose (k, i) (symmetric squares), B_kj as the
// columns of (k, j); every load of the wave reads 1 KiB contiguously.
__device__ inline void load_w2x2_colq(const float* __restrict__ cq, const int32_t (&sl)[4], int lane,
                                      W2x2Frag& f) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (sl[u] >= 0) {
      const v4f* at = reinterpret_cast<const v4f*>(cq + int64_t(sl[u]) * kLeaf2) + lane;
#pragma unroll
      for (int q = 0; q < 4; ++q) f.a[u][q] = at[q * 64];
    }
    if (sl[2 + u] >= 0) {
      const v4f* bt = reinterpret_cast<const v4f*>(cq + int64_t(sl[2 + u]) * kLeaf2) + lane;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const v4f v = bt[q * 64];
#pragma unroll
        for (int e = 0; e < 4; ++e) f.b[u][4 * q + e] = v[e];
      }
    }
  }
}

__device__ inline void mma_pair(const v4f (&a)[4], const float (&b)[16], v16f& acc) {
#pragma unroll
  for (int s = 0; s < 16; ++s)
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s >> 2][s & 3], b[s], acc, 0, 0, 0);
}

__device__ inline void mma_w2x2(const W2x2Frag& f, int mask, v16f (&acc)[4]) {
  if (mask & 1) mma_pair(f.a[0], f.b[0], acc[0]);
  if (mask & 2) mma_pair(f.a[0], f.b[1], acc[1]);
  if (mask & 4) mma_pair(f.a[1], f.b[0], acc[2]);
  if (mask & 8) mma_pair(f.a[1], f.b[1], acc[3]);
}

constexpr int kWBatch = 32;            // list entries per slot batch (64 steps)

// kAhead: operand sets in flight per wave (2: the next step's loads overlap
// the current step's products; 1: other waves hide the latency).
// Group p of g; tab: the wave's LDS step table (mask, 4 slots per step).
// kColq: operands from the column-quad copy (1), the row-major pools (0),
// or as g.colq_a says (2, batched launches of mixed products).
// stage (kColq != 0): the wave's LDS tile, through which each mirror is
// written transposed with coalesced stores.
constexpr int kStagePitch = 33;
template <int kAhead, int kColq>
__device__ __forceinline__ void f32_w2x2(const GemmArgs& g, int64_t p, int lane,
                                         int32_t (*tab)[2 * kWBatch], float* stage) {
  const int32_t IJ = uniform(g.sup_nodes[p]);
  const int I = unpack_i(IJ), J = unpack_j(IJ);
  const float* pa = static_cast<const float*>(g.pool_a);
  const float* pb = static_cast<const float*>(g.pool_b);
  const float* cq = kColq == 0 ? nullptr : static_cast<const float*>(g.colq_a);
  const int64_t e0 = uniform(g.sup_nptr[p]), e1 = uniform(g.sup_nptr[p + 1]);
  v16f acc[4] = {};
  W2x2Frag cur, nxt;
  // Operands from the row-major pools or from the column-quad copy.
  auto load = [&](const int32_t (&sl)[4], W2x2Frag& f) {
    if (kColq == 1 || (kColq == 2 && cq))
      load_w2x2_colq(cq, sl, lane, f);
    else
      load_w2x2(pa, pb, sl, lane, f);
  };
  for (int64_t eb = e0; eb < e1; eb += kWBatch) {
    // Steps of this batch: lane l takes entry l / 2, c = l % 2.
    int32_t mask = 0, sl[4] = {-1, -1, -1, -1};
    const int64_t e = eb + (lane >> 1);
    if (e < e1) {
      const int c = lane & 1;
      const int bits = g.sup_bits[e];
      for (int q = 0; q < 4; ++q) mask |= ((bits >> (2 * q + c)) & 1) << q;
      const int k = 2 * g.sup_ks[e] + c;
      // Column-quad operands: A_ik as its transpose, the stored block (k, i).
      if (mask & 0x3)
        sl[0] = cq ? g.map_a[int64_t(k) * g.nb + 2 * I] : g.map_a[int64_t(2 * I) * g.nb + k];
      if (mask & 0xC)
        sl[1] = cq ? g.map_a[int64_t(k) * g.nb + 2 * I + 1] : g.map_a[int64_t(2 * I + 1) * g.nb + k];
      if (mask & 0x5) sl[2] = g.map_b[int64_t(k) * g.nb + 2 * J];
      if (mask & 0xA) sl[3] = g.map_b[int64_t(k) * g.nb + 2 * J + 1];
    }
    const uint64_t live = __ballot(mask != 0);
    const int n_steps = __popcll(live);
    if (mask != 0) {
      const int at = __popcll(live & ((uint64_t(1) << lane) - 1));
      tab[0][at] = mask;
#pragma unroll
      for (int u = 0; u < 4; ++u) tab[1 + u][at] = sl[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    auto slots = [&](int x, int32_t (&out)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) out[u] = __builtin_amdgcn_readfirstlane(tab[1 + u][x]);
    };
    auto step_mask = [&](int x) { return __builtin_amdgcn_readfirstlane(tab[0][x]); };
    if (kAhead == 1) {
      for (int x = 0; x < n_steps; ++x) {
        int32_t s0[4];
        slots(x, s0);
        load(s0, cur);
        mma_w2x2(cur, step_mask(x), acc);
      }
    } else if (n_steps > 0) {
      int32_t s0[4];
      slots(0, s0);
      load(s0, cur);
      int x = 0;
      for (; x + 2 < n_steps; x += 2) {
        int32_t s1[4], s2[4];
        slots(x + 1, s1);
        load(s1, nxt);
        __builtin_amdgcn_sched_barrier(0);
        mma_w2x2(cur, step_mask(x), acc);
        __builtin_amdgcn_sched_barrier(0);
        slots(x + 2, s2);
        load(s2, cur);
        __builtin_amdgcn_sched_barrier(0);
        mma_w2x2(nxt, step_mask(x + 1), acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (x + 1 < n_steps) {
        int32_t s1[4];
        slots(x + 1, s1);
        load(s1, nxt);
        __builtin_amdgcn_sched_barrier(0);
        mma_w2x2(cur, step_mask(x), acc);
        mma_w2x2(nxt, step_mask(x + 1), acc);
      } else {
        mma_w2x2(cur, step_mask(x), acc);
      }
    }
    // The table is rewritten by the next batch only after every lane's reads.
    __builtin_amdgcn_wave_barrier();
  }
  const int col = lane & 31, kk = lane >> 5;
  auto emit = [&](int q, const v16f& a) {
    if (uniform(g.sup_cnt4[4 * p + q]) <= 0) return;
    const int64_t node = uniform(g.sup_noff[4 * p + q]);
    const int i = 2 * I + (q >> 1), j = 2 * J + (q & 1);
    float* out = static_cast<float*>(g.pool_c) + node * kLeaf2;
    const int64_t ms = uniform(mirror_slot(g, node, i, j));
    float* outm = ms >= 0 ? static_cast<float*>(g.pool_c) + ms * kLeaf2 : nullptr;
    const float* xt = nullptr;
    if (g.sp2) {
      const int32_t sx = g.map_x[int64_t(i) * g.nb + j];
      if (sx >= 0) xt = static_cast<const float*>(g.pool_x) + int64_t(sx) * kLeaf2;
    }
    // Column-quad copies of the block and of its mirror; with them the
    // mirror goes through the LDS tile.
    float* oq = kColq != 0 && g.colq_c ? static_cast<float*>(g.colq_c) + node * kLeaf2 : nullptr;
    float* omq = oq && ms >= 0 ? static_cast<float*>(g.colq_c) + ms * kLeaf2 : nullptr;
    Epi<float> e;
    v4f m4;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (r >> 2) * 8 + kk * 4 + (r & 3);
      const float x = xt ? xt[row * kLeaf + col] : 0.0f;
      const float v = e.apply(a[r], x, g.sp2, g.square, i == j && row == col);
      out[row * kLeaf + col] = v;
      if (omq) stage[row * kStagePitch + col] = v;
      // The mirror's row `col` holds this lane's 4 consecutive rows, and so
      // does the block's own column-quad copy.
      m4[r & 3] = v;
      if ((r & 3) == 3) {
        if (outm && !omq)
          *reinterpret_cast<v4f*>(outm + col * kLeaf + (r >> 2) * 8 + kk * 4) = m4;
        if (oq) *reinterpret_cast<v4f*>(oq + colq_index(row - 3, col)) = m4;
      }
    }
    if (omq) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // Mirror M = C^T: row 2t + kk of M is column 2t + kk of C; its
      // column-quad load q of lane (kk, c) holds C(c, 16 kk + 4 q .. + 3).
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int rm = 2 * t + kk;
        outm[rm * kLeaf + col] = stage[col * kStagePitch + rm];
      }
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        v4f w;
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = stage[col * kStagePitch + 16 * kk + 4 * q4 + u];
        *reinterpret_cast<v4f*>(omq + (q4 * 64 + lane) * 4) = w;
      }
      // Every lane's reads precede the next block's writes.
      __builtin_amdgcn_wave_barrier();
    }
    e.finish(g, node, pack_ij(i, j), lane, ms);
  };
  emit(0, acc[0]);
  emit(1, acc[1]);
  emit(2, acc[2]);
  emit(3, acc[3]);
}

// kW: waves (2 x 2 groups) per workgroup.
template <int kAhead, int kW, int kColq>
__global__ void __launch_bounds__(64 * kW) k_leaf_gemm_f32_w2x2(GemmArgs g) {
  __shared__ int32_t s_tab[kW][5][2 * kWBatch];
  __shared__ float s_stage[kW][kColq != 0 ? kLeaf * kStagePitch : 1];
  const int wave = threadIdx.x >> 6;
  const int64_t p = uniform(xcd_contiguous_block() * kW + wave);
  if (p >= g.n_super) return;
  f32_w2x2<kAhead, kColq>(g, p, threadIdx.x & 63, s_tab[wave], s_stage[wave]);
}

template <int kAhead, int kW>
__global__ void __launch_bounds__(64 * kW) k_leaf_gemm_f32_w2x2_batch(GemmBatch b) {
  __shared__ int32_t s_tab[kW][5][2 * kWBatch];
  __shared__ float s_stage[kW][kLeaf * kStagePitch];
  const int wave = threadIdx.x >> 6;
  int64_t p = 0;
  const GemmArgs* g = batch_locate(b, wave, p);
  if (!g) return;
  f32_w2x2<kAhead, 2>(*g, p, threadIdx.x & 63, s_tab[wave], s_stage[wave]);
}

// ---- FP32 leaf products on 4 x 4 groups of C blocks --------------------------
//
// One workgroup of 4 waves owns the 4 x 4 C blocks (4I + a, 4J + b) below a
// tier-(d-2) node (I, J); wave a owns row a, four accumulators.  Its work
// is the node's ascending K list, each entry carrying the 64 pass bits of
// its leaf products (bit 16c + 4a + b, leaf k = 4K + c).  For every leaf k
// in ascending order, the A tiles A_{4I+a,k} and B tiles B_{k,4J+b} that
// some owner needs are loaded once into LDS, double-buffered, with the
// tiles of step x + 2 requested while step x runs.  Each wave reads its A
// tile once per step and multiplies it with the B tiles of its set bits:
// a tile read from memory feeds up to four products, a quarter of the
// operand traffic of one wave per C block.  Every C block still
// accumulates over its own k in ascending order.

constexpr int kQBatch = 32;            // list entries staged per batch
constexpr int kQSteps = 4 * kQBatch;   // leaf steps per batch (c = 0..3)

struct QuadTable {
  int32_t mask[kQSteps];     // bit 4a + b: block (a, b) multiplies at this step
  int32_t slot[kQSteps][8];  // A rows 0..3, B columns 0..3; -1 if unused
};

__global__ void __launch_bounds__(256) k_leaf_gemm_f32_4x4(GemmArgs g) {
  __shared__ float s_a[2][4][kLeaf * kAStride];
  __shared__ float s_b[2][4][kLeaf2];
  __shared__ QuadTable st;
  __shared__ int32_t s_wcnt[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p = uniform(xcd_contiguous_block());
  if (p >= g.n_quad) return;
  const int32_t IJ = uniform(g.quad_nodes[p]);
  const int I = unpack_i(IJ), J = unpack_j(IJ);
  const float* pa = static_cast<const float*>(g.pool_a);
  const float* pb = static_cast<const float*>(g.pool_b);
  const int64_t e0 = uniform(g.quad_nptr[p]), e1 = uniform(g.quad_nptr[p + 1]);
  const int srow = tid >> 3, scol = (tid & 7) * 4;
  v16f acc0 = {}, acc1 = {}, acc2 = {}, acc3 = {};
  v4f r0[8], r1[8];
  for (int64_t eb = e0; eb < e1; eb += kQBatch) {
    // Step table: thread x < kQSteps takes entry x / 4, c = x % 4.
    int32_t mask = 0, sl[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sl[u] = -1;
    if (tid < kQSteps) {
      const int64_t e = eb + (tid >> 2);
      if (e < e1) {
        const int c = tid & 3;
        mask = int32_t((g.quad_masks[e] >> (16 * c)) & 0xffff);
        const int k = 4 * g.quad_ks[e] + c;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if ((mask >> (4 * u)) & 0xF) sl[u] = g.map_a[int64_t(4 * I + u) * g.nb + k];
          if (mask & (0x1111 << u)) sl[4 + u] = g.map_b[int64_t(k) * g.nb + 4 * J + u];
        }
      }
    }
    const uint64_t live = __ballot(mask != 0);
    if (lane == 0 && wave < 2) s_wcnt[wave] = __popcll(live);
    __syncthreads();
    const int n_steps = s_wcnt[0] + s_wcnt[1];
    if (mask != 0) {
      const int at = (wave == 1 ? s_wcnt[0] : 0) + __popcll(live & ((uint64_t(1) << lane) - 1));
      st.mask[at] = mask;
#pragma unroll
      for (int u = 0; u < 8; ++u) st.slot[at][u] = sl[u];
    }
    __syncthreads();
    auto stage = [&](int x, v4f (&reg)[8]) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int32_t sv = st.slot[x][u];
        if (sv >= 0) {
          const float* src = (u < 4 ? pa : pb) + int64_t(sv) * kLeaf2 + srow * kLeaf + scol;
          reg[u] = *reinterpret_cast<const v4f*>(src);
        }
      }
    };
    auto store = [&](int x, int buf, const v4f (&reg)[8]) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (st.slot[x][u] < 0) continue;
        float* dst = u < 4 ? &s_a[buf][u][srow * kAStride + scol]
                           : &s_b[buf][u - 4][srow * kLeaf + scol];
        *reinterpret_cast<v4f*>(dst) = reg[u];
      }
    };
    auto compute = [&](int x, int buf) {
      const int row = (st.mask[x] >> (4 * wave)) & 0xF;
      if (row == 0) return;
      const int m = lane & 31, kk = lane >> 5;
      F32Frag f;
      const v4f* ar = reinterpret_cast<const v4f*>(&s_a[buf][wave][m * kAStride + kk * 16]);
#pragma unroll
      for (int u = 0; u < 4; ++u) f.a[u] = ar[u];
      auto col = [&](int b, v16f& acc) {
        const float* br = &s_b[buf][b][(kk * 16) * kLeaf + m];
#pragma unroll
        for (int u = 0; u < 16; ++u) f.b[u] = br[u * kLeaf];
        mma_f32(f, acc);
      };
      if (row & 1) col(0, acc0);
      if (row & 2) col(1, acc1);
      if (row & 4) col(2, acc2);
      if (row & 8) col(3, acc3);
    };
    auto step = [&](int x, v4f (&ahead)[8], const v4f (&next)[8]) {
      if (x + 2 < n_steps) stage(x + 2, ahead);
      compute(x, x & 1);
      if (x + 1 < n_steps) store(x + 1, (x + 1) & 1, next);
      __syncthreads();
    };
    if (n_steps > 0) {
      stage(0, r0);
      if (n_steps > 1) stage(1, r1);
      store(0, 0, r0);
      __syncthreads();
    }
    for (int x = 0; x < n_steps; x += 2) {
      step(x, r0, r1);
      if (x + 1 < n_steps) step(x + 1, r1, r0);
    }
  }
  // Epilogue: wave a writes the blocks of its row that exist in C.
  const int i = 4 * I + wave;
  const int col = lane & 31, kk = lane >> 5;
  auto emit = [&](int b, const v16f& acc) {
    const int j = 4 * J + b;
    const int32_t node = uniform(g.map_c[int64_t(i) * g.nb + j]);
    if (node < 0) return;
    float* out = static_cast<float*>(g.pool_c) + int64_t(node) * kLeaf2;
    const float* xt = nullptr;
    if (g.sp2) {
      const int32_t sx = g.map_x[int64_t(i) * g.nb + j];
      if (sx >= 0) xt = static_cast<const float*>(g.pool_x) + int64_t(sx) * kLeaf2;
    }
    Epi<float> e;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int rr = (r >> 2) * 8 + kk * 4 + (r & 3);
      const float x = xt ? xt[rr * kLeaf + col] : 0.0f;
      out[rr * kLeaf + col] = e.apply(acc[r], x, g.sp2, g.square, i == j && rr == col);
    }
    e.finish(g, node, pack_ij(i, j), lane, -1);
  };
  emit(0, acc0);
  emit(1, acc1);
  emit(2, acc2);
  emit(3, acc3);
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

__device__ __forceinline__ void f64_block(const GemmArgs& g, int64_t node, int lane,
                                          int32_t* slots) {
  const int32_t ij = uniform(g.nodes[node]);
  const int i = unpack_i(ij), j = unpack_j(ij);
  const double* pa = static_cast<const double*>(g.pool_a);
  const double* pb = static_cast<const double*>(g.pool_b);
  const int64_t t0 = uniform(g.nptr[node]), t1 = uniform(g.nptr[node + 1]);
  v4d acc[2][2] = {};
  F64Frag cur, nxt;
  TaskSlots ts(g, i, j, t0, t1, slots, lane);
  if (t0 < t1) {
    // Two operand sets in alternation: the next product's loads are always
    // in flight while the current product runs on the MFMA unit.  The loop
    // body has no conditional loads, so the waits stay exact.
    auto fetch = [&](int64_t t, F64Frag& f) {
      ts.advance(t, lane);
      load_f64(pa + ts.a(t) * kLeaf2, pb + ts.b(t) * kLeaf2, lane, f);
    };
    fetch(t0, cur);
    int64_t t = t0;
    for (; t + 2 < t1; t += 2) {
      fetch(t + 1, nxt);
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
      mma_f64(cur, acc);
      __builtin_amdgcn_sched_barrier(0);
      fetch(t + 2, cur);
      __builtin_amdgcn_sched_barrier(0);
      mma_f64(nxt, acc);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (t + 1 < t1) {
      fetch(t + 1, nxt);
      mma_f64(cur, acc);
      mma_f64(nxt, acc);
    } else {
      mma_f64(cur, acc);
    }
  }
  double* out = static_cast<double*>(g.pool_c) + node * kLeaf2;
  const int64_t ms = uniform(mirror_slot(g, node, i, j));
  double* outm = ms >= 0 ? static_cast<double*>(g.pool_c) + ms * kLeaf2 : nullptr;
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
        const double v = e.apply(acc[p][q][r], x, g.sp2, g.square, i == j && row == col);
        out[row * kLeaf + col] = v;
        if (outm) outm[col * kLeaf + row] = v;
      }
  e.finish(g, node, ij, lane, ms);
}

__global__ void __launch_bounds__(256) k_leaf_gemm_f64(GemmArgs g) {
  __shared__ int32_t s_slots[kWaves][128];
  const int64_t node = uniform(xcd_contiguous_block() * kWaves + (threadIdx.x >> 6));
  if (node >= g.n_nodes) return;
  f64_block(g, node, threadIdx.x & 63, s_slots[threadIdx.x >> 6]);
}

__global__ void __launch_bounds__(256) k_leaf_gemm_f64_batch(GemmBatch b) {
  __shared__ int32_t s_slots[kWaves][128];
  int64_t node = 0;
  const GemmArgs* g = batch_locate(b, threadIdx.x >> 6, node);
  if (!g) return;
  f64_block(*g, node, threadIdx.x & 63, s_slots[threadIdx.x >> 6]);
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
  if (lane == 0)
    slot = r.base_slot + atomicAdd(reinterpret_cast<unsigned long long*>(r.counter), 1ull);
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
  // 2 X_n elementwise: the column-quad copy from X_n's, position by position.
  if (r.colq_out) {
    const T* xq = static_cast<const T*>(r.colq_x) + s * kLeaf2;
    T* oq = static_cast<T*>(r.colq_out) + slot * kLeaf2;
#pragma unroll
    for (int q = 0; q < 16; ++q) oq[q * 64 + lane] = T(2) * xq[q * 64 + lane];
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

// Column-quad copies of row-major FP32 tiles: one wave per tile, each lane
// writing 16 consecutive floats of the copy.
__global__ void __launch_bounds__(256) k_tiles_to_colq(const float* __restrict__ pool, int64_t n,
                                                       float* __restrict__ colq) {
  const int lane = threadIdx.x & 63;
  const int64_t t = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  if (t >= n) return;
  const float* src = pool + t * kLeaf2;
  float* dst = colq + t * kLeaf2;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int x = q * 64 + lane;  // position in the copy
    const int quad = x >> 2, e = x & 3;
    const int c = quad & 31, r = ((quad >> 6) << 2) + (((quad >> 5) & 1) << 4) + e;
    dst[x] = src[r * kLeaf + c];
  }
}

// Clears the per-iteration SP2 arrays in one launch.
__global__ void k_sp2_prepare(int32_t* __restrict__ map, double* __restrict__ norm_leaf,
                              double* __restrict__ err_part, int64_t cells,
                              double* __restrict__ trace_part, int nb, int64_t* counter) {
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < cells;
       x += int64_t(gridDim.x) * blockDim.x) {
    map[x] = -1;
    norm_leaf[x] = 0.0;
    err_part[x] = 0.0;
    if (x < nb) trace_part[x] = 0.0;
    if (x == 0) {
      counter[0] = 0;  // blocks carried over by the 2X - X^2 branch
      counter[1] = 0;  // FP16 overflow flag
    }
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

// Leaf-product kernel: SPAMM_LEAF_KERNEL = block | 2x2 | 4x4 | w2x2 | w2x2s
// picks one (all compute the same result, in the same order); unset or
// unknown picks the default.
int leaf_kernel_choice() {
  const char* v = std::getenv("SPAMM_LEAF_KERNEL");
  if (v == nullptr) return kLeafDefault;
  if (std::strcmp(v, "w2x2") == 0) return kLeafW2x2;
  if (std::strcmp(v, "w2x2s") == 0) return kLeafW2x2s;
  if (std::strcmp(v, "block") == 0) return kLeafBlock;
  if (std::strcmp(v, "2x2") == 0) return kLeaf2x2;
  if (std::strcmp(v, "4x4") == 0) return kLeaf4x4;
  return kLeafDefault;
}

// Waves (2 x 2 groups) per workgroup of the 2 x 2 kernels for a launch of
// `groups` groups (SPAMM_LEAF_WAVES = 1, 2 or 4 overrides).  Measured: with
// a few thousand groups (150 molecules: 3,481) one wave per workgroup is
// fastest, since a workgroup's CU slot is freed when its own group is done
// rather than when the slowest of four is (+4%); with 10^5 groups (1000
// molecules: 152,881) four neighbouring groups per workgroup share the CU's
// L1 and are faster (+4% FP32, +7% split FP16).
int w2x2_waves(int64_t groups) {
  const char* v = std::getenv("SPAMM_LEAF_WAVES");
  if (v && std::strcmp(v, "1") == 0) return 1;
  if (v && std::strcmp(v, "2") == 0) return 2;
  if (v && std::strcmp(v, "4") == 0) return 4;
  return groups >= kManyGroups ? 4 : 1;
}

template <int kAhead, int kColq>
static void launch_w2x2_c(int waves, const GemmArgs& g, hipStream_t s) {
  const unsigned grid = unsigned((g.n_super + waves - 1) / waves);
  if (waves == 1)
    k_leaf_gemm_f32_w2x2<kAhead, 1, kColq><<<grid, 64, 0, s>>>(g);
  else if (waves == 2)
    k_leaf_gemm_f32_w2x2<kAhead, 2, kColq><<<grid, 128, 0, s>>>(g);
  else
    k_leaf_gemm_f32_w2x2<kAhead, 4, kColq><<<grid, 256, 0, s>>>(g);
}

template <int kAhead>
static void launch_w2x2_a(int waves, const GemmArgs& g, hipStream_t s) {
  if (g.colq_a)
    launch_w2x2_c<kAhead, 1>(waves, g, s);
  else
    launch_w2x2_c<kAhead, 0>(waves, g, s);
}

static void launch_w2x2(int ahead, int waves, const GemmArgs& g, hipStream_t s) {
  if (ahead == 2)
    launch_w2x2_a<2>(waves, g, s);
  else
    launch_w2x2_a<1>(waves, g, s);
}

template <int kAhead>
static void launch_w2x2_batch_a(int waves, const GemmBatch& b, hipStream_t s) {
  const unsigned grid = unsigned(b.first[b.n]);
  if (waves == 1)
    k_leaf_gemm_f32_w2x2_batch<kAhead, 1><<<grid, 64, 0, s>>>(b);
  else if (waves == 2)
    k_leaf_gemm_f32_w2x2_batch<kAhead, 2><<<grid, 128, 0, s>>>(b);
  else
    k_leaf_gemm_f32_w2x2_batch<kAhead, 4><<<grid, 256, 0, s>>>(b);
}

void launch_leaf_gemm(int prec, const GemmArgs& g, hipStream_t s) {
  if (g.n_nodes <= 0) return;
  if (prec != SPAMM_FP64 && prec != SPAMM_FP32) {
    launch_leaf_gemm_half(prec, g, s);
    return;
  }
  const int choice = leaf_kernel_choice();
  if (prec == SPAMM_FP32 && g.n_quad > 0 && choice == kLeaf4x4) {
    k_leaf_gemm_f32_4x4<<<unsigned(g.n_quad), 256, 0, s>>>(g);
    return;
  }
  if (prec == SPAMM_FP32 && g.n_super > 0 && (choice == kLeafW2x2 || choice == kLeafW2x2s)) {
    launch_w2x2(choice == kLeafW2x2 ? 2 : 1, w2x2_waves(g.n_super), g, s);
    return;
  }
  if (prec == SPAMM_FP32 && g.n_super > 0 && (choice == kLeaf2x2 || choice == kLeaf4x4)) {
    k_leaf_gemm_f32_2x2<<<unsigned(g.n_super), 256, 0, s>>>(g);
    return;
  }
  const unsigned grid = unsigned((g.n_nodes + kWaves - 1) / kWaves);
  if (prec == SPAMM_FP64)
    k_leaf_gemm_f64<<<grid, 64 * kWaves, 0, s>>>(g);
  else
    k_leaf_gemm_f32<<<grid, 64 * kWaves, 0, s>>>(g);
}

void launch_leaf_gemm_batch(int prec, const GemmArgs* host, const GemmArgs* dev, int n,
                            hipStream_t s) {
  if (prec != SPAMM_FP64 && prec != SPAMM_FP32) {
    launch_leaf_gemm_half_batch(prec, host, dev, n, s);
    return;
  }
  const int choice = leaf_kernel_choice();
  const bool grouped = prec == SPAMM_FP32 && (choice == kLeafW2x2 || choice == kLeafW2x2s);
  if (prec == SPAMM_FP32 && !grouped && choice != kLeafBlock) {
    for (int r = 0; r < n; ++r) launch_leaf_gemm(prec, host[r], s);
    return;
  }
  auto grid = [](const GemmBatch& b) { return unsigned(b.first[b.n]); };
  // 2 x 2 groups (FP32 with a tier d-1 frontier).
  if (grouped) {
    int64_t groups = 0;
    for (int r = 0; r < n; ++r) groups += host[r].n_nodes > 0 ? host[r].n_super : 0;
    const int waves = w2x2_waves(groups);
    for_each_batch(dev, n, waves, [&](int r) { return host[r].n_nodes > 0 ? host[r].n_super : 0; },
                   [&](const GemmBatch& b) {
                     if (choice == kLeafW2x2)
                       launch_w2x2_batch_a<2>(waves, b, s);
                     else
                       launch_w2x2_batch_a<1>(waves, b, s);
                   });
  }
  // One wave per C block: FP64, FP32 trees of one tier, FP32 "block".
  for_each_batch(dev, n, kWaves,
                 [&](int r) { return grouped && host[r].n_super > 0 ? 0 : host[r].n_nodes; },
                 [&](const GemmBatch& b) {
                   if (prec == SPAMM_FP64)
                     k_leaf_gemm_f64_batch<<<grid(b), 256, 0, s>>>(b);
                   else
                     k_leaf_gemm_f32_batch<<<grid(b), 256, 0, s>>>(b);
                 });
}

void launch_sp2_rest(int prec, const RestArgs& r, hipStream_t s) {
  if (r.n_x <= 0) return;
  if (prec != SPAMM_FP64 && prec != SPAMM_FP32) {
    launch_sp2_rest_half(prec, r, s);
    return;
  }
  const unsigned grid = unsigned((r.n_x + kWaves - 1) / kWaves);
  if (prec == SPAMM_FP64)
    k_sp2_rest<double><<<grid, 64 * kWaves, 0, s>>>(r);
  else
    k_sp2_rest<float><<<grid, 64 * kWaves, 0, s>>>(r);
}

void launch_tiles_to_colq(const void* pool, int64_t n, void* colq, hipStream_t s) {
  if (n <= 0) return;
  k_tiles_to_colq<<<unsigned((n + kWaves - 1) / kWaves), 64 * kWaves, 0, s>>>(
      static_cast<const float*>(pool), n, static_cast<float*>(colq));
}

void launch_sp2_prepare(int32_t* map, double* norm_leaf, double* err_part, int nb,
                        double* trace_part, int64_t* counter, hipStream_t s) {
  const int64_t cells = int64_t(nb) * nb;
  const unsigned g = unsigned(std::min<int64_t>((cells + 255) / 256, 4096));
  k_sp2_prepare<<<g, 256, 0, s>>>(map, norm_leaf, err_part, cells, trace_part, nb, counter);
}

void launch_sp2_reduce(int nb, const double* trace_part, const double* err_part,
                       const double* norm_leaf, Control* ctl, hipStream_t s) {
  k_sp2_reduce<<<1, 1024, 0, s>>>(nb, trace_part, err_part, norm_leaf, ctl);
}

}  // namespace spamm
