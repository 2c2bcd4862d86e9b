// Leaf products of the 16-bit forms (BF16, FP16 and their split hi + lo
// variants) on the MFMA units, with FP32 accumulation and the SP2 update
// fused into the epilogue.  Tile formats are described in half.h.
//
// v_mfma_f32_32x32x16_{bf16,f16}: lane l supplies 8 consecutive k of row
// l % 32 of A (and of column l % 32 of B); two instructions cover the 32 k
// of a leaf product.  Step s of lane half kk takes k = 16 kk + 8 s .. + 7,
// so a lane's A operands are the 32 contiguous bytes of row m from k = 16 kk
// (part 0 / 2 of the tile) and its B operands the same run of row n of the
// transposed tile (part 1 / 3).  The output layout is that of the FP32
// 32x32 instructions.  The split forms add hi*lo + lo*hi into a second
// accumulator, scaled by 2^-L once at the end.
//
// Ownership and order are those of the FP32 kernels: one wave per 2 x 2
// group of C blocks (or one per C block when the tree has one tier), each C
// block accumulated over its own k in ascending order.
#include <cstdlib>
#include <cstring>

#include "device_util.h"
#include "half.h"
#include "internal.h"

namespace spamm {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;
constexpr int kWBatch = 32;  // list entries per slot batch (64 steps)

template <int P>
struct HFrag {
  typedef typename Half<P>::V V;
  V hi[2];
  V lo[2];  // split forms only
};

template <int P>
__device__ inline void load_frag(const typename Half<P>::T* tile, int part, int lane, HFrag<P>& f) {
  typedef typename Half<P>::V V;
  // Chunk 64 s + lane of the part (half_idx).
  const V* p = reinterpret_cast<const V*>(tile + half_part(part)) + lane;
  f.hi[0] = p[0];
  f.hi[1] = p[64];
  if (is_split(P)) {
    const V* q = reinterpret_cast<const V*>(tile + half_part(part + 2)) + lane;
    f.lo[0] = q[0];
    f.lo[1] = q[64];
  }
}

template <int P>
__device__ inline v16f mfma16(typename Half<P>::V a, typename Half<P>::V b, v16f c) {
  if constexpr (is_bf16(P))
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// acc.hh += A_hi B_hi; acc.x += A_hi B_lo + A_lo B_hi (split forms only).
template <int P, bool kSplit = is_split(P)>
struct HAcc {
  v16f hh = {};
  v16f x = {};
  __device__ inline void add(const HFrag<P>& a, const HFrag<P>& b) {
#pragma unroll
    for (int s = 0; s < 2; ++s) hh = mfma16<P>(a.hi[s], b.hi[s], hh);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      x = mfma16<P>(a.hi[s], b.lo[s], x);
      x = mfma16<P>(a.lo[s], b.hi[s], x);
    }
  }
  __device__ inline float value(int r) const { return hh[r] + x[r] * (1.0f / lo_scale(P)); }
};
template <int P>
struct HAcc<P, false> {
  v16f hh = {};
  __device__ inline void add(const HFrag<P>& a, const HFrag<P>& b) {
#pragma unroll
    for (int s = 0; s < 2; ++s) hh = mfma16<P>(a.hi[s], b.hi[s], hh);
  }
  __device__ inline float value(int r) const { return hh[r]; }
};

// Epilogue: value c of C block (i, j) -> stored tile (hi, lo and their
// transposes), SP2 update, FP64 norm, trace and ||C - X_n||^2 partials.
constexpr int kSymPitch = kLeaf + 1;  // padded rows of the diagonal-block transpose

// 16-bit staging rows (80 bytes: 16-byte aligned, and the row segments of
// 8 consecutive lanes fall in distinct banks).
constexpr int kStgPitch = 40;
template <int P>
__host__ __device__ constexpr int stg_elems() {
  return is_split(P) ? 2 * kLeaf * kStgPitch : 1;
}

// sym_lds: the wave's kLeaf * kSymPitch floats, used by the split forms for
// diagonal blocks of symmetric products.  stg: the wave's stg_elems<P>()
// 16-bit values, through which the split forms store the block: each lane
// writes its values row-major, then reads back and stores whole 16-byte
// chunks of the operand-order parts (1 KiB per wave and store).  Measured
// at 150 molecules: split forms +6%, plain forms -3% (they store directly).
template <int P>
__device__ __forceinline__ void epilogue(const GemmArgs& g, int64_t node, int i, int j, const HAcc<P>& acc,
                                int lane, float* sym_lds, typename Half<P>::T* stg) {
  typedef typename Half<P>::T T;
  const int stride = (is_split(P) ? 4 : 2) * kLeaf2;
  T* out = static_cast<T*>(g.pool_c) + node * stride;
  // Symmetric products: the mirror (j, i) is the transpose, i.e. the same
  // parts with the row-major and transposed roles swapped.
  const int64_t ms = uniform(mirror_slot(g, node, i, j));
  T* outm = ms >= 0 ? static_cast<T*>(g.pool_c) + ms * stride : nullptr;
  const T* xt = nullptr;
  if (g.sp2) {
    const int32_t sx = g.map_x[int64_t(i) * g.nb + j];
    if (sx >= 0) xt = static_cast<const T*>(g.pool_x) + int64_t(sx) * stride;
  }
  const int col = lane & 31, kk = lane >> 5;
  double nrm = 0.0, err = 0.0, tr = 0.0;
  bool over = false;
  float cv[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) cv[r] = acc.value(r);
  if (is_split(P) && g.sym && i == j) {
    // A diagonal block of a symmetric product is symmetric, but the split
    // forms add hi_a lo_b and lo_a hi_b in opposite orders for (a, b) and
    // (b, a); the mean of the two is exactly symmetric.
#pragma unroll
    for (int r = 0; r < 16; ++r) sym_lds[((r >> 2) * 8 + kk * 4 + (r & 3)) * kSymPitch + col] = cv[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < 16; ++r)
      cv[r] = 0.5f * (cv[r] + sym_lds[col * kSymPitch + (r >> 2) * 8 + kk * 4 + (r & 3)]);
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = (r >> 2) * 8 + kk * 4 + (r & 3);
    const float c = cv[r];
    float v = c;
    if (g.sp2) {
      const float x =
          xt ? decode_half_f<P>(xt[half_idx(row, col)],
                                is_split(P) ? xt[half_part(2) + half_idx(row, col)] : T(0.0f))
             : 0.0f;
      v = g.square ? c : 2.0f * x - c;
      const double d = double(c) - double(x);
      err += d * d;
    }
    over |= !(fabsf(v) <= float(half_max(P)));
    T hi, lo;
    encode_half_f<P>(v, hi, lo);
    if constexpr (is_split(P)) {
      stg[row * kStgPitch + col] = hi;
      stg[kLeaf * kStgPitch + row * kStgPitch + col] = lo;
    } else {
      // Plain forms: direct 2-byte stores measured faster than staging.
      const int rc = half_idx(row, col), cr = half_idx(col, row);
      out[rc] = hi;
      out[half_part(1) + cr] = hi;
      if (outm) {
        outm[cr] = hi;
        outm[half_part(1) + rc] = hi;
      }
    }
    const double stored = double(decode_half_f<P>(hi, lo));
    nrm += stored * stored;
    if (i == j && row == col) tr += stored;
  }
  if constexpr (is_split(P)) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Chunk 64 s + lane of a part holds, for lane (kk, m), elements
    // c0 .. c0 + 7 (c0 = 16 kk + 8 s) of row m of its matrix (half_idx):
    // row m of the block for the direct parts, column m for the transposed
    // ones.  The mirror is the transpose: the same chunks, roles swapped.
    typedef typename Half<P>::V V;
    const int m = col;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const T* st = stg + h * kLeaf * kStgPitch;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int c0 = 16 * kk + 8 * s;
        const V a = *reinterpret_cast<const V*>(st + m * kStgPitch + c0);
        V t;
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = st[(c0 + e) * kStgPitch + m];
        const int64_t chunk = int64_t(s * 64 + lane) * 8;
        *reinterpret_cast<V*>(out + half_part(2 * h) + chunk) = a;
        *reinterpret_cast<V*>(out + half_part(2 * h + 1) + chunk) = t;
        if (outm) {
          *reinterpret_cast<V*>(outm + half_part(2 * h) + chunk) = t;
          *reinterpret_cast<V*>(outm + half_part(2 * h + 1) + chunk) = a;
        }
      }
    }
    // Every lane's reads precede the next block's writes.
    __builtin_amdgcn_wave_barrier();
  }
  const double n2 = wave_sum(nrm);
  const double e2 = g.sp2 ? wave_sum(err) : 0.0;
  const double t = (g.sp2 && i == j) ? wave_sum(tr) : 0.0;
  const bool any_over = __ballot(over) != 0;
  if (lane == 0) {
    const int64_t cell = int64_t(i) * g.nb + j;
    g.norm_c[cell] = sqrt(n2);
    g.map_c[cell] = int32_t(node);
    g.coords_c[node] = pack_ij(i, j);
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
    if (any_over && g.overflow) *g.overflow = 1;
  }
}

// One wave per 2 x 2 group of C blocks (tier d-1 node), operands in
// registers; kAhead = 2: the next step's tiles in flight during the current
// products; 1: one operand set (fewer registers, other waves hide the
// latency).
template <int P, int kAhead>
__device__ __forceinline__ void half_w2x2(const GemmArgs& g, int64_t p, int lane,
                                          int32_t (*tab)[2 * kWBatch], float* sym_lds,
                                          typename Half<P>::T* stg) {
  typedef typename Half<P>::T T;
  const int32_t IJ = uniform(g.sup_nodes[p]);
  const int I = unpack_i(IJ), J = unpack_j(IJ);
  const int stride = (is_split(P) ? 4 : 2) * kLeaf2;
  const T* pa = static_cast<const T*>(g.pool_a);
  const T* pb = static_cast<const T*>(g.pool_b);
  const int64_t e0 = uniform(g.sup_nptr[p]), e1 = uniform(g.sup_nptr[p + 1]);
  HAcc<P> acc[4];
  HFrag<P> fa[2][2], fb[2][2];  // [set][row or column]
  for (int64_t eb = e0; eb < e1; eb += kWBatch) {
    int32_t mask = 0, sl[4] = {-1, -1, -1, -1};
    const int64_t e = eb + (lane >> 1);
    if (e < e1) {
      const int c = lane & 1;
      const int bits = g.sup_bits[e];
      for (int q = 0; q < 4; ++q) mask |= ((bits >> (2 * q + c)) & 1) << q;
      const int k = 2 * g.sup_ks[e] + c;
      if (mask & 0x3) sl[0] = g.map_a[int64_t(2 * I) * g.nb + k];
      if (mask & 0xC) sl[1] = g.map_a[int64_t(2 * I + 1) * g.nb + k];
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
    auto fetch = [&](int x, HFrag<P> (&ra)[2], HFrag<P> (&rb)[2]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int32_t sa = __builtin_amdgcn_readfirstlane(tab[1 + u][x]);
        const int32_t sb = __builtin_amdgcn_readfirstlane(tab[3 + u][x]);
        if (sa >= 0) load_frag<P>(pa + int64_t(sa) * stride, 0, lane, ra[u]);
        if (sb >= 0) load_frag<P>(pb + int64_t(sb) * stride, 1, lane, rb[u]);
      }
    };
    auto compute = [&](int x, const HFrag<P> (&ra)[2], const HFrag<P> (&rb)[2]) {
      const int m = __builtin_amdgcn_readfirstlane(tab[0][x]);
      if (m & 1) acc[0].add(ra[0], rb[0]);
      if (m & 2) acc[1].add(ra[0], rb[1]);
      if (m & 4) acc[2].add(ra[1], rb[0]);
      if (m & 8) acc[3].add(ra[1], rb[1]);
    };
    if (kAhead == 1) {
      for (int x = 0; x < n_steps; ++x) {
        fetch(x, fa[0], fb[0]);
        compute(x, fa[0], fb[0]);
      }
    } else if (n_steps > 0) {
      fetch(0, fa[0], fb[0]);
      int x = 0;
      for (; x + 2 < n_steps; x += 2) {
        fetch(x + 1, fa[1], fb[1]);
        __builtin_amdgcn_sched_barrier(0);
        compute(x, fa[0], fb[0]);
        __builtin_amdgcn_sched_barrier(0);
        fetch(x + 2, fa[0], fb[0]);
        __builtin_amdgcn_sched_barrier(0);
        compute(x + 1, fa[1], fb[1]);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (x + 1 < n_steps) {
        fetch(x + 1, fa[1], fb[1]);
        __builtin_amdgcn_sched_barrier(0);
        compute(x, fa[0], fb[0]);
        compute(x + 1, fa[1], fb[1]);
      } else {
        compute(x, fa[0], fb[0]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (uniform(g.sup_cnt4[4 * p + q]) <= 0) continue;
    epilogue<P>(g, uniform(g.sup_noff[4 * p + q]), 2 * I + (q >> 1), 2 * J + (q & 1), acc[q], lane,
                sym_lds, stg);
  }
}

// kW: waves (2 x 2 groups) per workgroup.
// With one operand set the kernels are held to two waves per SIMD (the
// split forms then keep their accumulators in VGPRs and still fit).
template <int P, int kW, int kAhead>
__global__ void __launch_bounds__(64 * kW, kAhead == 1 ? 2 : 1) k_leaf_gemm_half_w2x2(GemmArgs g) {
  __shared__ int32_t s_tab[kW][5][2 * kWBatch];
  __shared__ float s_sym[kW][is_split(P) ? kLeaf * kSymPitch : 1];
  __shared__ __attribute__((aligned(16))) typename Half<P>::T s_stg[kW][stg_elems<P>()];
  const int wave = threadIdx.x >> 6;
  const int64_t p = uniform(xcd_contiguous_block() * kW + wave);
  if (p >= g.n_super) return;
  half_w2x2<P, kAhead>(g, p, threadIdx.x & 63, s_tab[wave], s_sym[wave], s_stg[wave]);
}

template <int P, int kW, int kAhead>
__global__ void __launch_bounds__(64 * kW, kAhead == 1 ? 2 : 1)
    k_leaf_gemm_half_w2x2_batch(GemmBatch b) {
  __shared__ int32_t s_tab[kW][5][2 * kWBatch];
  __shared__ float s_sym[kW][is_split(P) ? kLeaf * kSymPitch : 1];
  __shared__ __attribute__((aligned(16))) typename Half<P>::T s_stg[kW][stg_elems<P>()];
  const int wave = threadIdx.x >> 6;
  int64_t p = 0;
  const GemmArgs* g = batch_locate(b, wave, p);
  if (!g) return;
  half_w2x2<P, kAhead>(*g, p, threadIdx.x & 63, s_tab[wave], s_sym[wave], s_stg[wave]);
}

// One wave per C block over the leaf task list (trees of one tier).
template <int P>
__device__ __forceinline__ void half_block(const GemmArgs& g, int64_t node, int lane,
                                           float* sym_lds,
                                           typename Half<P>::T* stg) {
  typedef typename Half<P>::T T;
  const int32_t ij = uniform(g.nodes[node]);
  const int i = unpack_i(ij), j = unpack_j(ij);
  const int stride = (is_split(P) ? 4 : 2) * kLeaf2;
  const T* pa = static_cast<const T*>(g.pool_a);
  const T* pb = static_cast<const T*>(g.pool_b);
  const int64_t t0 = uniform(g.nptr[node]), t1 = uniform(g.nptr[node + 1]);
  HAcc<P> acc;
  for (int64_t t = t0; t < t1; ++t) {
    const int k = uniform(g.ks[t]);
    const int32_t sa = uniform(g.map_a[int64_t(i) * g.nb + k]);
    const int32_t sb = uniform(g.map_b[int64_t(k) * g.nb + j]);
    HFrag<P> fa, fb;
    load_frag<P>(pa + int64_t(sa) * stride, 0, lane, fa);
    load_frag<P>(pb + int64_t(sb) * stride, 1, lane, fb);
    acc.add(fa, fb);
  }
  epilogue<P>(g, node, i, j, acc, lane, sym_lds, stg);
}

template <int P>
__global__ void __launch_bounds__(256) k_leaf_gemm_half_block(GemmArgs g) {
  __shared__ float s_sym[kWaves][is_split(P) ? kLeaf * kSymPitch : 1];
  __shared__ __attribute__((aligned(16))) typename Half<P>::T s_stg[kWaves][stg_elems<P>()];
  const int64_t node = uniform(int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6));
  if (node >= g.n_nodes) return;
  half_block<P>(g, node, threadIdx.x & 63, s_sym[threadIdx.x >> 6], s_stg[threadIdx.x >> 6]);
}

template <int P>
__global__ void __launch_bounds__(256) k_leaf_gemm_half_block_batch(GemmBatch b) {
  __shared__ float s_sym[kWaves][is_split(P) ? kLeaf * kSymPitch : 1];
  __shared__ __attribute__((aligned(16))) typename Half<P>::T s_stg[kWaves][stg_elems<P>()];
  int64_t node = 0;
  const GemmArgs* g = batch_locate(b, threadIdx.x >> 6, node);
  if (!g) return;
  half_block<P>(*g, node, threadIdx.x & 63, s_sym[threadIdx.x >> 6], s_stg[threadIdx.x >> 6]);
}

// SP2 blocks of X_n with no executed product (see k_sp2_rest).
template <int P>
__global__ void __launch_bounds__(256) k_sp2_rest_half(RestArgs r) {
  typedef typename Half<P>::T T;
  const int lane = threadIdx.x & 63;
  const int64_t s = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  if (s >= r.n_x) return;
  const int32_t ij = r.coords_x[s];
  const int i = unpack_i(ij), j = unpack_j(ij);
  const int64_t cell = int64_t(i) * r.nb + j;
  if (r.map_out[cell] >= 0) return;
  const int stride = (is_split(P) ? 4 : 2) * kLeaf2;
  const T* x = static_cast<const T*>(r.pool_x) + s * stride;
  double e = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int el = q * 64 + lane;
    const double v = decode_half<P>(x[el], is_split(P) ? x[half_part(2) + el] : T(0.0f));
    e += v * v;
  }
  e = wave_sum(e);
  if (lane == 0) r.err_part[cell] = e;
  if (r.square) return;
  int64_t slot = 0;
  if (lane == 0)
    slot = r.base_slot + atomicAdd(reinterpret_cast<unsigned long long*>(r.counter), 1ull);
  slot = __shfl(slot, 0, 64);
  T* out = static_cast<T*>(r.pool_out) + slot * stride;
  double nrm = 0.0, tr = 0.0;
  // Doubling is exact in both parts, so the transposes are copied as well.
#pragma unroll
  for (int q = 0; q < 16 * (is_split(P) ? 4 : 2); ++q) {
    const int el = q * 64 + lane;
    out[el] = T(2.0f * float(x[el]));
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int el = q * 64 + lane;
    const double v = 2.0 * decode_half<P>(x[el], is_split(P) ? x[half_part(2) + el] : T(0.0f));
    nrm += v * v;
    if (i == j && half_idx_diag(el)) tr += v;
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

// Operand sets in flight per wave of the 16-bit 2 x 2 kernels for a launch
// of `groups` groups (SPAMM_HALF_AHEAD = 1 or 2 overrides).  One set holds
// the kernels to fewer registers: the plain forms run three waves per SIMD
// and the split forms two instead of one.  Measured: the extra waves win
// while a single product is a few thousand groups (150 molecules, 1,770
// groups per symmetric square: BF16 +22%, split FP16 +9%); with 10^5 groups
// (1000 molecules) the
// look-ahead hides more of the operand fetch than the extra waves do (BF16
// +5%, split FP16 +16%), and so it does in the batched launches of a serving
// stream of mixed sizes (split FP16 +7%).
int half_ahead(int prec, int64_t groups, bool batched) {
  const char* v = std::getenv("SPAMM_HALF_AHEAD");
  if (v && std::strcmp(v, "1") == 0) return 1;
  if (v && std::strcmp(v, "2") == 0) return 2;
  if (batched && is_split(prec)) return 2;
  return groups >= kManyGroups ? 2 : 1;
}

template <int P, int kA>
void launch_w2x2_p(const GemmArgs& g, hipStream_t s) {
  const int w = w2x2_waves(g.n_super);
  const unsigned gw = unsigned((g.n_super + w - 1) / w);
  if (w == 1)
    k_leaf_gemm_half_w2x2<P, 1, kA><<<gw, 64, 0, s>>>(g);
  else if (w == 2)
    k_leaf_gemm_half_w2x2<P, 2, kA><<<gw, 128, 0, s>>>(g);
  else
    k_leaf_gemm_half_w2x2<P, 4, kA><<<gw, 256, 0, s>>>(g);
}

template <int P>
void launch_p(const GemmArgs& g, hipStream_t s) {
  if (g.n_super > 0 && half_ahead(P, g.n_super, false) == 1)
    launch_w2x2_p<P, 1>(g, s);
  else if (g.n_super > 0)
    launch_w2x2_p<P, 2>(g, s);
  else
    k_leaf_gemm_half_block<P><<<unsigned((g.n_nodes + kWaves - 1) / kWaves), 256, 0, s>>>(g);
}

template <int P>
void launch_batch_p(const GemmArgs* host, const GemmArgs* dev, int n, hipStream_t s) {
  auto grid = [](const GemmBatch& b) { return unsigned(b.first[b.n]); };
  int64_t groups = 0;
  for (int r = 0; r < n; ++r) groups += host[r].n_nodes > 0 ? host[r].n_super : 0;
  const int w = w2x2_waves(groups);
  for_each_batch(dev, n, w, [&](int r) { return host[r].n_nodes > 0 ? host[r].n_super : 0; },
                 [&](const GemmBatch& b) {
                   const bool a1 = half_ahead(P, groups, true) == 1;
                   if (w == 1 && a1)
                     k_leaf_gemm_half_w2x2_batch<P, 1, 1><<<grid(b), 64, 0, s>>>(b);
                   else if (w == 1)
                     k_leaf_gemm_half_w2x2_batch<P, 1, 2><<<grid(b), 64, 0, s>>>(b);
                   else if (w == 2 && a1)
                     k_leaf_gemm_half_w2x2_batch<P, 2, 1><<<grid(b), 128, 0, s>>>(b);
                   else if (w == 2)
                     k_leaf_gemm_half_w2x2_batch<P, 2, 2><<<grid(b), 128, 0, s>>>(b);
                   else if (a1)
                     k_leaf_gemm_half_w2x2_batch<P, 4, 1><<<grid(b), 256, 0, s>>>(b);
                   else
                     k_leaf_gemm_half_w2x2_batch<P, 4, 2><<<grid(b), 256, 0, s>>>(b);
                 });
  for_each_batch(dev, n, kWaves, [&](int r) { return host[r].n_super > 0 ? 0 : host[r].n_nodes; },
                 [&](const GemmBatch& b) { k_leaf_gemm_half_block_batch<P><<<grid(b), 256, 0, s>>>(b); });
}

template <int P>
void launch_rest_p(const RestArgs& r, hipStream_t s) {
  k_sp2_rest_half<P><<<unsigned((r.n_x + kWaves - 1) / kWaves), 256, 0, s>>>(r);
}

}  // namespace

void launch_leaf_gemm_half(int prec, const GemmArgs& g, hipStream_t s) {
  if (g.n_nodes <= 0) return;
  switch (prec) {
    case SPAMM_BF16: launch_p<SPAMM_BF16>(g, s); break;
    case SPAMM_FP16: launch_p<SPAMM_FP16>(g, s); break;
    case SPAMM_BF16X3: launch_p<SPAMM_BF16X3>(g, s); break;
    case SPAMM_FP16X3: launch_p<SPAMM_FP16X3>(g, s); break;
    default: break;
  }
}

void launch_leaf_gemm_half_batch(int prec, const GemmArgs* host, const GemmArgs* dev, int n,
                                 hipStream_t s) {
  switch (prec) {
    case SPAMM_BF16: launch_batch_p<SPAMM_BF16>(host, dev, n, s); break;
    case SPAMM_FP16: launch_batch_p<SPAMM_FP16>(host, dev, n, s); break;
    case SPAMM_BF16X3: launch_batch_p<SPAMM_BF16X3>(host, dev, n, s); break;
    case SPAMM_FP16X3: launch_batch_p<SPAMM_FP16X3>(host, dev, n, s); break;
    default: break;
  }
}

void launch_sp2_rest_half(int prec, const RestArgs& r, hipStream_t s) {
  if (r.n_x <= 0) return;
  switch (prec) {
    case SPAMM_BF16: launch_rest_p<SPAMM_BF16>(r, s); break;
    case SPAMM_FP16: launch_rest_p<SPAMM_FP16>(r, s); break;
    case SPAMM_BF16X3: launch_rest_p<SPAMM_BF16X3>(r, s); break;
    case SPAMM_FP16X3: launch_rest_p<SPAMM_FP16X3>(r, s); break;
    default: break;
  }
}

}  // namespace spamm
