// Occlusion pass of SpAMM: the breadth-first walk of the (i, j, k) octree of
// Algs. 2-3, tier by tier, keeping a child triple when the product of its
// norms exceeds tau (Eq. 4, strict).
//
// Frontier of tier t: the C nodes (I, J) that still have work, in Morton
// order, each with its ascending list of K.  One 64-lane wave expands one C
// node: every lane takes one K, tests the 8 children (2I+a, 2J+b, 2K+c)
// against the norms of tier t+1, and wave ballots turn the pass bits into
// counts (first pass) and into write positions (second pass).  Child node
// 4p+q (q = 2a+b) of parent p is again in Morton order and its K' = 2K+c
// come out ascending, so the leaf tier is the task list grouped by C block
// with k ascending, in a fixed order, with no sort and no atomics.
//
// Launches: the frontier of tier min(depth, 5) (at most 4^5 nodes, 8^5
// triples, so its buffers are sized for the dense case) comes from one
// single-workgroup launch.
// Every deeper tier takes three launches over a fixed partition of its
// parents into kParts chunks: count (+ chunk totals), scan of the chunk
// totals, then in-chunk offsets + write.
//
// Deeper frontier buffers have host-side capacities; kernels never write
// past them.  When a tier's true size (computed on the device) exceeds its
// capacity, the pass is resumed from the tier above it with enough room.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace spamm {

namespace {

constexpr int kWaves = 4;      // waves per chunk workgroup
constexpr int kParts = 1024;   // chunks per deep tier
constexpr int kTopTier = 5;    // tier of the dense single-workgroup start
constexpr int kTopThreads = 1024;

struct TierIn {
  const int32_t* nodes;
  const int64_t* nptr;
  const int32_t* ks;
  int64_t cap_nodes, cap_tasks;
  int upper;  // keep only C nodes with I <= J (symmetric products)
};

struct TierOut {
  int32_t* nodes;
  int64_t* nptr;
  int32_t* ks;
  int64_t cap_nodes, cap_tasks;
};

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline int64_t wave_incl_scan(int64_t v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Pass bits of the 8 children of (I, J, K): bit (q * 2 + c), q = 2a + b.
// *culled gets the sum of the failing norm products.  With `upper`, the
// child (2I + 1, 2J) of a diagonal node lies below the diagonal: it is
// neither executed nor culled (its block is the mirror of an upper one).
__device__ inline uint32_t child_bits(const double* __restrict__ na, const double* __restrict__ nb,
                                      int64_t w, int I, int J, int K, double tau, double* culled,
                                      bool upper) {
  double av[2][2], bv[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) av[a][c] = na[int64_t(2 * I + a) * w + (2 * K + c)];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[c][b] = nb[int64_t(2 * K + c) * w + (2 * J + b)];
  uint32_t bits = 0;
  double e = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (upper && I == J && a == 1 && b == 0) continue;
        const double p = av[a][c] * bv[c][b];
        if (p > tau)
          bits |= 1u << ((2 * a + b) * 2 + c);
        else
          e += p;
      }
  *culled = e;
  return bits;
}

// Counts of the 4 child C nodes of parent p (tasks per child) and the sum
// of the culled products, for the wave that owns p.
__device__ inline void count_parent(const TierIn& in, const double* na, const double* nb, int64_t w,
                                    double tau, int64_t p, int lane, int32_t cq[4], double* err,
                                    uint8_t* bits_out = nullptr) {
  const int32_t ij = in.nodes[p];
  const int I = unpack_i(ij), J = unpack_j(ij);
  const int64_t beg = in.nptr[p], end = in.nptr[p + 1];
  cq[0] = cq[1] = cq[2] = cq[3] = 0;
  double e = 0.0;
  for (int64_t x0 = beg; x0 < end; x0 += 64) {
    const int64_t x = x0 + lane;
    uint32_t bits = 0;
    if (x < end) {
      double ce;
      bits = child_bits(na, nb, w, I, J, in.ks[x], tau, &ce, in.upper);
      e += ce;
      if (bits_out) bits_out[x] = uint8_t(bits);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      cq[q] += __popcll(__ballot((bits >> (2 * q)) & 1)) +
               __popcll(__ballot((bits >> (2 * q + 1)) & 1));
  }
  *err = wave_sum(e);
}

// Writes the children of parent p: child node q (if non-empty) at index
// noff[q] with its tasks from toff[q].
__device__ inline void write_parent(const TierIn& in, const double* na, const double* nb, int64_t w,
                                    double tau, int64_t p, int lane, const int32_t cq[4],
                                    const int64_t toff[4], const int64_t noff[4],
                                    const TierOut& out) {
  const int32_t ij = in.nodes[p];
  const int I = unpack_i(ij), J = unpack_j(ij);
  const uint64_t below = (uint64_t(1) << lane) - 1;
  int64_t pos[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    pos[q] = toff[q];
    if (lane == 0 && cq[q] > 0) {
      out.nodes[noff[q]] = pack_ij(2 * I + (q >> 1), 2 * J + (q & 1));
      out.nptr[noff[q]] = toff[q];
    }
  }
  const int64_t beg = in.nptr[p], end = in.nptr[p + 1];
  for (int64_t x0 = beg; x0 < end; x0 += 64) {
    const int64_t x = x0 + lane;
    uint32_t bits = 0;
    int K = 0;
    if (x < end) {
      double ce;
      K = in.ks[x];
      bits = child_bits(na, nb, w, I, J, K, tau, &ce, in.upper);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool p0 = (bits >> (2 * q)) & 1, p1 = (bits >> (2 * q + 1)) & 1;
      const uint64_t b0 = __ballot(p0), b1 = __ballot(p1);
      const int64_t at = pos[q] + __popcll(b0 & below) + __popcll(b1 & below);
      if (p0) out.ks[at] = 2 * K;
      if (p1) out.ks[at + (p0 ? 1 : 0)] = 2 * K + 1;
      pos[q] += __popcll(b0) + __popcll(b1);
    }
  }
}

// ---- top tiers: one workgroup ------------------------------------------------
//
// Tier t0 = min(depth, 5) is built directly from its own norms: by Eq. 3 a
// node's norm bounds its descendants', so a tier-t0 triple passes every
// ancestor test whenever it passes its own, and the frontier the walk would
// reach at t0 is the flat set {(I, J, K) : ||A_IK|| ||B_KJ|| > tau} there
// (up to rounding in the last bit of the norms, inside the tie band).
// One thread per tier-t0 C node (Morton index), one bit per K.  The same
// launch adds up the culled-product bound over the tiers 1..t0: a triple
// counts when it fails and its parent passes (the root is never tested).

struct TopArgs {
  int depth, t0;
  int want_err;  // also the culled-product bound of tiers 1..t0
  int upper;     // only C nodes with I <= J
  double tau;
  const double* norms_a;
  const double* norms_b;
  int32_t* nodes;
  int64_t* nptr;
  int32_t* ks;
  Control* ctl;
  double* pyr_norms;  // with pyr_top >= 0: first the pyramid tiers pyr_top .. 0
  int pyr_top;
};

constexpr int kTopNorms = 1365;  // tiers 0..5: (4^6 - 1) / 3

__device__ inline void demorton(int m, int bits, int* I, int* J) {
  int i = 0, j = 0;
  for (int b = 0; b < bits; ++b) {
    j |= ((m >> (2 * b)) & 1) << b;
    i |= ((m >> (2 * b + 1)) & 1) << b;
  }
  *I = i;
  *J = j;
}

__global__ void __launch_bounds__(kTopThreads) k_cull_top(TopArgs g) {
  __shared__ double sa[kTopNorms], sb[kTopNorms];
  __shared__ int64_t s_wc[kTopThreads / 64], s_wz[kTopThreads / 64];
  __shared__ double s_e[kTopThreads];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The single-workgroup top of the operands' pyramid, when the caller left
  // it to this launch (the operands are then one matrix).
  if (g.pyr_top >= 0) pyramid_tiers(g.pyr_norms, g.pyr_top);
  Control* ctl = g.ctl;
  const int t0 = g.t0;
  if (tid < kMaxTiers) {
    ctl->n_nodes[tid] = -1;
    ctl->n_tasks[tid] = -1;
    ctl->err[tid] = 0.0;
  }
  if (tid == 0) ctl->nonzero_pairs = 0;
  const int n_norms = int(tier_offset(t0 + 1));
  for (int x = tid; x < n_norms; x += kTopThreads) {
    sa[x] = g.norms_a[x];
    sb[x] = g.norms_b[x];
  }
  __syncthreads();
  if (g.depth == 0) {
    // A single leaf: the product itself is tested (the root is a leaf).
    if (tid == 0) {
      const double p = sa[0] * sb[0];
      const bool keep = p > g.tau;
      g.nptr[0] = 0;
      if (keep) {
        g.nodes[0] = pack_ij(0, 0);
        g.ks[0] = 0;
        g.nptr[1] = 1;
      } else {
        ctl->err[0] = p;
      }
      ctl->n_nodes[0] = keep ? 1 : 0;
      ctl->n_tasks[0] = keep ? 1 : 0;
    }
    return;
  }
  const int W = 1 << t0;
  const double* A = sa + tier_offset(t0);
  const double* B = sb + tier_offset(t0);
  int I = 0, J = 0;
  uint32_t mask = 0;
  if (tid < W * W) {
    demorton(tid, t0, &I, &J);
    if (!(g.upper && I > J))
      for (int K = 0; K < W; ++K)
        if (A[I * W + K] * B[K * W + J] > g.tau) mask |= 1u << K;
  }
  const int v = __popc(mask);
  const int64_t ic = wave_incl_scan(v, lane), iz = wave_incl_scan(v > 0 ? 1 : 0, lane);
  if (lane == 63) {
    s_wc[wave] = ic;
    s_wz[wave] = iz;
  }
  // Culled-product bound of tiers 1..t0, summed per thread in a fixed order
  // (only when asked for: SP2 never reads it, and it is most of this
  // kernel's time).
  double e = 0.0;
  for (int t = 1; g.want_err && t <= t0; ++t) {
    const int w = 1 << t;
    const double* a = sa + tier_offset(t);
    const double* b = sb + tier_offset(t);
    const double* ap = sa + tier_offset(t - 1);
    const double* bp = sb + tier_offset(t - 1);
    for (int x = tid; x < w * w * w; x += kTopThreads) {
      const int i = x >> (2 * t), j = (x >> t) & (w - 1), k = x & (w - 1);
      if (g.upper && i > j) continue;
      const double p = a[i * w + k] * b[k * w + j];
      if (p > g.tau) continue;
      if (t > 1 && !(ap[(i / 2) * (w / 2) + k / 2] * bp[(k / 2) * (w / 2) + j / 2] > g.tau))
        continue;
      e += p;
    }
  }
  s_e[tid] = e;
  __syncthreads();
  int64_t pc = 0, pz = 0, tc = 0, tz = 0;
  for (int x = 0; x < kTopThreads / 64; ++x) {
    if (x < wave) {
      pc += s_wc[x];
      pz += s_wz[x];
    }
    tc += s_wc[x];
    tz += s_wz[x];
  }
  if (v > 0) {
    const int64_t to = pc + ic - v, no = pz + iz - 1;
    g.nodes[no] = pack_ij(I, J);
    g.nptr[no] = to;
    int r = 0;
    for (uint32_t m = mask; m; m &= m - 1) g.ks[to + r++] = __ffs(m) - 1;
  }
  // (want_err is uniform: every thread takes the same branch.)
  if (g.want_err) {
    for (int o = kTopThreads / 2; o > 0; o >>= 1) {
      if (tid < o) s_e[tid] += s_e[tid + o];
      __syncthreads();
    }
  }
  if (tid == 0) {
    g.nptr[tz] = tc;
    ctl->n_nodes[t0] = tz;
    ctl->n_tasks[t0] = tc;
    ctl->err[1] = g.want_err ? s_e[0] : 0.0;
  }
}

// ---- deep tiers: kParts chunks ---------------------------------------------

__device__ inline int64_t parents_in(const Control* ctl, int t, int64_t cap_n, int64_t cap_t) {
  const int64_t n = ctl->n_nodes[t], k = ctl->n_tasks[t];
  return (n >= 0 && n <= cap_n && k >= 0 && k <= cap_t) ? n : 0;
}

// Per chunk: child counts into cnt4, and the chunk's totals (tasks,
// non-empty children, culled-product sum, non-empty children off the
// diagonal) into part.
__global__ void __launch_bounds__(64 * kWaves) k_cull_count(TierIn in, const double* __restrict__ na,
                                                            const double* __restrict__ nb, int t,
                                                            double tau, Control* ctl,
                                                            int32_t* __restrict__ cnt4,
                                                            int64_t* __restrict__ part,
                                                            uint8_t* __restrict__ bits_out) {
  __shared__ int64_t s_c[kWaves], s_z[kWaves], s_m[kWaves];
  __shared__ double s_e[kWaves];
  const int64_t P = parents_in(ctl, t, in.cap_nodes, in.cap_tasks);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->scratch[0] = P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ch = (P + kParts - 1) / kParts;
  const int64_t b0 = int64_t(blockIdx.x) * ch, b1 = min(P, b0 + ch);
  const int64_t w = int64_t(2) << t;
  int64_t c = 0, z = 0, m = 0;
  double e = 0.0;
  for (int64_t p = b0 + wave; p < b1; p += kWaves) {
    int32_t cq[4];
    double pe;
    count_parent(in, na, nb, w, tau, p, lane, cq, &pe, bits_out);
    e += pe;
    const int32_t ij = in.nodes[p];
    const bool diag = unpack_i(ij) == unpack_j(ij);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c += cq[q];
      z += cq[q] > 0;
      m += cq[q] > 0 && !(diag && (q == 0 || q == 3));
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) cnt4[4 * p + q] = cq[q];
    }
  }
  if (lane == 0) {
    s_c[wave] = c;
    s_z[wave] = z;
    s_m[wave] = m;
    s_e[wave] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t tc = 0, tz = 0, tm = 0;
    double te = 0.0;
    for (int x = 0; x < kWaves; ++x) {
      tc += s_c[x];
      tz += s_z[x];
      tm += s_m[x];
      te += s_e[x];
    }
    part[blockIdx.x] = tc;
    part[kParts + blockIdx.x] = tz;
    reinterpret_cast<double*>(part + 2 * kParts)[blockIdx.x] = te;
    part[3 * kParts + blockIdx.x] = tm;
  }
}

__device__ inline int64_t wave_sum_i(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Chunk bases and tier totals from the chunk counts, in every workgroup of
// the write pass (the counts are 32 KiB and stay in L2): for x = tasks,
// nodes, off-diagonal nodes, the sum over the chunks before `self`
// (base[x]) and over all chunks (total[x]).  Integer sums: any order gives
// the same result.
__device__ inline void chunk_bases(const int64_t* __restrict__ part, int self, int64_t base[3],
                                   int64_t total[3]) {
  __shared__ int64_t s_r[6][kWaves];
  constexpr int kPer = kParts / (64 * kWaves);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int comp[3] = {0, 1, 3};
  int64_t v[6];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    int64_t before = 0, all = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int b = threadIdx.x * kPer + u;
      const int64_t y = part[comp[x] * kParts + b];
      all += y;
      before += b < self ? y : 0;
    }
    v[2 * x] = wave_sum_i(before);
    v[2 * x + 1] = wave_sum_i(all);
  }
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < 6; ++r) s_r[r][wave] = v[r];
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    base[x] = 0;
    total[x] = 0;
    for (int y = 0; y < kWaves; ++y) {
      base[x] += s_r[2 * x][y];
      total[x] += s_r[2 * x + 1][y];
    }
  }
}

// Culled-product sum of the tier over the chunks, in the fixed pairwise
// order of a kParts-leaf tree (one workgroup).
__device__ inline double chunk_err(const int64_t* __restrict__ part) {
  __shared__ double s_e[kParts];
  const double* pe = reinterpret_cast<const double*>(part + 2 * kParts);
  for (int b = threadIdx.x; b < kParts; b += 64 * kWaves) s_e[b] = pe[b];
  __syncthreads();
  for (int o = kParts / 2; o > 0; o >>= 1) {
    for (int b = threadIdx.x; b < o; b += 64 * kWaves) s_e[b] += s_e[b + o];
    __syncthreads();
  }
  return s_e[0];
}

// Per chunk: the chunk's bases (workgroup 0 also stores the tier totals in
// the control block), in-chunk exclusive offsets of the child counts, then
// the children themselves.  With `moff` (the leaf tier of symmetric
// products) also each leaf node's mirror offset: the number of off-diagonal
// C blocks before it, with their total in ctl->scratch[3].
__global__ void __launch_bounds__(64 * kWaves) k_cull_write(TierIn in, const double* __restrict__ na,
                                                            const double* __restrict__ nb, int t,
                                                            double tau, Control* ctl,
                                                            const int32_t* __restrict__ cnt4,
                                                            const int64_t* __restrict__ part,
                                                            int64_t* __restrict__ toff,
                                                            int64_t* __restrict__ noff,
                                                            int64_t* __restrict__ moff,
                                                            TierOut out) {
  __shared__ int64_t s_wc[kWaves], s_wz[kWaves], s_wm[kWaves];
  const int64_t P = ctl->scratch[0];
  int64_t base[3], total[3];
  chunk_bases(part, blockIdx.x, base, total);
  const int64_t k_out = total[0], n_out = total[1];
  if (blockIdx.x == 0) {
    const double e = chunk_err(part);
    if (threadIdx.x == 0) {
      ctl->n_tasks[t + 1] = k_out;
      ctl->n_nodes[t + 1] = n_out;
      ctl->err[t + 1] = e;
      if (moff) ctl->scratch[3] = total[2];
    }
  }
  if (n_out > out.cap_nodes || k_out > out.cap_tasks) return;  // resumed with more room
  if (blockIdx.x == 0 && threadIdx.x == 0) out.nptr[n_out] = k_out;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ch = (P + kParts - 1) / kParts;
  const int64_t b0 = int64_t(blockIdx.x) * ch, b1 = min(P, b0 + ch);
  if (b0 >= b1) return;
  int64_t base_c = base[0], base_z = base[1], base_m = base[2];
  for (int64_t x0 = 4 * b0; x0 < 4 * b1; x0 += 64 * kWaves) {
    const int64_t x = x0 + threadIdx.x;
    const int32_t v = x < 4 * b1 ? cnt4[x] : 0;
    const int fz = v > 0 ? 1 : 0;
    int fm = 0;
    if (moff && fz) {
      const int32_t ij = in.nodes[x >> 2];
      const int q = int(x & 3);
      fm = !(unpack_i(ij) == unpack_j(ij) && (q == 0 || q == 3));
    }
    const int64_t ic = wave_incl_scan(v, lane), iz = wave_incl_scan(fz, lane);
    const int64_t im = moff ? wave_incl_scan(fm, lane) : 0;
    if (lane == 63) {
      s_wc[wave] = ic;
      s_wz[wave] = iz;
      s_wm[wave] = im;
    }
    __syncthreads();
    int64_t pc = 0, pz = 0, pm = 0, tc = 0, tz = 0, tm = 0;
    for (int y = 0; y < kWaves; ++y) {
      if (y < wave) {
        pc += s_wc[y];
        pz += s_wz[y];
        pm += s_wm[y];
      }
      tc += s_wc[y];
      tz += s_wz[y];
      tm += s_wm[y];
    }
    if (x < 4 * b1) {
      const int64_t node = base_z + pz + iz - fz;
      toff[x] = base_c + pc + ic - v;
      noff[x] = node;
      if (moff && fz) moff[node] = base_m + pm + im - fm;
    }
    base_c += tc;
    base_z += tz;
    base_m += tm;
    __syncthreads();
  }
  const int64_t w = int64_t(2) << t;
  for (int64_t p = b0 + wave; p < b1; p += kWaves) {
    int32_t cq[4];
    int64_t to[4], no[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cq[q] = cnt4[4 * p + q];
      to[q] = toff[4 * p + q];
      no[q] = noff[4 * p + q];
    }
    write_parent(in, na, nb, w, tau, p, lane, cq, to, no, out);
  }
}

// #(i, j, k) with A_ik != 0 and B_kj != 0: sum over k of (non-zero blocks of
// column k of A) x (non-zero blocks of row k of B).
__global__ void __launch_bounds__(1024) k_nonzero_pairs(const double* __restrict__ na,
                                                        const double* __restrict__ nb, int n,
                                                        Control* ctl) {
  __shared__ int64_t sh[1024];
  int64_t acc = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    int64_t ca = 0, rb = 0;
    for (int i = 0; i < n; ++i) ca += na[int64_t(i) * n + k] != 0.0;
    for (int j = 0; j < n; ++j) rb += nb[int64_t(k) * n + j] != 0.0;
    acc += ca * rb;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) ctl->nonzero_pairs = sh[0];
}

// One wave per tier-(d-2) node, one lane per entry K: bit 16c + 4a + b is
// set when leaf product (4I + a, 4J + b, 4K + c) passes and its tier-(d-1)
// parent (2I + a/2, 2J + b/2, 2K + c/2) passes too, the same two tests, on
// the same values, that the tier walk made for it.
__global__ void __launch_bounds__(64 * kWaves) k_quad_masks(TierIn in, const double* __restrict__ na1,
                                                            const double* __restrict__ nb1,
                                                            const double* __restrict__ na,
                                                            const double* __restrict__ nb, int d,
                                                            double tau, int64_t P,
                                                            uint64_t* __restrict__ masks) {
  const int lane = threadIdx.x & 63;
  const int64_t w1 = int64_t(1) << (d - 1), w = int64_t(1) << d;
  for (int64_t p = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6); p < P;
       p += int64_t(gridDim.x) * kWaves) {
    const int32_t ij = in.nodes[p];
    const int I = unpack_i(ij), J = unpack_j(ij);
    const int64_t beg = in.nptr[p], end = in.nptr[p + 1];
    for (int64_t x = beg + lane; x < end; x += 64) {
      const int K = in.ks[x];
      uint64_t m = 0;
      for (int c = 0; c < 4; ++c) {
        const int k = 4 * K + c, k1 = 2 * K + c / 2;
        for (int a = 0; a < 4; ++a) {
          const double pa1 = na1[int64_t(2 * I + a / 2) * w1 + k1];
          const double pa = na[int64_t(4 * I + a) * w + k];
          for (int b = 0; b < 4; ++b) {
            const bool parent = pa1 * nb1[int64_t(k1) * w1 + 2 * J + b / 2] > tau;
            const bool leaf = pa * nb[int64_t(k) * w + 4 * J + b] > tau;
            if (parent && leaf) m |= uint64_t(1) << (16 * c + 4 * a + b);
          }
        }
      }
      masks[x] = m;
    }
  }
}

__global__ void k_scatter_nodes(const int32_t* __restrict__ nodes, int64_t n, int nb,
                                int32_t* __restrict__ map_c, int32_t* __restrict__ coords_c) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int32_t ij = nodes[x];
  map_c[int64_t(unpack_i(ij)) * nb + unpack_j(ij)] = int32_t(x);
  coords_c[x] = ij;
}

inline int64_t pow_cap(int base_log2, int t, int64_t cap) {
  const int sh = base_log2 * t;
  if (sh >= 62) return cap;
  return std::min<int64_t>(int64_t(1) << sh, cap);
}

Error reserve_tier(CullWork& w, int t, hipStream_t s) {
  SPAMM_TRY(w.nodes[t].reserve(size_t(std::max<int64_t>(w.cap_nodes[t], 1)) * 4, s));
  SPAMM_TRY(w.nptr[t].reserve(size_t(w.cap_nodes[t] + 1) * 8, s));
  SPAMM_TRY(w.ks[t].reserve(size_t(std::max<int64_t>(w.cap_tasks[t], 1)) * 4, s));
  if (t + 1 == w.depth)
    SPAMM_TRY(w.bits.reserve(size_t(std::max<int64_t>(w.cap_tasks[t], 1)), s));
  if (t + 2 == w.depth)
    SPAMM_TRY(w.quad.reserve(size_t(std::max<int64_t>(w.cap_tasks[t], 1)) * 8, s));
  const int64_t need = 4 * std::max<int64_t>(w.cap_nodes[t], 1);
  if (need > w.cap_count) {
    SPAMM_TRY(w.cnt4.reserve(size_t(need) * 4, s));
    SPAMM_TRY(w.toff.reserve(size_t(need) * 8, s));
    SPAMM_TRY(w.noff.reserve(size_t(need) * 8, s));
    w.cap_count = need;
  }
  return Error{};
}

TierIn tier_in(CullWork& w, int t) {
  return TierIn{static_cast<const int32_t*>(w.nodes[t].p), static_cast<const int64_t*>(w.nptr[t].p),
                static_cast<const int32_t*>(w.ks[t].p), w.cap_nodes[t], w.cap_tasks[t],
                w.upper ? 1 : 0};
}

TierOut tier_out(CullWork& w, int t) {
  return TierOut{static_cast<int32_t*>(w.nodes[t].p), static_cast<int64_t*>(w.nptr[t].p),
                 static_cast<int32_t*>(w.ks[t].p), w.cap_nodes[t], w.cap_tasks[t]};
}

void expand(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, int t, double tau,
            hipStream_t s) {
  const TierIn in = tier_in(w, t);
  const double* na = a->norms + tier_offset(t + 1);
  const double* nb = b->norms + tier_offset(t + 1);
  int64_t* part = static_cast<int64_t*>(w.part.p);
  Control* ctl = w.ctl_dev;
  // The last expansion also keeps each tier-(d-1) triple's 8 pass bits for
  // the leaf products' 2 x 2 block groups.
  uint8_t* bits = t + 1 == a->depth ? static_cast<uint8_t*>(w.bits.p) : nullptr;
  int64_t* moff = w.upper && t + 1 == a->depth ? static_cast<int64_t*>(w.moff.p) : nullptr;
  k_cull_count<<<kParts, 64 * kWaves, 0, s>>>(in, na, nb, t, tau, ctl,
                                              static_cast<int32_t*>(w.cnt4.p), part, bits);
  k_cull_write<<<kParts, 64 * kWaves, 0, s>>>(in, na, nb, t, tau, ctl,
                                              static_cast<const int32_t*>(w.cnt4.p), part,
                                              static_cast<int64_t*>(w.toff.p),
                                              static_cast<int64_t*>(w.noff.p), moff,
                                              tier_out(w, t + 1));
}

void launch_top(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, int t0, double tau,
                bool want_err, int pyr_top, hipStream_t s) {
  TopArgs g{};
  g.pyr_norms = a->norms;
  g.pyr_top = pyr_top;
  g.depth = a->depth;
  g.t0 = t0;
  g.want_err = want_err ? 1 : 0;
  g.upper = w.upper ? 1 : 0;
  g.tau = tau;
  g.norms_a = a->norms;
  g.norms_b = b->norms;
  g.nodes = static_cast<int32_t*>(w.nodes[t0].p);
  g.nptr = static_cast<int64_t*>(w.nptr[t0].p);
  g.ks = static_cast<int32_t*>(w.ks[t0].p);
  g.ctl = w.ctl_dev;
  k_cull_top<<<1, kTopThreads, 0, s>>>(g);
}

}  // namespace

Error ensure_control(CullWork& w) {
  if (w.ctl_dev == nullptr) SPAMM_HIP(hipMalloc(reinterpret_cast<void**>(&w.ctl_dev), sizeof(Control)));
  if (w.ctl_host == nullptr)
    SPAMM_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.ctl_host), sizeof(Control), 0));
  return Error{};
}

void CullWork::release(hipStream_t s) {
  for (int t = 0; t < kMaxTiers; ++t) {
    nodes[t].release(s);
    nptr[t].release(s);
    ks[t].release(s);
  }
  cnt4.release(s);
  bits.release(s);
  quad.release(s);
  mflag.release(s);
  moff.release(s);
  mscan.part.release(s);
  toff.release(s);
  noff.release(s);
  part.release(s);
  cap_count = 0;
  depth = -1;
}

CullWork::~CullWork() {
  // Device buffers are released by the owner on its stream; the control
  // block is synchronous memory.
  if (ctl_dev) (void)hipFree(ctl_dev);
  if (ctl_host) (void)hipHostFree(ctl_host);
}

namespace {

__global__ void k_offdiag_flags(const int32_t* __restrict__ nodes, const int64_t* len_dev,
                                int64_t cap, int32_t* __restrict__ flag) {
  int64_t n = *len_dev;
  if (n < 0 || n > cap) n = 0;  // a pass that overflowed: recomputed after the regrowth
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < n;
       x += int64_t(gridDim.x) * blockDim.x)
    flag[x] = unpack_i(nodes[x]) != unpack_j(nodes[x]) ? 1 : 0;
}

// The same for short lists, in one workgroup: each thread counts a
// contiguous chunk, one scan over the 1024 chunk counts, then offsets.
constexpr int64_t kMirrorSmall = 65536;
__global__ void __launch_bounds__(1024) k_mirror_small(const int32_t* __restrict__ nodes,
                                                       const int64_t* len_dev, int64_t cap,
                                                       int64_t* __restrict__ moff,
                                                       int64_t* total) {
  __shared__ int64_t s[1024];
  int64_t n = *len_dev;
  if (n < 0 || n > cap) n = 0;
  const int t = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t b0 = min(n, t * chunk), b1 = min(n, b0 + chunk);
  int64_t c = 0;
  for (int64_t x = b0; x < b1; ++x) c += unpack_i(nodes[x]) != unpack_j(nodes[x]);
  s[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t add = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int64_t run = s[t] - c;
  for (int64_t x = b0; x < b1; ++x) {
    moff[x] = run;
    run += unpack_i(nodes[x]) != unpack_j(nodes[x]);
  }
  if (t == 1023) *total = s[1023];
}

// Symmetric products: moff[x] = number of off-diagonal C blocks before leaf
// node x (their mirrors take the slots after the direct ones), the total
// into ctl->scratch[3].  Lengths come from the control block.
Error mirror_offsets(CullWork& w, int d, hipStream_t s) {
  const int64_t cap = std::max<int64_t>(w.cap_nodes[d], 1);
  SPAMM_TRY(w.mflag.grow(size_t(cap) * sizeof(int32_t), s));
  SPAMM_TRY(w.moff.grow(size_t(cap) * sizeof(int64_t), s));
  Control* ctl = w.ctl_dev;
  if (w.cap_nodes[d] <= kMirrorSmall) {
    k_mirror_small<<<1, 1024, 0, s>>>(static_cast<const int32_t*>(w.nodes[d].p), &ctl->n_nodes[d],
                                      w.cap_nodes[d], static_cast<int64_t*>(w.moff.p),
                                      &ctl->scratch[3]);
    return Error{};
  }
  int32_t* flag = static_cast<int32_t*>(w.mflag.p);
  const unsigned grid = unsigned(std::min<int64_t>((cap + 255) / 256, 1024));
  k_offdiag_flags<<<grid, 256, 0, s>>>(static_cast<const int32_t*>(w.nodes[d].p),
                                       &ctl->n_nodes[d], w.cap_nodes[d], flag);
  return launch_scan(flag, static_cast<int64_t*>(w.moff.p), nullptr, nullptr, &ctl->n_nodes[d],
                     w.cap_nodes[d], 1, 0, &ctl->scratch[3], nullptr, nullptr, w.mscan, s);
}

}  // namespace

Error cull_launch(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
                  bool want_pairs, hipStream_t s, bool upper, int pyr_top) {
  if (pyr_top >= 0 && a != b) return err(SPAMM_ERR_INVALID_ARG, "deferred pyramid needs A == B");
  const int d = a->depth;
  w.upper = upper;
  const int t_top = std::min(d, kTopTier);
  SPAMM_TRY(ensure_control(w));
  if (w.depth != d) {
    // Top tiers: the dense bound (4^t nodes, 8^t triples).  Deeper tiers:
    // modest capacities, regrown on demand.
    for (int t = 0; t <= d; ++t) {
      if (t <= t_top) {
        w.cap_nodes[t] = pow_cap(2, t, int64_t(1) << 62);
        w.cap_tasks[t] = pow_cap(3, t, int64_t(1) << 62);
      } else {
        w.cap_nodes[t] = std::max<int64_t>(1, pow_cap(2, t, int64_t(1) << 16));
        w.cap_tasks[t] = std::max<int64_t>(1, pow_cap(3, t, int64_t(1) << 18));
      }
    }
    w.depth = d;
  }
  for (int t = 0; t <= d; ++t) SPAMM_TRY(reserve_tier(w, t, s));
  SPAMM_TRY(w.part.reserve(4 * kParts * sizeof(int64_t), s));
  if (upper)
    SPAMM_TRY(w.moff.grow(size_t(std::max<int64_t>(w.cap_nodes[d], 1)) * sizeof(int64_t), s));
  Control* ctl = w.ctl_dev;
  {
    PhaseTimer timer(SPAMM_PHASE_CULL, s);
    launch_top(w, a, b, t_top, tau, want_pairs, pyr_top, s);
    for (int t = t_top; t < d; ++t) expand(w, a, b, t, tau, s);
    // The leaf tier's write pass stores the mirror offsets; a tree no
    // deeper than the top tier needs the separate pass.
    if (upper && t_top == d) SPAMM_TRY(mirror_offsets(w, d, s));
    if (want_pairs)
      k_nonzero_pairs<<<1, 1024, 0, s>>>(a->norms + tier_offset(d), b->norms + tier_offset(d),
                                         a->nb, ctl);
  }
  SPAMM_HIP(hipMemcpyAsync(w.ctl_host, ctl, sizeof(Control), hipMemcpyDeviceToHost, s));
  return Error{};
}

Error cull_finish(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
                  bool want_pairs, hipStream_t s, CullResult* out) {
  const int d = a->depth;
  Control* ctl = w.ctl_dev;
  out->restarts = 0;
  for (bool first = true;; first = false) {
    if (!first) {
      SPAMM_HIP(hipMemcpyAsync(w.ctl_host, ctl, sizeof(Control), hipMemcpyDeviceToHost, s));
      SPAMM_HIP(hipStreamSynchronize(s));
    }
    const Control& h = *w.ctl_host;
    int bad = -1;
    for (int t = 1; t <= d; ++t)
      if (h.n_nodes[t] > w.cap_nodes[t] || h.n_tasks[t] > w.cap_tasks[t]) {
        bad = t;
        break;
      }
    if (bad < 0) break;
    // Tier `bad` is known exactly; its children are bounded by 4x nodes
    // and 8x tasks.  Resume from the expansion that produced it.
    w.cap_nodes[bad] = std::max(w.cap_nodes[bad], h.n_nodes[bad] + h.n_nodes[bad] / 2 + 16);
    w.cap_tasks[bad] = std::max(w.cap_tasks[bad], h.n_tasks[bad] + h.n_tasks[bad] / 2 + 16);
    if (bad < d) {
      const int64_t cn = pow_cap(2, bad + 1, 4 * h.n_nodes[bad]);
      const int64_t ct = std::min<int64_t>(pow_cap(3, bad + 1, 8 * h.n_tasks[bad]),
                                           int64_t(a->nb) * a->nb * a->nb);
      w.cap_nodes[bad + 1] = std::max(w.cap_nodes[bad + 1], cn);
      w.cap_tasks[bad + 1] = std::max(w.cap_tasks[bad + 1], ct);
    }
    for (int t = bad - 1; t <= std::min(d, bad + 1); ++t) SPAMM_TRY(reserve_tier(w, t, s));
    if (w.upper)
      SPAMM_TRY(w.moff.grow(size_t(std::max<int64_t>(w.cap_nodes[d], 1)) * sizeof(int64_t), s));
    ++out->restarts;
    PhaseTimer timer(SPAMM_PHASE_CULL, s);
    for (int t = bad - 1; t < d; ++t) expand(w, a, b, t, tau, s);
  }
  const Control& h = *w.ctl_host;
  out->n_cblocks = h.n_nodes[d];
  out->n_tasks = h.n_tasks[d];
  out->n_mirrors = w.upper ? h.scratch[3] : 0;
  out->moff = w.upper ? static_cast<const int64_t*>(w.moff.p) : nullptr;
  out->nonzero_pairs = want_pairs ? h.nonzero_pairs : -1;
  double e = 0.0;
  for (int t = 0; t <= d; ++t) e += h.err[t];
  out->err_bound = e;
  out->nodes = static_cast<const int32_t*>(w.nodes[d].p);
  out->nptr = static_cast<const int64_t*>(w.nptr[d].p);
  out->ks = static_cast<const int32_t*>(w.ks[d].p);
  if (d >= 1) {
    out->n_super = h.n_nodes[d - 1];
    out->sup_nodes = static_cast<const int32_t*>(w.nodes[d - 1].p);
    out->sup_nptr = static_cast<const int64_t*>(w.nptr[d - 1].p);
    out->sup_ks = static_cast<const int32_t*>(w.ks[d - 1].p);
    out->sup_bits = static_cast<const uint8_t*>(w.bits.p);
    out->sup_cnt4 = static_cast<const int32_t*>(w.cnt4.p);
    out->sup_noff = static_cast<const int64_t*>(w.noff.p);
  }
  if (d >= 2) {
    out->n_quad = h.n_nodes[d - 2];
    out->quad_nodes = static_cast<const int32_t*>(w.nodes[d - 2].p);
    out->quad_nptr = static_cast<const int64_t*>(w.nptr[d - 2].p);
    out->quad_ks = static_cast<const int32_t*>(w.ks[d - 2].p);
    out->quad_masks = static_cast<uint64_t*>(w.quad.p);
  }
  return Error{};
}

void launch_quad_masks(const CullResult& r, const spamm_matrix* a, const spamm_matrix* b,
                       double tau, hipStream_t s) {
  if (r.n_quad <= 0) return;
  const int d = a->depth;
  TierIn in{r.quad_nodes, r.quad_nptr, r.quad_ks, 0, 0, 0};
  const unsigned grid = unsigned(std::min<int64_t>((r.n_quad + kWaves - 1) / kWaves, 8192));
  k_quad_masks<<<grid, 64 * kWaves, 0, s>>>(in, a->norms + tier_offset(d - 1),
                                            b->norms + tier_offset(d - 1), a->norms + tier_offset(d),
                                            b->norms + tier_offset(d), d, tau, r.n_quad,
                                            r.quad_masks);
}

void launch_scatter_nodes(const int32_t* nodes, int64_t n, int nb, int32_t* map_c,
                          int32_t* coords_c, hipStream_t s) {
  if (n <= 0) return;
  k_scatter_nodes<<<unsigned((n + 255) / 256), 256, 0, s>>>(nodes, n, nb, map_c, coords_c);
}

Error run_cull(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
               bool want_pairs, hipStream_t s, CullResult* out) {
  SPAMM_TRY(cull_launch(w, a, b, tau, want_pairs, s, false));
  SPAMM_HIP(hipStreamSynchronize(s));
  return cull_finish(w, a, b, tau, want_pairs, s, out);
}

}  // namespace spamm
