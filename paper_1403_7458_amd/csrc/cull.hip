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
// Frontier buffers have host-side capacities; kernels never write past
// them.  When a tier's true size (computed on the device) exceeds its
// capacity, the pass is resumed from the tier above it with enough room.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace spamm {

namespace {

constexpr int kWaves = 4;  // waves per workgroup
constexpr int kMaxGrid = 4096;

struct TierIn {
  const int32_t* nodes;
  const int64_t* nptr;
  const int32_t* ks;
  int64_t cap_nodes, cap_tasks;
};

__device__ inline int64_t parents_in(const Control* ctl, int t, int64_t cap_n, int64_t cap_t) {
  const int64_t n = ctl->n_nodes[t], k = ctl->n_tasks[t];
  return (n >= 0 && n <= cap_n && k >= 0 && k <= cap_t) ? n : 0;
}

__global__ void k_cull_init(Control* ctl, int depth, int32_t* nodes0, int64_t* nptr0, int32_t* ks0,
                            const double* na_root, const double* nb_root, double tau) {
  for (int t = 0; t < kMaxTiers; ++t) {
    ctl->n_nodes[t] = -1;
    ctl->n_tasks[t] = -1;
    ctl->err[t] = 0.0;
  }
  ctl->nonzero_pairs = 0;
  bool keep = true;
  if (depth == 0) {
    // A single leaf: the product itself is tested (the root is a leaf).
    const double p = na_root[0] * nb_root[0];
    keep = p > tau;
    if (!keep) ctl->err[0] = p;
  }
  nptr0[0] = 0;
  if (keep) {
    nodes0[0] = pack_ij(0, 0);
    ks0[0] = 0;
    nptr0[1] = 1;
    ctl->n_nodes[0] = 1;
    ctl->n_tasks[0] = 1;
  } else {
    ctl->n_nodes[0] = 0;
    ctl->n_tasks[0] = 0;
  }
}

// Pass bits of the 8 children of (I, J, K): bit (q * 2 + c), q = 2a + b.
__device__ inline uint32_t child_bits(const double* __restrict__ na, const double* __restrict__ nb,
                                      int64_t w, int I, int J, int K, double tau, double* culled) {
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
        const double p = av[a][c] * bv[c][b];
        if (p > tau)
          bits |= 1u << ((2 * a + b) * 2 + c);
        else
          e += p;
      }
  *culled = e;
  return bits;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(256) k_cull_count(TierIn in, const double* __restrict__ na,
                                                    const double* __restrict__ nb, int t,
                                                    double tau, Control* ctl,
                                                    int32_t* __restrict__ cnt4,
                                                    double* __restrict__ errp) {
  const int64_t P = parents_in(ctl, t, in.cap_nodes, in.cap_tasks);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->scratch[0] = P;
  const int lane = threadIdx.x & 63;
  const int64_t w = int64_t(2) << t;  // width of tier t+1
  for (int64_t p = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6); p < P;
       p += int64_t(gridDim.x) * kWaves) {
    const int32_t ij = in.nodes[p];
    const int I = unpack_i(ij), J = unpack_j(ij);
    const int64_t beg = in.nptr[p], end = in.nptr[p + 1];
    int32_t cq[4] = {0, 0, 0, 0};
    double e = 0.0;
    for (int64_t x0 = beg; x0 < end; x0 += 64) {
      const int64_t x = x0 + lane;
      uint32_t bits = 0;
      if (x < end) {
        double ce;
        bits = child_bits(na, nb, w, I, J, in.ks[x], tau, &ce);
        e += ce;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        cq[q] += __popcll(__ballot((bits >> (2 * q)) & 1)) +
                 __popcll(__ballot((bits >> (2 * q + 1)) & 1));
    }
    e = wave_sum(e);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) cnt4[4 * p + q] = cq[q];
      errp[p] = e;
    }
  }
}

__global__ void __launch_bounds__(256) k_cull_write(TierIn in, const double* __restrict__ na,
                                                    const double* __restrict__ nb, int t,
                                                    double tau, const Control* ctl,
                                                    const int32_t* __restrict__ cnt4,
                                                    const int64_t* __restrict__ toff,
                                                    const int32_t* __restrict__ noff,
                                                    int32_t* __restrict__ out_nodes,
                                                    int64_t* __restrict__ out_nptr,
                                                    int32_t* __restrict__ out_ks,
                                                    int64_t cap_nodes_out,
                                                    int64_t cap_tasks_out) {
  const int64_t P = ctl->scratch[0];
  const int64_t n_out = ctl->n_nodes[t + 1], k_out = ctl->n_tasks[t + 1];
  if (n_out > cap_nodes_out || k_out > cap_tasks_out) return;  // resumed with more room
  if (blockIdx.x == 0 && threadIdx.x == 0) out_nptr[n_out] = k_out;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int64_t w = int64_t(2) << t;
  for (int64_t p = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6); p < P;
       p += int64_t(gridDim.x) * kWaves) {
    const int32_t ij = in.nodes[p];
    const int I = unpack_i(ij), J = unpack_j(ij);
    int64_t pos[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pos[q] = toff[4 * p + q];
      if (lane == 0 && cnt4[4 * p + q] > 0) {
        const int32_t c = noff[4 * p + q];
        out_nodes[c] = pack_ij(2 * I + (q >> 1), 2 * J + (q & 1));
        out_nptr[c] = pos[q];
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
        bits = child_bits(na, nb, w, I, J, K, tau, &ce);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool p0 = (bits >> (2 * q)) & 1, p1 = (bits >> (2 * q + 1)) & 1;
        const uint64_t b0 = __ballot(p0), b1 = __ballot(p1);
        const int64_t at = pos[q] + __popcll(b0 & below) + __popcll(b1 & below);
        if (p0) out_ks[at] = 2 * K;
        if (p1) out_ks[at + (p0 ? 1 : 0)] = 2 * K + 1;
        pos[q] += __popcll(b0) + __popcll(b1);
      }
    }
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

inline int64_t pow_cap(int base_log2, int t, int64_t cap) {
  const int sh = base_log2 * t;
  if (sh >= 62) return cap;
  return std::min<int64_t>(int64_t(1) << sh, cap);
}

Error reserve_tier(CullWork& w, int t, hipStream_t s) {
  SPAMM_TRY(w.nodes[t].reserve(size_t(std::max<int64_t>(w.cap_nodes[t], 1)) * 4, s));
  SPAMM_TRY(w.nptr[t].reserve(size_t(w.cap_nodes[t] + 1) * 8, s));
  SPAMM_TRY(w.ks[t].reserve(size_t(std::max<int64_t>(w.cap_tasks[t], 1)) * 4, s));
  const int64_t need = 4 * std::max<int64_t>(w.cap_nodes[t], 1);
  if (need > w.cap_count) {
    SPAMM_TRY(w.cnt4.reserve(size_t(need) * 4, s));
    SPAMM_TRY(w.toff.reserve(size_t(need) * 8, s));
    SPAMM_TRY(w.noff.reserve(size_t(need) * 4, s));
    SPAMM_TRY(w.errp.reserve(size_t(need / 4) * 8, s));
    w.cap_count = need;
  }
  return Error{};
}

Error expand(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, int t, double tau,
             hipStream_t s) {
  TierIn in{static_cast<const int32_t*>(w.nodes[t].p), static_cast<const int64_t*>(w.nptr[t].p),
            static_cast<const int32_t*>(w.ks[t].p), w.cap_nodes[t], w.cap_tasks[t]};
  const double* na = a->norms + tier_offset(t + 1);
  const double* nb = b->norms + tier_offset(t + 1);
  const unsigned grid =
      unsigned(std::min<int64_t>((w.cap_nodes[t] + kWaves - 1) / kWaves, kMaxGrid));
  Control* ctl = w.ctl_dev;
  k_cull_count<<<grid, 256, 0, s>>>(in, na, nb, t, tau, ctl, static_cast<int32_t*>(w.cnt4.p),
                                    static_cast<double*>(w.errp.p));
  SPAMM_TRY(launch_scan(static_cast<const int32_t*>(w.cnt4.p), static_cast<int64_t*>(w.toff.p),
                        static_cast<int32_t*>(w.noff.p), static_cast<const double*>(w.errp.p),
                        &ctl->scratch[0], w.cap_nodes[t], 4, 0, &ctl->n_tasks[t + 1],
                        &ctl->n_nodes[t + 1], &ctl->err[t + 1], w.scan, s));
  k_cull_write<<<grid, 256, 0, s>>>(
      in, na, nb, t, tau, ctl, static_cast<const int32_t*>(w.cnt4.p),
      static_cast<const int64_t*>(w.toff.p), static_cast<const int32_t*>(w.noff.p),
      static_cast<int32_t*>(w.nodes[t + 1].p), static_cast<int64_t*>(w.nptr[t + 1].p),
      static_cast<int32_t*>(w.ks[t + 1].p), w.cap_nodes[t + 1], w.cap_tasks[t + 1]);
  return Error{};
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
  toff.release(s);
  noff.release(s);
  errp.release(s);
  scan.part.release(s);
  cap_count = 0;
  depth = -1;
}

CullWork::~CullWork() {
  // Device buffers are released by the owner on its stream; the control
  // block is synchronous memory.
  if (ctl_dev) (void)hipFree(ctl_dev);
  if (ctl_host) (void)hipHostFree(ctl_host);
}

Error run_cull(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
               bool want_pairs, hipStream_t s, CullResult* out) {
  const int d = a->depth;
  SPAMM_TRY(ensure_control(w));
  if (w.depth != d) {
    // First use at this depth: modest capacities, regrown on demand.
    for (int t = 0; t <= d; ++t) {
      w.cap_nodes[t] = std::max<int64_t>(1, pow_cap(2, t, int64_t(1) << 16));
      w.cap_tasks[t] = std::max<int64_t>(1, pow_cap(3, t, int64_t(1) << 18));
    }
    w.depth = d;
  }
  for (int t = 0; t <= d; ++t) SPAMM_TRY(reserve_tier(w, t, s));
  Control* ctl = w.ctl_dev;
  out->restarts = 0;
  {
    PhaseTimer timer(SPAMM_PHASE_CULL, s);
    k_cull_init<<<1, 1, 0, s>>>(ctl, d, static_cast<int32_t*>(w.nodes[0].p),
                                static_cast<int64_t*>(w.nptr[0].p), static_cast<int32_t*>(w.ks[0].p),
                                a->norms, b->norms, tau);
    for (int t = 0; t < d; ++t) SPAMM_TRY(expand(w, a, b, t, tau, s));
    if (want_pairs)
      k_nonzero_pairs<<<1, 1024, 0, s>>>(a->norms + tier_offset(d), b->norms + tier_offset(d),
                                         a->nb, ctl);
  }
  for (;;) {
    SPAMM_HIP(hipMemcpyAsync(w.ctl_host, ctl, sizeof(Control), hipMemcpyDeviceToHost, s));
    SPAMM_HIP(hipStreamSynchronize(s));
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
    for (int t = bad; t <= std::min(d, bad + 1); ++t) SPAMM_TRY(reserve_tier(w, t, s));
    ++out->restarts;
    PhaseTimer timer(SPAMM_PHASE_CULL, s);
    for (int t = bad - 1; t < d; ++t) SPAMM_TRY(expand(w, a, b, t, tau, s));
  }
  const Control& h = *w.ctl_host;
  out->n_cblocks = h.n_nodes[d];
  out->n_tasks = h.n_tasks[d];
  out->nonzero_pairs = want_pairs ? h.nonzero_pairs : -1;
  double e = 0.0;
  for (int t = 0; t <= d; ++t) e += h.err[t];
  out->err_bound = e;
  out->nodes = static_cast<const int32_t*>(w.nodes[d].p);
  out->nptr = static_cast<const int64_t*>(w.nptr[d].p);
  out->ks = static_cast<const int32_t*>(w.ks[d].p);
  return Error{};
}

}  // namespace spamm
