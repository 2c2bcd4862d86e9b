// Quadtree construction: ingest of a dense FP64 matrix into 32 x 32 tiles,
// FP64 leaf norms (Eq. 2), the tier pyramid (Eq. 3), Gershgorin scaling for
// SP2 and the dense read-back.  All kernels here are bandwidth-bound: each
// 64-lane wave owns one 32 x 32 block and touches it in 128-byte row segments.
#include <cmath>

#include "half.h"
#include "internal.h"

namespace spamm {

namespace {

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Scaled input value (diag * [i == j] + sign * a_ij) / div; see Scale.
__device__ inline double scaled(const double* a, int64_t lda, int64_t r, int64_t c,
                                const Scale& sc) {
  double v = sc.sign * a[r * lda + c];
  if (r == c) v = sc.diag + v;
  return v / sc.div;
}

__global__ void __launch_bounds__(256) k_leaf_norms_dense(const double* __restrict__ a,
                                                          int64_t lda, int64_t n, int nb,
                                                          double* __restrict__ leaf,
                                                          Scale* scale) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (blk >= int64_t(nb) * nb) return;
  const int bi = int(blk / nb), bj = int(blk % nb);
  const Scale sc = *scale;
  double s = 0.0, mx = 0.0;
  bool bad = false;
  const int64_t r0 = int64_t(bi) * kLeaf, c = int64_t(bj) * kLeaf + (lane & 31);
  if (r0 < n && int64_t(bj) * kLeaf < n) {
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
      const int64_t r = r0 + rr * 2 + (lane >> 5);
      if (r < n && c < n) {
        const double v = scaled(a, lda, r, c, sc);
        bad |= !isfinite(v);
        s += v * v;
        mx = fmax(mx, fabs(v));
      }
    }
  }
  s = wave_sum(s);
  mx = wave_max(mx);
  if (bad) scale->nonfinite = 1;
  if (lane == 0) {
    leaf[blk] = sqrt(s);
    // One address for every block: skip the atomic when the running maximum
    // (which only grows) already covers this block, so that the blocks do
    // not queue up behind each other on it.
    if (mx > 0.0 && mx > *reinterpret_cast<volatile const double*>(&scale->max_val))
      atomicMax(reinterpret_cast<unsigned long long*>(&scale->max_val),
                static_cast<unsigned long long>(__double_as_longlong(mx)));
  }
}

__global__ void k_nonzero_flags(const double* __restrict__ leaf, int64_t m,
                                int32_t* __restrict__ flag) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x < m) flag[x] = leaf[x] != 0.0 ? 1 : 0;
}

__global__ void k_scatter_slots(const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                                int64_t m, int nb, int32_t* __restrict__ map,
                                int32_t* __restrict__ coords) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= m) return;
  if (flag[x]) {
    map[x] = off[x];
    coords[off[x]] = pack_ij(int(x / nb), int(x % nb));
  } else {
    map[x] = -1;
  }
}

template <class T>
__global__ void __launch_bounds__(256) k_write_tiles(const double* __restrict__ a, int64_t lda,
                                                     int64_t n, int64_t n_blocks,
                                                     const int32_t* __restrict__ coords,
                                                     T* __restrict__ pool, const Scale* scale,
                                                     double* __restrict__ trace_part) {
  const int lane = threadIdx.x & 63;
  const int64_t slot = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (slot >= n_blocks) return;
  const int32_t ij = coords[slot];
  const int bi = unpack_i(ij), bj = unpack_j(ij);
  const Scale sc = *scale;
  T* tile = pool + slot * kLeaf2;
  double tr = 0.0;
  const int col = lane & 31;
#pragma unroll 4
  for (int rr = 0; rr < 16; ++rr) {
    const int row = rr * 2 + (lane >> 5);
    const int64_t r = int64_t(bi) * kLeaf + row, c = int64_t(bj) * kLeaf + col;
    const T v = (r < n && c < n) ? T(scaled(a, lda, r, c, sc)) : T(0);
    tile[row * kLeaf + col] = v;
    if (bi == bj && row == col) tr += double(v);
  }
  if (trace_part != nullptr && bi == bj) {
    tr = wave_sum(tr);
    if (lane == 0) trace_part[bi] = tr;
  }
}

// 16-bit forms: hi (+ lo) and their transposes (layout in half.h).
template <int P>
__global__ void __launch_bounds__(256) k_write_tiles_half(const double* __restrict__ a, int64_t lda,
                                                          int64_t n, int64_t n_blocks,
                                                          const int32_t* __restrict__ coords,
                                                          void* __restrict__ pool_v,
                                                          const Scale* scale,
                                                          double* __restrict__ trace_part) {
  typedef typename Half<P>::T T;
  const int lane = threadIdx.x & 63;
  const int64_t slot = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (slot >= n_blocks) return;
  const int32_t ij = coords[slot];
  const int bi = unpack_i(ij), bj = unpack_j(ij);
  const Scale sc = *scale;
  T* tile = static_cast<T*>(pool_v) + slot * (is_split(P) ? 4 : 2) * kLeaf2;
  double tr = 0.0;
  const int col = lane & 31;
#pragma unroll 4
  for (int rr = 0; rr < 16; ++rr) {
    const int row = rr * 2 + (lane >> 5);
    const int64_t r = int64_t(bi) * kLeaf + row, c = int64_t(bj) * kLeaf + col;
    T hi, lo;
    encode_half<P>((r < n && c < n) ? scaled(a, lda, r, c, sc) : 0.0, hi, lo);
    const int rc = half_idx(row, col), cr = half_idx(col, row);
    tile[rc] = hi;
    tile[half_part(1) + cr] = hi;
    if (is_split(P)) {
      tile[half_part(2) + rc] = lo;
      tile[half_part(3) + cr] = lo;
    }
    if (bi == bj && row == col) tr += decode_half<P>(hi, lo);
  }
  if (trace_part != nullptr && bi == bj) {
    tr = wave_sum(tr);
    if (lane == 0) trace_part[bi] = tr;
  }
}

template <int P>
__global__ void __launch_bounds__(256) k_to_dense_half(const void* __restrict__ pool_v,
                                                       const int32_t* __restrict__ map, int nb,
                                                       int64_t n, int nbr, double* __restrict__ out,
                                                       int64_t ld) {
  typedef typename Half<P>::T T;
  const int lane = threadIdx.x & 63;
  const int64_t blk = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (blk >= int64_t(nbr) * nbr) return;
  const int bi = int(blk / nbr), bj = int(blk % nbr);
  const int32_t slot = map[int64_t(bi) * nb + bj];
  const T* tile =
      slot >= 0 ? static_cast<const T*>(pool_v) + int64_t(slot) * (is_split(P) ? 4 : 2) * kLeaf2
                : nullptr;
  const int col = lane & 31;
#pragma unroll 4
  for (int rr = 0; rr < 16; ++rr) {
    const int row = rr * 2 + (lane >> 5);
    const int64_t r = int64_t(bi) * kLeaf + row, c = int64_t(bj) * kLeaf + col;
    if (r < n && c < n)
      out[r * ld + c] =
          tile ? decode_half<P>(tile[half_idx(row, col)],
                                is_split(P) ? tile[half_part(2) + half_idx(row, col)] : T(0.0f))
               : 0.0;
  }
}

__global__ void k_pyramid_level(double* __restrict__ norms, int t) {
  const int64_t w = int64_t(1) << t;
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= w * w) return;
  const double* ch = norms + tier_offset(t + 1);
  norms[tier_offset(t) + x] = parent_norm(ch, 2 * w, x / w, x % w);
}

__global__ void __launch_bounds__(1024) k_pyramid_top(double* __restrict__ norms, int t_top) {
  pyramid_tiers(norms, t_top);
}

// Gershgorin discs per row: one wave per row.
__global__ void __launch_bounds__(256) k_gershgorin_rows(const double* __restrict__ f, int64_t n,
                                                         int64_t ldf, double* __restrict__ lo,
                                                         double* __restrict__ hi,
                                                         double* __restrict__ rmax,
                                                         Scale* scale) {
  const int lane = threadIdx.x & 63;
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* row = f + i * ldf;
  double r = 0.0, m = 0.0;
  bool bad = false;
  for (int64_t j = lane; j < n; j += 64) {
    const double v = row[j];
    bad |= !isfinite(v);
    m = fmax(m, fabs(v));
    if (j != i) r += fabs(v);
  }
  r = wave_sum(r);
  m = wave_max(m);
  if (bad) scale->nonfinite = 1;
  if (lane == 0) {
    const double d = row[i];
    lo[i] = d - r;
    hi[i] = d + r;
    rmax[i] = m;
  }
}

__global__ void __launch_bounds__(1024) k_scale_finish(const double* __restrict__ lo,
                                                        const double* __restrict__ hi,
                                                        const double* __restrict__ rmax, int64_t n,
                                                        Scale* scale) {
  __shared__ double s_lo[1024], s_hi[1024], s_m[1024];
  double a = INFINITY, b = -INFINITY, m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    a = fmin(a, lo[i]);
    b = fmax(b, hi[i]);
    m = fmax(m, rmax[i]);
  }
  s_lo[threadIdx.x] = a;
  s_hi[threadIdx.x] = b;
  s_m[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + o]);
      s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + o]);
      s_m[threadIdx.x] = fmax(s_m[threadIdx.x], s_m[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double emin = s_lo[0], emax = s_hi[0];
    const double width = emax - emin;
    scale->max_abs = s_m[0];
    scale->eps_min = emin;
    scale->eps_max = emax;
    if (!(width > 0.0) || !isfinite(width)) {
      scale->bad_bounds = 1;
      scale->diag = 0.0;
      scale->sign = 0.0;
      scale->div = 1.0;
      return;
    }
    // X_0 = (eps_max I - F) / (eps_max - eps_min), zero outside the n x n block.
    scale->diag = emax;
    scale->sign = -1.0;
    scale->div = width;
  }
}

// max |F_ij - F_ji| over one block pair, folded with atomicMax on the bit
// pattern (non-negative doubles order like their bits).
__global__ void __launch_bounds__(256) k_asymmetry(const double* __restrict__ f, int64_t n,
                                                   int64_t ldf, int nbr, Scale* scale) {
  __shared__ double t[kLeaf][kLeaf + 1];
  const int bi = blockIdx.x / nbr, bj = blockIdx.x % nbr;
  if (bi > bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows per pass
  for (int rr = ty; rr < kLeaf; rr += 8) {
    const int64_t r = int64_t(bj) * kLeaf + rr, c = int64_t(bi) * kLeaf + tx;
    t[rr][tx] = (r < n && c < n) ? f[r * ldf + c] : 0.0;
  }
  __syncthreads();
  double m = 0.0;
  for (int rr = ty; rr < kLeaf; rr += 8) {
    const int64_t r = int64_t(bi) * kLeaf + rr, c = int64_t(bj) * kLeaf + tx;
    if (r < n && c < n) m = fmax(m, fabs(f[r * ldf + c] - t[tx][rr]));
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0 && m > 0.0)
    atomicMax(reinterpret_cast<unsigned long long*>(&scale->max_asym),
              static_cast<unsigned long long>(__double_as_longlong(m)));
}

__global__ void k_init_scale(Scale* s) {
  s->diag = 0.0;
  s->sign = 1.0;
  s->div = 1.0;
  s->eps_min = 0.0;
  s->eps_max = 0.0;
  s->max_abs = 0.0;
  s->max_asym = 0.0;
  s->max_val = 0.0;
  s->nonfinite = 0;
  s->bad_bounds = 0;
}

template <class T>
__global__ void __launch_bounds__(256) k_to_dense(const T* __restrict__ pool,
                                                  const int32_t* __restrict__ map, int nb,
                                                  int64_t n, int nbr, double* __restrict__ out,
                                                  int64_t ld) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (blk >= int64_t(nbr) * nbr) return;
  const int bi = int(blk / nbr), bj = int(blk % nbr);
  const int32_t slot = map[int64_t(bi) * nb + bj];
  const T* tile = slot >= 0 ? pool + int64_t(slot) * kLeaf2 : nullptr;
  const int col = lane & 31;
#pragma unroll 4
  for (int rr = 0; rr < 16; ++rr) {
    const int row = rr * 2 + (lane >> 5);
    const int64_t r = int64_t(bi) * kLeaf + row, c = int64_t(bj) * kLeaf + col;
    if (r < n && c < n) out[r * ld + c] = tile ? double(tile[row * kLeaf + col]) : 0.0;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < n;
       x += int64_t(gridDim.x) * blockDim.x)
    p[x] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < n;
       x += int64_t(gridDim.x) * blockDim.x)
    p[x] = v;
}

inline unsigned grid_for(int64_t items, int per_block) {
  return unsigned((items + per_block - 1) / per_block);
}

}  // namespace

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = unsigned(std::min<int64_t>((n + 255) / 256, 8192));
  k_fill_i32<<<g, 256, 0, s>>>(p, n, v);
}
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = unsigned(std::min<int64_t>((n + 255) / 256, 8192));
  k_fill_f64<<<g, 256, 0, s>>>(p, n, v);
}

void launch_init_scale(Scale* scale, hipStream_t s) { k_init_scale<<<1, 1, 0, s>>>(scale); }

void launch_leaf_norms_dense(const double* a, int64_t lda, const spamm_matrix* m, Scale* scale,
                             hipStream_t s) {
  const int64_t blocks = int64_t(m->nb) * m->nb;
  k_leaf_norms_dense<<<grid_for(blocks, 4), 256, 0, s>>>(
      a, lda, m->n, m->nb, m->norms + tier_offset(m->depth), scale);
}

Error compact_nonzero_blocks(spamm_matrix* m, int64_t* count_dev, hipStream_t s) {
  const int64_t cells = int64_t(m->nb) * m->nb;
  if (m->coords == nullptr) SPAMM_TRY(dev_alloc_n(&m->coords, cells, s));
  int32_t* flag = nullptr;
  int32_t* off = nullptr;
  int64_t* off_cnt = nullptr;
  SPAMM_TRY(dev_alloc_n(&flag, cells, s));
  Error e = dev_alloc_n(&off, cells, s);
  if (e.ok()) e = dev_alloc_n(&off_cnt, cells, s);
  if (!e.ok()) {
    dev_free(flag, s);
    dev_free(off, s);
    return e;
  }
  k_nonzero_flags<<<grid_for(cells, 256), 256, 0, s>>>(m->norms + tier_offset(m->depth), cells,
                                                        flag);
  ScanWork w;
  e = launch_scan(flag, off_cnt, off, nullptr, nullptr, 0, 1, cells, count_dev + 1, count_dev,
                  nullptr, w, s);
  if (!e.ok()) {
    dev_free(flag, s);
    dev_free(off, s);
    dev_free(off_cnt, s);
    return e;
  }
  k_scatter_slots<<<grid_for(cells, 256), 256, 0, s>>>(flag, off, cells, m->nb, m->map,
                                                        m->coords);
  w.part.release(s);
  dev_free(flag, s);
  dev_free(off, s);
  dev_free(off_cnt, s);
  return Error{};
}

void launch_write_tiles(const double* a, int64_t lda, const spamm_matrix* m, const Scale* scale,
                        double* trace_part, hipStream_t s) {
  if (m->n_blocks == 0) return;
  const unsigned g = grid_for(m->n_blocks, 4);
  switch (m->prec) {
    case SPAMM_BF16:
      k_write_tiles_half<SPAMM_BF16><<<g, 256, 0, s>>>(a, lda, m->n, m->n_blocks, m->coords, m->pool,
                                                       scale, trace_part);
      return;
    case SPAMM_FP16:
      k_write_tiles_half<SPAMM_FP16><<<g, 256, 0, s>>>(a, lda, m->n, m->n_blocks, m->coords, m->pool,
                                                       scale, trace_part);
      return;
    case SPAMM_BF16X3:
      k_write_tiles_half<SPAMM_BF16X3><<<g, 256, 0, s>>>(a, lda, m->n, m->n_blocks, m->coords,
                                                         m->pool, scale, trace_part);
      return;
    case SPAMM_FP16X3:
      k_write_tiles_half<SPAMM_FP16X3><<<g, 256, 0, s>>>(a, lda, m->n, m->n_blocks, m->coords,
                                                         m->pool, scale, trace_part);
      return;
    default:
      break;
  }
  if (m->prec == SPAMM_FP64)
    k_write_tiles<double><<<g, 256, 0, s>>>(a, lda, m->n, m->n_blocks, m->coords,
                                            static_cast<double*>(m->pool), scale, trace_part);
  else
    k_write_tiles<float><<<g, 256, 0, s>>>(a, lda, m->n, m->n_blocks, m->coords,
                                           static_cast<float*>(m->pool), scale, trace_part);
}

int launch_pyramid(const spamm_matrix* m, hipStream_t s, bool leave_top) {
  PhaseTimer timer(SPAMM_PHASE_PYRAMID, s);
  // Tiers of up to 4^6 nodes go to the single-workgroup kernel (4 nodes per
  // thread): one launch instead of one per tier for trees of depth <= 7.
  int t = m->depth - 1;
  for (; t > 6; --t) {
    const int64_t w2 = int64_t(1) << (2 * t);
    k_pyramid_level<<<grid_for(w2, 256), 256, 0, s>>>(m->norms, t);
  }
  if (t < 0) return -1;
  if (leave_top) return t;
  k_pyramid_top<<<1, 1024, 0, s>>>(m->norms, t);
  return -1;
}

void launch_gershgorin_scale(const double* f, int64_t n, int64_t ldf, double* row_lo,
                             double* row_hi, double* row_max, Scale* scale, hipStream_t s) {
  k_gershgorin_rows<<<grid_for(n, 4), 256, 0, s>>>(f, n, ldf, row_lo, row_hi, row_max, scale);
  k_scale_finish<<<1, 1024, 0, s>>>(row_lo, row_hi, row_max, n, scale);
}

void launch_asymmetry(const double* f, int64_t n, int64_t ldf, Scale* scale, hipStream_t s) {
  const int nbr = int((n + kLeaf - 1) / kLeaf);
  k_asymmetry<<<unsigned(int64_t(nbr) * nbr), 256, 0, s>>>(f, n, ldf, nbr, scale);
}

void launch_to_dense(const spamm_matrix* m, double* out, int64_t ld, hipStream_t s) {
  PhaseTimer timer(SPAMM_PHASE_DENSE, s);
  const int nbr = int((m->n + kLeaf - 1) / kLeaf);
  const unsigned g = grid_for(int64_t(nbr) * nbr, 4);
  switch (m->prec) {
    case SPAMM_BF16:
      k_to_dense_half<SPAMM_BF16><<<g, 256, 0, s>>>(m->pool, m->map, m->nb, m->n, nbr, out, ld);
      return;
    case SPAMM_FP16:
      k_to_dense_half<SPAMM_FP16><<<g, 256, 0, s>>>(m->pool, m->map, m->nb, m->n, nbr, out, ld);
      return;
    case SPAMM_BF16X3:
      k_to_dense_half<SPAMM_BF16X3><<<g, 256, 0, s>>>(m->pool, m->map, m->nb, m->n, nbr, out, ld);
      return;
    case SPAMM_FP16X3:
      k_to_dense_half<SPAMM_FP16X3><<<g, 256, 0, s>>>(m->pool, m->map, m->nb, m->n, nbr, out, ld);
      return;
    default:
      break;
  }
  if (m->prec == SPAMM_FP64)
    k_to_dense<double><<<g, 256, 0, s>>>(static_cast<const double*>(m->pool), m->map, m->nb,
                                         m->n, nbr, out, ld);
  else
    k_to_dense<float><<<g, 256, 0, s>>>(static_cast<const float*>(m->pool), m->map, m->nb,
                                        m->n, nbr, out, ld);
}

}  // namespace spamm
