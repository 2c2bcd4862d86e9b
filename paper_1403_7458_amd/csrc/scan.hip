// Deterministic device-wide exclusive scan used for every compaction (block
// slots, culling frontiers).  Fixed grid of kParts workgroups, each owning a
// contiguous chunk; the length may live in device memory so that the host
// never waits for it.  Sums are in a fixed order, so results do not depend
// on timing.
#include "internal.h"

namespace spamm {

namespace {

constexpr int kParts = 256;
constexpr int kThreads = 256;

__device__ inline int64_t eff_len(const int64_t* len_dev, int64_t len_cap, int mult,
                                  int64_t len_host) {
  if (len_dev == nullptr) return len_host;
  const int64_t v = *len_dev;
  return (v >= 0 && v <= len_cap) ? v * mult : 0;
}

template <class V>
__device__ inline V block_sum(V v, V* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const V r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kThreads) k_scan_part(const int32_t* __restrict__ cnt,
                                                        const double* __restrict__ err,
                                                        const int64_t* len_dev, int64_t len_cap,
                                                        int mult, int64_t len_host,
                                                        int64_t* __restrict__ part) {
  __shared__ int64_t sh_i[kThreads];
  __shared__ double sh_d[kThreads];
  const int64_t L = eff_len(len_dev, len_cap, mult, len_host);
  const int64_t chunk = (L + kParts - 1) / kParts;
  const int64_t b0 = blockIdx.x * chunk, b1 = min(L, b0 + chunk);
  int64_t c = 0, z = 0;
  for (int64_t x = b0 + threadIdx.x; x < b1; x += kThreads) {
    const int32_t v = cnt[x];
    c += v;
    z += v > 0;
  }
  c = block_sum(c, sh_i);
  z = block_sum(z, sh_i);
  double e = 0.0;
  if (err != nullptr) {
    const int64_t Le = L / mult;
    const int64_t ch = (Le + kParts - 1) / kParts;
    const int64_t e0 = blockIdx.x * ch, e1 = min(Le, e0 + ch);
    for (int64_t x = e0 + threadIdx.x; x < e1; x += kThreads) e += err[x];
    e = block_sum(e, sh_d);
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = c;
    part[kParts + blockIdx.x] = z;
    reinterpret_cast<double*>(part + 2 * kParts)[blockIdx.x] = e;
  }
}

__global__ void __launch_bounds__(kParts) k_scan_top(int64_t* __restrict__ part,
                                                     int64_t* tot_cnt, int64_t* tot_nz,
                                                     double* tot_err) {
  __shared__ int64_t sc[kParts], sz[kParts];
  __shared__ double se[kParts];
  const int t = threadIdx.x;
  sc[t] = part[t];
  sz[t] = part[kParts + t];
  se[t] = reinterpret_cast<double*>(part + 2 * kParts)[t];
  __syncthreads();
  // Inclusive Hillis-Steele scan of the partial sums.
  for (int o = 1; o < kParts; o <<= 1) {
    const int64_t a = t >= o ? sc[t - o] : 0, b = t >= o ? sz[t - o] : 0;
    __syncthreads();
    sc[t] += a;
    sz[t] += b;
    __syncthreads();
  }
  part[t] = sc[t] - part[t];
  part[kParts + t] = sz[t] - part[kParts + t];
  for (int o = kParts / 2; o > 0; o >>= 1) {
    if (t < o) se[t] += se[t + o];
    __syncthreads();
  }
  if (t == 0) {
    if (tot_cnt) *tot_cnt = sc[kParts - 1];
    if (tot_nz) *tot_nz = sz[kParts - 1];
    if (tot_err) *tot_err = se[0];
  }
}

__device__ inline int64_t wave_incl_scan(int64_t v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

__global__ void __launch_bounds__(kThreads) k_scan_apply(const int32_t* __restrict__ cnt,
                                                         const int64_t* len_dev, int64_t len_cap,
                                                         int mult, int64_t len_host,
                                                         const int64_t* __restrict__ part,
                                                         int64_t* __restrict__ off_cnt,
                                                         int32_t* __restrict__ off_nz) {
  __shared__ int64_t wc[kThreads / 64], wz[kThreads / 64];
  const int64_t L = eff_len(len_dev, len_cap, mult, len_host);
  const int64_t chunk = (L + kParts - 1) / kParts;
  const int64_t b0 = blockIdx.x * chunk, b1 = min(L, b0 + chunk);
  int64_t base_c = part[blockIdx.x], base_z = part[kParts + blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t x0 = b0; x0 < b1; x0 += kThreads) {
    const int64_t x = x0 + threadIdx.x;
    const int32_t v = x < b1 ? cnt[x] : 0;
    int64_t ic = wave_incl_scan(v, lane);
    int64_t iz = wave_incl_scan(v > 0 ? 1 : 0, lane);
    if (lane == 63) {
      wc[wave] = ic;
      wz[wave] = iz;
    }
    __syncthreads();
    int64_t pc = 0, pz = 0, tc = 0, tz = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      if (w < wave) {
        pc += wc[w];
        pz += wz[w];
      }
      tc += wc[w];
      tz += wz[w];
    }
    if (x < b1) {
      if (off_cnt) off_cnt[x] = base_c + pc + ic - v;
      if (off_nz) off_nz[x] = int32_t(base_z + pz + iz - (v > 0 ? 1 : 0));
    }
    base_c += tc;
    base_z += tz;
    __syncthreads();
  }
}

}  // namespace

Error launch_scan(const int32_t* cnt, int64_t* off_cnt, int32_t* off_nz, const double* err,
                  const int64_t* len_dev, int64_t len_cap, int mult, int64_t len_host,
                  int64_t* tot_cnt, int64_t* tot_nz, double* tot_err, ScanWork& w,
                  hipStream_t s) {
  // part: kParts counts, kParts non-zero counts, kParts FP64 sums.
  SPAMM_TRY(w.part.reserve(3 * kParts * sizeof(int64_t), s));
  int64_t* part = static_cast<int64_t*>(w.part.p);
  k_scan_part<<<kParts, kThreads, 0, s>>>(cnt, err, len_dev, len_cap, mult, len_host, part);
  k_scan_top<<<1, kParts, 0, s>>>(part, tot_cnt, tot_nz, tot_err);
  k_scan_apply<<<kParts, kThreads, 0, s>>>(cnt, len_dev, len_cap, mult, len_host, part, off_cnt,
                                           off_nz);
  return Error{};
}

}  // namespace spamm
