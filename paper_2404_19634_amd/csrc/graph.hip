// Graph storage kernels: building the slack-padded CSR (the "holey" CSR of
// the paper's aggregation phase, Alg. 6, reused for in-place batch
// updates), relayout with more slack, weighted degrees (Section 3), and the
// per-arc / per-community terms of modularity (Eq. 1).
#include <map>
#include <mutex>
#include <tuple>

#include "lv_internal.hpp"

namespace lv {

int64_t resident_blocks(const void* kernel, int block, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INT32_MAX;
  const auto key = std::make_tuple(dev, kernel, block, lds);
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  int64_t r = INT32_MAX;  // unknown: no cap
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0 && cus > 0)
    r = static_cast<int64_t>(per_cu) * cus;
  cache[key] = r;
  return r;
}

int grid_for(int64_t items, int per_block, int max_blocks) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return static_cast<int>(b);
}

namespace {

__global__ void k_build_count(const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                              const int32_t* __restrict__ w, int64_t m, int32_t n,
                              int32_t* __restrict__ deg, int64_t* __restrict__ ctr) {
  int64_t wsum = 0;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < m;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t a = u[k], b = v[k], x = w[k];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b || x <= 0) {
      set_error(ctr, LV_EINVAL);
      continue;
    }
    atomicAdd(&deg[a], 1);
    atomicAdd(&deg[b], 1);
    wsum += 2 * static_cast<int64_t>(x);
  }
  wsum = wave_sum_i64(wsum);
  if (lane_id() == 0 && wsum) atomic_add_i64(&ctr[CTR_TOTAL], wsum);
}

__global__ void k_row_capacity(const int32_t* __restrict__ deg, int64_t* __restrict__ capv, int32_t n,
                               float frac, int32_t smin) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t d = deg[i];
    int64_t s = static_cast<int64_t>(ceilf(frac * static_cast<float>(d)));
    if (s < smin) s = smin;
    capv[i] = d + s;
  }
}

__global__ void k_build_scatter(const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                const int32_t* __restrict__ w, int64_t m,
                                const int64_t* __restrict__ row_start, int32_t* __restrict__ row_len,
                                int32_t* __restrict__ col, int32_t* __restrict__ wt,
                                int64_t* __restrict__ two_m) {
  int64_t wsum = 0;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < m;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t a = u[k], b = v[k], x = w[k];
    const int64_t pa = row_start[a] + atomicAdd(&row_len[a], 1);
    col[pa] = b;
    wt[pa] = x;
    const int64_t pb = row_start[b] + atomicAdd(&row_len[b], 1);
    col[pb] = a;
    wt[pb] = x;
    wsum += 2 * static_cast<int64_t>(x);
  }
  wsum = wave_sum_i64(wsum);
  if (lane_id() == 0 && wsum) atomic_add_i64(two_m, wsum);
}

// One wavefront copies one row (rows handed out grid-stride).
__global__ void k_relayout_copy(const int64_t* __restrict__ s_start, const int32_t* __restrict__ s_len,
                                const int32_t* __restrict__ s_col, const int32_t* __restrict__ s_w,
                                int32_t n, const int64_t* __restrict__ d_start, int32_t* __restrict__ d_len,
                                int32_t* __restrict__ d_col, int32_t* __restrict__ d_w) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t i = wave; i < n; i += nwaves) {
    const int64_t a = s_start[i], b = d_start[i];
    const int32_t len = s_len[i];
    for (int32_t k = lane; k < len; k += kWave) {
      d_col[b + k] = s_col[a + k];
      d_w[b + k] = s_w[a + k];
    }
    if (lane == 0) d_len[i] = len;
  }
}

// Row sums: a group of 16 lanes per row for rows of up to 1024 arcs; longer
// rows are listed and summed by a whole workgroup each.  With C given, also
// the total weight of arcs whose endpoints share a community (modularity).
constexpr int kRowGroup = 16;
constexpr int kRowGroupMax = 1024;

__global__ void __launch_bounds__(kBlock) k_rows_group(const int64_t* __restrict__ row_start,
                                                      const int32_t* __restrict__ row_len,
                                                      const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                      int32_t n, const int32_t* __restrict__ C, int64_t* __restrict__ K,
                                                      int64_t* __restrict__ Sigma, int32_t* __restrict__ Cinit,
                                                      int32_t* __restrict__ size, int32_t* __restrict__ longlist,
                                                      int64_t* __restrict__ ctr) {
  const int lane = lane_id();
  const int sub = lane % kRowGroup;
  const int64_t first = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kRowGroup;
  const int64_t ngroups = static_cast<int64_t>(gridDim.x) * blockDim.x / kRowGroup;
  int64_t intra = 0;
  for (int64_t i = first; i < n; i += ngroups) {
    const int32_t len = row_len[i];
    if (len > kRowGroupMax) {
      if (sub == 0) {
        const int64_t pos = static_cast<int64_t>(
            atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_AUX1]), 1ull));
        longlist[pos] = static_cast<int32_t>(i);
      }
      continue;
    }
    const int64_t s = row_start[i];
    const int32_t ci = C ? C[i] : 0;
    int64_t acc = 0, in = 0;
    // four arcs per lane per step, loads first, so their latencies overlap
    for (int32_t k0 = sub; k0 < len; k0 += 4 * kRowGroup) {
      int32_t x[4], c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = k0 + q * kRowGroup < len ? wt[s + k0 + q * kRowGroup] : 0;
      if (C) {
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = k0 + q * kRowGroup < len ? col[s + k0 + q * kRowGroup] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = c[q] >= 0 ? C[c[q]] : ci - 1;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc += x[q];
        if (C && c[q] == ci) in += x[q];
      }
    }
#pragma unroll
    for (int q = 1; q < kRowGroup; q <<= 1) acc += __shfl_xor(acc, q);
    intra += in;
    if (sub == 0) {
      K[i] = acc;
      if (Sigma) Sigma[i] = acc;
      if (Cinit) Cinit[i] = static_cast<int32_t>(i);
      if (size) size[i] = 1;
    }
  }
  intra = wave_sum_i64(intra);
  if (lane == 0 && C && intra) stat_add(ctr + CTR_STATS0, ST_INTRA, intra);
}

__global__ void __launch_bounds__(kBlock) k_rows_long(const int64_t* __restrict__ row_start,
                                                     const int32_t* __restrict__ row_len,
                                                     const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                     const int32_t* __restrict__ C, int64_t* __restrict__ K,
                                                     int64_t* __restrict__ Sigma, int32_t* __restrict__ Cinit,
                                                     int32_t* __restrict__ size, const int32_t* __restrict__ longlist,
                                                     int64_t* __restrict__ ctr) {
  __shared__ int64_t r[kBlock / kWave];
  const int64_t count = ctr[CTR_AUX1];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int64_t intra = 0;
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t i = longlist[idx];
    const int64_t s = row_start[i];
    const int32_t len = row_len[i];
    const int32_t ci = C ? C[i] : 0;
    int64_t acc = 0;
    for (int32_t k = threadIdx.x; k < len; k += kBlock) {
      const int32_t x = wt[s + k];
      acc += x;
      if (C && C[col[s + k]] == ci) intra += x;
    }
    acc = wave_sum_i64(acc);
    if (lane == 0) r[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int q = 0; q < kBlock / kWave; ++q) t += r[q];
      K[i] = t;
      if (Sigma) Sigma[i] = t;
      if (Cinit) Cinit[i] = i;
      if (size) size[i] = 1;
    }
    __syncthreads();
  }
  intra = wave_sum_i64(intra);
  if (lane == 0 && C && intra) stat_add(ctr + CTR_STATS0, ST_INTRA, intra);
}

__global__ void k_sum_squares(const int64_t* __restrict__ v, int32_t n, int64_t* __restrict__ out) {
  int64_t s = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t x = v[i];
    s += x * x;
  }
  s = wave_sum_i64(s);
  if (lane_id() == 0 && s) atomic_add_i64(out, s);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_iota_i32(int32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = static_cast<int32_t>(i);
}

__global__ void k_set_all_bits(uint32_t* __restrict__ bm, int32_t n) {
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < words;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t hi = (k + 1) * 32;
    bm[k] = hi <= n ? 0xFFFFFFFFu : ((1u << (n - k * 32)) - 1u);
  }
}

__global__ void k_copy_bits(const uint32_t* __restrict__ s, uint32_t* __restrict__ d, int64_t words) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < words;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    d[k] = s[k];
}

}  // namespace

void launch_build_count(const lv_edges& e, int32_t n, int32_t* deg, int64_t* ctr, hipStream_t st) {
  if (e.count == 0) return;
  hipLaunchKernelGGL(k_build_count, dim3(grid_for(e.count, kBlock, 8192)), dim3(kBlock), 0, st, e.u, e.v,
                     e.w, e.count, n, deg, ctr);
}

void launch_row_capacity(const int32_t* deg, int64_t* capv, int32_t n, float frac, int32_t smin,
                         hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_row_capacity, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, deg, capv, n,
                     frac, smin);
}

void launch_build_scatter(const lv_edges& e, const int64_t* row_start, int32_t* row_len, int32_t* col,
                          int32_t* w, int64_t* two_m, hipStream_t st) {
  if (e.count == 0) return;
  hipLaunchKernelGGL(k_build_scatter, dim3(grid_for(e.count, kBlock, 8192)), dim3(kBlock), 0, st, e.u,
                     e.v, e.w, e.count, row_start, row_len, col, w, two_m);
}

void launch_relayout_copy(const lv_graph& src, const int64_t* dst_start, int32_t* dst_len,
                          int32_t* dst_col, int32_t* dst_w, hipStream_t st) {
  if (src.n == 0) return;
  hipLaunchKernelGGL(k_relayout_copy, dim3(grid_for(static_cast<int64_t>(src.n) * kWave, kBlock, 8192)),
                     dim3(kBlock), 0, st, src.row_start, src.row_len, src.col, src.w, src.n, dst_start,
                     dst_len, dst_col, dst_w);
}

// K[i] = row sum (and Sigma = K, C = identity, size = 1 when given); with
// C_mod given, ctr[CTR_AUX0] += weight of intra-community arcs.  Uses
// ctr[CTR_AUX1] and `longlist` (n entries) as scratch.
void launch_row_sums(const LevelGraph& g, const int32_t* C_mod, int64_t* K, int64_t* Sigma, int32_t* Cinit,
                     int32_t* size, int32_t* longlist, int64_t* ctr, hipStream_t st) {
  if (g.n == 0) return;
  (void)hipMemsetAsync(ctr + CTR_AUX1, 0, sizeof(int64_t), st);
  hipLaunchKernelGGL(k_rows_group, dim3(grid_for(static_cast<int64_t>(g.n) * kRowGroup, kBlock, 8192)),
                     dim3(kBlock), 0, st, g.row_start, g.row_len, g.col, g.w, g.n, C_mod, K, Sigma, Cinit, size,
                     longlist, ctr);
  hipLaunchKernelGGL(k_rows_long, dim3(1024), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col, g.w, C_mod, K,
                     Sigma, Cinit, size, longlist, ctr);
}

void launch_sum_squares(const int64_t* v, int32_t n, int64_t* out, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_sum_squares, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, v, n, out);
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, p, v, n);
}

void launch_iota_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, p, n);
}

void launch_set_all_bits(uint32_t* bm, int32_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_set_all_bits, dim3(grid_for((n + 31) / 32, kBlock, 8192)), dim3(kBlock), 0, st, bm,
                     n);
}

void launch_copy_bits(const uint32_t* src, uint32_t* dst, int64_t words, hipStream_t st) {
  if (words <= 0) return;
  hipLaunchKernelGGL(k_copy_bits, dim3(grid_for(words, kBlock, 8192)), dim3(kBlock), 0, st, src, dst, words);
}

}  // namespace lv
