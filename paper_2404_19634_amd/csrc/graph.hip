// Graph storage kernels: building the slack-padded CSR (the "holey" CSR of
// the paper's aggregation phase, Alg. 6, reused for in-place batch
// updates), relayout with more slack, weighted degrees (Section 3), and the
// per-arc / per-community terms of modularity (Eq. 1).
#include <algorithm>
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

// Row sums (K_i, and with C given the weight of arcs inside communities
// for Eq. 1) by row length, so that every lane has loads in flight and no
// wavefront walks a long row alone:
//  - rows of at most kLaneMax arcs: each lane sums its own row, all of its
//    loads issued at once (one memory round trip);
//  - rows up to kGroupMax arcs: listed, then 16 lanes per row (four rows per
//    wavefront at a time);
//  - rows up to kMidMax arcs: listed, then one wavefront per row, the next
//    row's metadata loaded before this row's arcs are summed;
//  - longer rows are listed in chunks of kChunk arcs, one wavefront per
//    chunk, whose partial sums are added atomically (K and Sigma of such a
//    row are zeroed by the first kernel).
// The lists are kept per region (row task mod kRegions), each region with
// its own counters, so a workgroup reserves its entries with one atomic per
// class on a counter shared with few others.
constexpr int kLaneMax = 16;
constexpr int kGroupMax = 64;
constexpr int kMidMax = 4096;
constexpr int kRegions = 32;
constexpr int kChunk = 4096;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kRowUnroll = 4;

struct RowSumOut {
  int64_t* K;
  int64_t* Sigma;  // = K (static start), or null
  int32_t* Cinit;  // identity, or null
  int32_t* size;   // all ones, or null
  int32_t* lrow;   // chunks of long rows: row, first arc
  int32_t* loff;
  int64_t* ctr;    // CTR_AUX1: listed chunks
  int32_t* grp;    // group rows, region r at grp[r * cap ...]
  int32_t* mid;    // wavefront rows, likewise
  int64_t cap;     // list entries per region
  int64_t* cnt;    // region r's counts: cnt[(2r) * kCtrLine] (group), cnt[(2r + 1) * kCtrLine] (wavefront)
};


// Sum of arcs [a, b) of the row starting at s, over the wavefront, 256 arcs
// per step; with C, adds the weight of arcs into community ci to *intra.
__device__ __forceinline__ int64_t wave_row_sum(const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                const int32_t* __restrict__ C, int64_t s, int32_t a, int32_t b,
                                                int32_t ci, int64_t* intra) {
  const int lane = lane_id();
  int64_t acc = 0;
  for (int32_t k0 = a + lane; k0 < b; k0 += kWave * kRowUnroll) {
    int32_t x[kRowUnroll], j[kRowUnroll];
#pragma unroll
    for (int q = 0; q < kRowUnroll; ++q) {
      const int32_t k = k0 + q * kWave;
      x[q] = k < b ? wt[s + k] : 0;
      j[q] = (C && k < b) ? col[s + k] : -1;
    }
#pragma unroll
    for (int q = 0; q < kRowUnroll; ++q) {
      acc += x[q];
      if (C && j[q] >= 0 && C[j[q]] == ci) *intra += x[q];
    }
  }
  return wave_sum_i64(acc);
}

__global__ void __launch_bounds__(kBlock) k_rows_flat(const int64_t* __restrict__ row_start,
                                                     const int32_t* __restrict__ row_len,
                                                     const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                     int32_t n, const int32_t* __restrict__ C, RowSumOut o) {
  __shared__ int32_t s_n[2];
  __shared__ int64_t s_b[2];
  const int lane = lane_id();
  int64_t intra = 0;
  const int64_t tasks = (static_cast<int64_t>(n) + kBlock - 1) / kBlock;
  for (int64_t t = blockIdx.x; t < tasks; t += gridDim.x) {
    const int region = static_cast<int>(t % kRegions);
    if (threadIdx.x < 2) s_n[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = t * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int32_t len = valid ? row_len[i] : 0;
    const int64_t st = valid ? row_start[i] : 0;
    const int32_t ci = (C && valid) ? C[i] : 0;
    const bool is_long = len > kMidMax;
    const bool is_mid = len > kGroupMax && !is_long;
    const bool is_grp = len > kLaneMax && len <= kGroupMax;
    {  // chunks of long rows, reserved together by the wavefront
      const int32_t nch = is_long ? (len + kChunk - 1) / kChunk : 0;
      int32_t incl = nch;
      for (int s = 1; s < kWave; s <<= 1) {
        const int32_t u = __shfl_up(incl, s);
        if (lane >= s) incl += u;
      }
      const int32_t tot = __shfl(incl, kWave - 1);
      int64_t base = 0;
      if (tot > 0) {
        if (lane == 0)
          base = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&o.ctr[CTR_AUX1]),
                                                static_cast<unsigned long long>(tot)));
        base = __shfl(base, 0);
      }
      for (int32_t k = 0; k < nch; ++k) {
        o.lrow[base + incl - nch + k] = static_cast<int32_t>(i);
        o.loff[base + incl - nch + k] = k * kChunk;
      }
    }
    // the group and wavefront rows: LDS counts, one reservation per class
    int32_t pg = -1, pm = -1;
    if (is_grp) pg = atomicAdd(&s_n[0], 1);
    if (is_mid) pm = atomicAdd(&s_n[1], 1);
    __syncthreads();
    if (threadIdx.x < 2) {
      const int32_t c = s_n[threadIdx.x];
      s_b[threadIdx.x] = c ? static_cast<int64_t>(atomicAdd(
                                 reinterpret_cast<unsigned long long*>(&o.cnt[(region * 2 + threadIdx.x) * kCtrLine]),
                                 static_cast<unsigned long long>(c)))
                           : 0;
    }
    __syncthreads();
    if (pg >= 0) o.grp[region * o.cap + s_b[0] + pg] = static_cast<int32_t>(i);
    if (pm >= 0) o.mid[region * o.cap + s_b[1] + pm] = static_cast<int32_t>(i);
    if (valid) {
      int64_t sum = 0;
      if (len <= kLaneMax) {  // this lane's own row: all of its loads at once
        int32_t x[kLaneMax], j[kLaneMax];
#pragma unroll
        for (int k = 0; k < kLaneMax; ++k) {
          x[k] = k < len ? wt[st + k] : 0;
          j[k] = (C && k < len) ? col[st + k] : -1;
        }
#pragma unroll
        for (int k = 0; k < kLaneMax; ++k) {
          sum += x[k];
          if (C && j[k] >= 0 && C[j[k]] == ci) intra += x[k];
        }
      }
      if (len <= kLaneMax || is_long) {
        o.K[i] = sum;  // (long rows: zero, their chunks add)
        if (o.Sigma) o.Sigma[i] = sum;
      }
      if (o.Cinit) o.Cinit[i] = static_cast<int32_t>(i);
      if (o.size) o.size[i] = 1;
    }
    __syncthreads();
  }
  intra = wave_sum_i64(intra);
  if (lane == 0 && C && intra) stat_add(o.ctr + CTR_STATS0, ST_INTRA, intra);
}

// First entry of each region in the concatenation of a class's lists
// (cls 0: group rows, 1: wavefront rows); rb has kRegions + 1 entries.
__device__ __forceinline__ void region_bases(const int64_t* cnt, int cls, int64_t* rb) {
  if (threadIdx.x < kWave) {
    const int64_t c = threadIdx.x < kRegions ? cnt[(threadIdx.x * 2 + cls) * kCtrLine] : 0;
    int64_t incl = c;
    for (int s = 1; s < kWave; s <<= 1) {
      const int64_t u = __shfl_up(incl, s);
      if (static_cast<int>(threadIdx.x) >= s) incl += u;
    }
    if (threadIdx.x < kRegions) rb[threadIdx.x] = incl - c;
    if (threadIdx.x == kRegions - 1) rb[kRegions] = incl;
  }
  __syncthreads();
}

__device__ __forceinline__ int32_t listed(const int64_t* rb, const int32_t* list, int64_t cap, int64_t idx) {
  int r = 0;
#pragma unroll
  for (int h = kRegions / 2; h > 0; h >>= 1)
    if (rb[r + h] <= idx) r += h;
  return list[r * cap + (idx - rb[r])];
}

// group rows: 16 lanes per row, four rows per wavefront at a time
__global__ void __launch_bounds__(kBlock) k_rows_grp(const int64_t* __restrict__ row_start,
                                                    const int32_t* __restrict__ row_len,
                                                    const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                    const int32_t* __restrict__ C, RowSumOut o) {
  __shared__ int64_t s_rb[kRegions + 1];
  region_bases(o.cnt, 0, s_rb);
  const int64_t count = s_rb[kRegions];
  const int sub = threadIdx.x & 15;
  const int64_t ngroups = static_cast<int64_t>(gridDim.x) * (kBlock / 16);
  int64_t intra = 0;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(kBlock / 16) + threadIdx.x / 16; idx < count;
       idx += ngroups) {
    const int32_t i = listed(s_rb, o.grp, o.cap, idx);
    const int64_t s = row_start[i];
    const int32_t len = row_len[i];
    const int32_t ci = C ? C[i] : 0;
    int32_t x[kGroupMax / 16], j[kGroupMax / 16];
#pragma unroll
    for (int q = 0; q < kGroupMax / 16; ++q) {
      const int32_t k = sub + q * 16;
      x[q] = k < len ? wt[s + k] : 0;
      j[q] = (C && k < len) ? col[s + k] : -1;
    }
    int64_t acc = 0;
#pragma unroll
    for (int q = 0; q < kGroupMax / 16; ++q) {
      acc += x[q];
      if (C && j[q] >= 0 && C[j[q]] == ci) intra += x[q];
    }
    for (int m = 8; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 16);
    if (sub == 0) {
      o.K[i] = acc;
      if (o.Sigma) o.Sigma[i] = acc;
    }
  }
  intra = wave_sum_i64(intra);
  if (lane_id() == 0 && C && intra) stat_add(o.ctr + CTR_STATS0, ST_INTRA, intra);
}

// wavefront rows, the next row's list entry and metadata loaded before this
// row's arcs are summed
__global__ void __launch_bounds__(kBlock) k_rows_mid(const int64_t* __restrict__ row_start,
                                                    const int32_t* __restrict__ row_len,
                                                    const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                    const int32_t* __restrict__ C, RowSumOut o) {
  __shared__ int64_t s_rb[kRegions + 1];
  region_bases(o.cnt, 1, s_rb);
  const int64_t count = s_rb[kRegions];
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  int64_t intra = 0;
  int64_t idx = blockIdx.x * static_cast<int64_t>(kWavesPerBlock) + threadIdx.x / kWave;
  int32_t i = idx < count ? listed(s_rb, o.mid, o.cap, idx) : -1;
  int64_t s = i >= 0 ? row_start[i] : 0;
  int32_t len = i >= 0 ? row_len[i] : 0;
  int32_t ci = (C && i >= 0) ? C[i] : 0;
  while (idx < count) {
    const int64_t nidx = idx + nwaves;
    const int32_t ni = nidx < count ? listed(s_rb, o.mid, o.cap, nidx) : -1;
    const int64_t ns = ni >= 0 ? row_start[ni] : 0;
    const int32_t nlen = ni >= 0 ? row_len[ni] : 0;
    const int32_t nci = (C && ni >= 0) ? C[ni] : 0;
    const int64_t sum = wave_row_sum(col, wt, C, s, 0, len, ci, &intra);
    if (lane_id() == 0) {
      o.K[i] = sum;
      if (o.Sigma) o.Sigma[i] = sum;
    }
    idx = nidx;
    i = ni;
    s = ns;
    len = nlen;
    ci = nci;
  }
  intra = wave_sum_i64(intra);
  if (lane_id() == 0 && C && intra) stat_add(o.ctr + CTR_STATS0, ST_INTRA, intra);
}

__global__ void __launch_bounds__(kBlock) k_rows_chunks(const int64_t* __restrict__ row_start,
                                                       const int32_t* __restrict__ row_len,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ wt,
                                                       const int32_t* __restrict__ C, RowSumOut o) {
  const int64_t count = o.ctr[CTR_AUX1];
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  int64_t intra = 0;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(kWavesPerBlock) + threadIdx.x / kWave; idx < count;
       idx += nwaves) {
    const int32_t i = o.lrow[idx];
    const int32_t a = o.loff[idx];
    const int32_t b = min(row_len[i], a + kChunk);
    const int32_t ci = C ? C[i] : 0;
    const int64_t sum = wave_row_sum(col, wt, C, row_start[i], a, b, ci, &intra);
    if (lane_id() == 0 && sum) {
      atomic_add_i64(&o.K[i], sum);
      if (o.Sigma) atomic_add_i64(&o.Sigma[i], sum);
    }
  }
  intra = wave_sum_i64(intra);
  if (lane_id() == 0 && C && intra) stat_add(o.ctr + CTR_STATS0, ST_INTRA, intra);
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
// C_mod given, the weight of intra-community arcs is added to statistic
// ST_INTRA of the first statistics set.  Uses ctr[CTR_AUX1], the second
// statistics set (list counters), the first two bin lists (the group and
// wavefront row lists, n + kRowListPad entries each) and the two unit lists
// (n + cap/2048 + 64 entries each, more than the chunks of cap arcs in rows
// of over 4096 arcs can take) for the chunks of long rows.
void launch_row_sums(const LevelGraph& g, const int32_t* C_mod, int64_t* K, int64_t* Sigma, int32_t* Cinit,
                     int32_t* size, Workspace& ws, hipStream_t st) {
  if (g.n == 0) return;
  static_assert(kChunk >= 2048, "the unit lists hold cap / 2048 chunks");
  static_assert(2 * kRegions * kCtrLine <= kStatSet, "the list counters fit a statistics set");
  static_assert(kRegions * kBlock <= kRowListPad, "region lists of whole row tasks fit the padded bin lists");
  int64_t* cnt = ws.ctr + CTR_STATS0 + kStatSet;
  (void)hipMemsetAsync(ws.ctr + CTR_AUX1, 0, sizeof(int64_t) * kCtrLine, st);
  (void)hipMemsetAsync(cnt, 0, sizeof(int64_t) * 2 * kRegions * kCtrLine, st);
  // region r takes the row tasks t = r mod kRegions: ceil(tasks / kRegions)
  // tasks of kBlock rows
  const int64_t tasks = (static_cast<int64_t>(g.n) + kBlock - 1) / kBlock;
  const int64_t cap = (tasks + kRegions - 1) / kRegions * kBlock;
  RowSumOut o{K, Sigma, Cinit, size, ws.u_ins_b, ws.u_emit_b, ws.ctr, ws.bins[0], ws.bins[1], cap, cnt};
  hipLaunchKernelGGL(k_rows_flat, dim3(static_cast<uint32_t>(std::min<int64_t>(tasks, 8192))), dim3(kBlock), 0, st,
                     g.row_start, g.row_len, g.col, g.w, g.n, C_mod, o);
  // (grids of many waves, so the memory latencies of the rows overlap; the
  // waves without a row or chunk return at once)
  hipLaunchKernelGGL(k_rows_grp, dim3(8192), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col, g.w, C_mod, o);
  hipLaunchKernelGGL(k_rows_mid, dim3(8192), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col, g.w, C_mod, o);
  hipLaunchKernelGGL(k_rows_chunks, dim3(8192), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col, g.w, C_mod, o);
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
