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
// for Eq. 1) in three degree classes, so that no lane idles on a short row
// and no wavefront walks a long one alone:
//  - rows of at most kFlatMax arcs: one wavefront per 64 consecutive rows
//    reads their starts and lengths (coalesced) and walks their arcs as one
//    flat sequence, 256 consecutive arcs per step (four loads in flight per
//    lane); an LDS map gives each flat position's row, and LDS atomics add
//    each arc to its row's sum;
//  - rows up to kMidMax arcs are summed by the same wavefront right after,
//    one at a time, 256 arcs per step (a list of them would take one device
//    atomic per wavefront on a single counter, and those serialise);
//  - longer rows are listed in chunks of kChunk arcs, one wavefront per
//    chunk, whose partial sums are added atomically (K and Sigma of such a
//    row are zeroed by the first kernel).
constexpr int kFlatMax = 64;
constexpr int kMidMax = 4096;
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
};

__device__ __forceinline__ void wave_barrier_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
  constexpr int kSpan = kWave * kFlatMax;  // flat positions of a wavefront's short rows, at most
  __shared__ uint8_t s_own[kWavesPerBlock][kSpan];  // row (lane) of each flat position
  __shared__ int64_t s_base[kWavesPerBlock][kWave];  // row start minus the row's first flat position
  __shared__ int32_t s_c[kWavesPerBlock][kWave];
  __shared__ unsigned long long s_acc[kWavesPerBlock][kWave];
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  uint8_t* own = s_own[w];
  unsigned long long* acc = s_acc[w];
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  int64_t intra = 0;
  for (int64_t r0 = (blockIdx.x * static_cast<int64_t>(kWavesPerBlock) + w) * kWave; r0 < n;
       r0 += nwaves * kWave) {
    const int64_t i = r0 + lane;
    const bool valid = i < n;
    const int32_t row_len_l = valid ? row_len[i] : 0;
    int32_t len = row_len_l;
    const int64_t st = valid ? row_start[i] : 0;
    const int32_t ci = (C && valid) ? C[i] : 0;
    const bool is_mid = len > kFlatMax && len <= kMidMax;
    const bool is_long = len > kMidMax;
    {  // chunks of long rows, reserved together by the wavefront
      const int32_t nch = is_long ? (len + kChunk - 1) / kChunk : 0;
      int32_t incl = nch;
      for (int s = 1; s < kWave; s <<= 1) {
        const int32_t t = __shfl_up(incl, s);
        if (lane >= s) incl += t;
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
    if (valid) {
      if (is_long) {
        o.K[i] = 0;
        if (o.Sigma) o.Sigma[i] = 0;
      }
      if (o.Cinit) o.Cinit[i] = static_cast<int32_t>(i);
      if (o.size) o.size[i] = 1;
    }
    const bool is_short = valid && !is_mid && !is_long;
    if (!is_short) len = 0;
    // exclusive prefix of the short rows' lengths over the wavefront; each
    // lane marks its row's flat positions as its own
    int32_t incl = len;
    for (int s = 1; s < kWave; s <<= 1) {
      const int32_t t = __shfl_up(incl, s);
      if (lane >= s) incl += t;
    }
    const int32_t total = __shfl(incl, kWave - 1);
    const int32_t first = incl - len;
    for (int32_t k = 0; k < len; ++k) own[first + k] = static_cast<uint8_t>(lane);
    s_base[w][lane] = st - first;
    s_c[w][lane] = ci;
    acc[lane] = 0;
    wave_barrier_lds();
    for (int32_t b = 0; b < total; b += kWave * kRowUnroll) {
      int32_t r[kRowUnroll];
      int64_t x[kRowUnroll];
      int32_t cj[kRowUnroll];
#pragma unroll
      for (int q = 0; q < kRowUnroll; ++q) {
        const int32_t p = b + q * kWave + lane;
        r[q] = p < total ? own[p] : -1;
      }
#pragma unroll
      for (int q = 0; q < kRowUnroll; ++q) {
        const int32_t p = b + q * kWave + lane;
        x[q] = 0;
        cj[q] = -1;
        if (r[q] >= 0) {
          const int64_t a = s_base[w][r[q]] + p;
          x[q] = wt[a];
          if (C) cj[q] = col[a];
        }
      }
#pragma unroll
      for (int q = 0; q < kRowUnroll; ++q) {
        if (r[q] < 0) continue;
        atomicAdd(&acc[r[q]], static_cast<unsigned long long>(x[q]));
        if (C && C[cj[q]] == s_c[w][r[q]]) intra += x[q];
      }
    }
    wave_barrier_lds();
    if (is_short) {
      const int64_t sum = static_cast<int64_t>(acc[lane]);
      o.K[i] = sum;
      if (o.Sigma) o.Sigma[i] = sum;
    }
    wave_barrier_lds();
    // the middle rows of the 64, one after the other over the wavefront
    for (uint64_t mm = __ballot(is_mid); mm; mm &= mm - 1) {
      const int l = __ffsll(static_cast<unsigned long long>(mm)) - 1;
      const int64_t rs = __shfl(st, l);
      const int32_t rl = __shfl(row_len_l, l);
      const int32_t rc = __shfl(ci, l);
      const int64_t sum = wave_row_sum(col, wt, C, rs, 0, rl, rc, &intra);
      if (lane == l) {
        o.K[i] = sum;
        if (o.Sigma) o.Sigma[i] = sum;
      }
    }
  }
  intra = wave_sum_i64(intra);
  if (lane == 0 && C && intra) stat_add(o.ctr + CTR_STATS0, ST_INTRA, intra);
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
// ST_INTRA of the first statistics set.  Uses ctr[CTR_AUX1] and the two
// unit lists (n + cap/2048 + 64 entries each, more than the chunks of cap
// arcs in rows of over 4096 arcs can take) for the chunks of long rows.
void launch_row_sums(const LevelGraph& g, const int32_t* C_mod, int64_t* K, int64_t* Sigma, int32_t* Cinit,
                     int32_t* size, Workspace& ws, hipStream_t st) {
  if (g.n == 0) return;
  static_assert(kChunk >= 2048, "the unit lists hold cap / 2048 chunks");
  (void)hipMemsetAsync(ws.ctr + CTR_AUX1, 0, sizeof(int64_t) * kCtrLine, st);
  RowSumOut o{K, Sigma, Cinit, size, ws.u_ins_b, ws.u_emit_b, ws.ctr};
  const int64_t waves = (static_cast<int64_t>(g.n) + kWave - 1) / kWave;
  // (a grid-stride loop: each wavefront ends with one statistics atomic)
  const int64_t blocks = std::min<int64_t>((waves + kWavesPerBlock - 1) / kWavesPerBlock, 8192);
  hipLaunchKernelGGL(k_rows_flat, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, st, g.row_start, g.row_len,
                     g.col, g.w, g.n, C_mod, o);
  // (many waves, so the memory latencies of the chunks overlap; the waves
  // without a chunk return at once)
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
