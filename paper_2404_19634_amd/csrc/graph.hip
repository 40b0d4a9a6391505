// Graph storage kernels: building the slack-padded CSR (the "holey" CSR of
// the paper's aggregation phase, Alg. 6, reused for in-place batch
// updates), relayout with more slack, weighted degrees (Section 3), and the
// per-arc / per-community terms of modularity (Eq. 1).
#include "lv_internal.hpp"

namespace lv {

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

// Row reduction pattern: each lane owns one row of the wave's 64; rows of
// at most kWave arcs are summed by their own lane, longer rows by the whole
// wavefront one after another.
template <class PerArc, class PerRow>
__device__ __forceinline__ void wave_rows(int64_t row0, int32_t n, const int64_t* __restrict__ row_start,
                                          const int32_t* __restrict__ row_len, PerArc arc, PerRow fin) {
  const int lane = lane_id();
  const int64_t i = row0 + lane;
  const bool valid = i < n;
  const int32_t len = valid ? row_len[i] : 0;
  const int64_t start = valid ? row_start[i] : 0;
  const bool shortrow = valid && len <= kWave;
  int64_t a0 = 0, a1 = 0;
  if (shortrow) {
    for (int32_t k = 0; k < len; ++k) arc(static_cast<int32_t>(i), start + k, a0, a1);
    fin(static_cast<int32_t>(i), a0, a1);
  }
  uint64_t longmask = __ballot(valid && !shortrow);
  while (longmask) {
    const int src = __ffsll(static_cast<unsigned long long>(longmask)) - 1;
    longmask &= longmask - 1;
    const int32_t r = static_cast<int32_t>(row0 + src);
    const int64_t rs = __shfl(start, src);
    const int32_t rl = __shfl(len, src);
    int64_t b0 = 0, b1 = 0;
    for (int32_t k = lane; k < rl; k += kWave) arc(r, rs + k, b0, b1);
    b0 = wave_sum_i64(b0);
    b1 = wave_sum_i64(b1);
    if (lane == 0) fin(r, b0, b1);
  }
}

__global__ void k_degrees(const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len,
                          const int32_t* __restrict__ wt, int32_t n, int64_t* __restrict__ K,
                          int64_t* __restrict__ Sigma, int32_t* __restrict__ C, int32_t* __restrict__ size) {
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t r0 = wave * kWave; r0 < n; r0 += nwaves * kWave) {
    wave_rows(
        r0, n, row_start, row_len,
        [&](int32_t, int64_t p, int64_t& s, int64_t&) { s += wt[p]; },
        [&](int32_t i, int64_t s, int64_t) {
          K[i] = s;
          if (Sigma) Sigma[i] = s;
          if (C) C[i] = i;
          if (size) size[i] = 1;
        });
  }
}

// Per vertex i: Σ_c[C_i] += K_i; total intra-community arc weight += Σ of
// w over arcs (i, j) with C_j = C_i.
__global__ void k_modularity_terms(const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len,
                                   const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                   int32_t n, const int32_t* __restrict__ C, int64_t* __restrict__ sig_tot,
                                   int64_t* __restrict__ ctr) {
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  int64_t intra = 0;
  for (int64_t r0 = wave * kWave; r0 < n; r0 += nwaves * kWave) {
    wave_rows(
        r0, n, row_start, row_len,
        [&](int32_t i, int64_t p, int64_t& s, int64_t& in) {
          const int32_t x = wt[p];
          s += x;
          if (C[col[p]] == C[i]) in += x;
        },
        [&](int32_t i, int64_t s, int64_t in) {
          if (s) atomic_add_i64(&sig_tot[C[i]], s);
          intra += in;
        });
  }
  intra = wave_sum_i64(intra);
  if (lane_id() == 0 && intra) atomic_add_i64(&ctr[CTR_AUX0], intra);
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

void launch_degrees(const LevelGraph& g, int64_t* K, int64_t* Sigma, int32_t* C, int32_t* size,
                    hipStream_t st) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_degrees, dim3(grid_for(g.n, kBlock, 4096)), dim3(kBlock), 0, st, g.row_start,
                     g.row_len, g.w, g.n, K, Sigma, C, size);
}

void launch_modularity_terms(const LevelGraph& g, const int32_t* C, int64_t* sig_tot, int64_t* ctr,
                             hipStream_t st) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_modularity_terms, dim3(grid_for(g.n, kBlock, 4096)), dim3(kBlock), 0, st,
                     g.row_start, g.row_len, g.col, g.w, g.n, C, sig_tot, ctr);
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
