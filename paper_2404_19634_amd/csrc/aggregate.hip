// Community renumbering and dendrogram lookup (Alg. 4) and the aggregation
// phase (Alg. 6): the community-vertex CSR by count / scan / fill, super-
// vertex row capacities from community volumes (the paper's over-estimated,
// "holey" offsets), and per community a hashtable over its members' arcs,
// self-loops included, whose entries become the super-vertex's row.
//
// Communities of volume <= the wave threshold are merged by one wavefront
// with an LDS table; larger ones by a workgroup with a global table from
// the workspace pool.  The super-vertex weight K''_c (= Σ''_c) is the row
// sum written at the same time.
#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int kAggWaveVol = 256;  // volume limit of the wavefront merge
constexpr int kAggTS = 512;       // LDS slots per wavefront (>= 2 * kAggWaveVol)

__global__ void k_mark_exists(const int32_t* __restrict__ C, int32_t n, int32_t* __restrict__ flags) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    flags[C[i]] = 1;
}

__global__ void k_relabel(int32_t* __restrict__ C, int32_t n, const int32_t* __restrict__ newid) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    C[i] = newid[C[i]];
}

__global__ void k_lookup(int32_t* __restrict__ Ctop, int32_t n, const int32_t* __restrict__ Cl) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    Ctop[i] = Cl[Ctop[i]];
}

// count members and volume (arcs incl. self-loops) of each community
__global__ void k_count_members(const int32_t* __restrict__ C, const int32_t* __restrict__ row_len, int32_t n,
                                int32_t* __restrict__ ccount, int64_t* __restrict__ vol) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t c = C[i];
    atomicAdd(&ccount[c], 1);
    const int32_t l = row_len[i];
    if (l) atomic_add_i64(&vol[c], l);
  }
}

// fill the community-vertex CSR; ccount is consumed as a per-community cursor
__global__ void k_fill_members(const int32_t* __restrict__ C, int32_t n, const int32_t* __restrict__ coff,
                               int32_t* __restrict__ ccount, int32_t* __restrict__ cmem) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t c = C[i];
    const int32_t slot = atomicSub(&ccount[c], 1) - 1;
    cmem[coff[c] + slot] = static_cast<int32_t>(i);
  }
}

// split communities into the wavefront list and the workgroup list; big
// communities get a global table of 2*volume slots
__global__ void k_bin_communities(const int64_t* __restrict__ row_start_out, int32_t nc,
                                  int32_t* __restrict__ small, int32_t* __restrict__ big,
                                  int64_t* __restrict__ big_off, int32_t* __restrict__ row_len_out,
                                  int64_t* __restrict__ Kout, int64_t* __restrict__ Sout, int64_t* __restrict__ ctr) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t c0 = blockIdx.x * static_cast<int64_t>(blockDim.x); c0 < nc; c0 += stride) {
    const int64_t c = c0 + threadIdx.x;
    int64_t vol = 0;
    const bool valid = c < nc;
    if (valid) {
      vol = row_start_out[c + 1] - row_start_out[c];
      if (vol == 0) {
        row_len_out[c] = 0;
        Kout[c] = 0;
        Sout[c] = 0;
      }
    }
    const int64_t ps = wave_append(valid && vol > 0 && vol <= kAggWaveVol, &ctr[CTR_AUX1]);
    if (ps >= 0) small[ps] = static_cast<int32_t>(c);
    const int64_t pb = wave_append(valid && vol > kAggWaveVol, &ctr[CTR_AUX2]);
    if (pb >= 0) {
      big[pb] = static_cast<int32_t>(c);
      big_off[pb] = static_cast<int64_t>(
          atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_POOL]), 2ull * static_cast<unsigned long long>(vol)));
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_merge_wave(
    const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len, const int32_t* __restrict__ col,
    const int32_t* __restrict__ wt, const int32_t* __restrict__ C, const int32_t* __restrict__ coff,
    const int32_t* __restrict__ cmem, const int32_t* __restrict__ list, const int64_t* __restrict__ ctr,
    const int64_t* __restrict__ out_start, int32_t* __restrict__ out_len, int32_t* __restrict__ out_col,
    int32_t* __restrict__ out_w, int64_t* __restrict__ Kout, int64_t* __restrict__ Sout) {
  __shared__ int32_t s_keys[kBlock / kWave][kAggTS];
  __shared__ int32_t s_vals[kBlock / kWave][kAggTS];
  const int64_t count = ctr[CTR_AUX1];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int32_t* keys = s_keys[wid];
  int32_t* vals = s_vals[wid];
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t idx = wave; idx < count; idx += nwaves) {
    const int32_t c = list[idx];
    for (int t = lane; t < kAggTS; t += kWave) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t m0 = coff[c], m1 = coff[c + 1];
    for (int32_t m = m0; m < m1; ++m) {
      const int32_t i = cmem[m];
      const int64_t s = row_start[i];
      const int32_t l = row_len[i];
      for (int32_t k = lane; k < l; k += kWave) {
        const int32_t d = C[col[s + k]];
        const int32_t x = wt[s + k];
        uint32_t h = hash_slot(static_cast<uint32_t>(d), kAggTS);
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, d);
          if (old == -1 || old == d) {
            atomicAdd(&vals[h], x);
            break;
          }
          h = (h + 1) & (kAggTS - 1);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t base = out_start[c];
    int32_t written = 0;
    int64_t ksum = 0;
    for (int t0 = 0; t0 < kAggTS; t0 += kWave) {
      const int32_t d = keys[t0 + lane];
      const bool occ = d >= 0;
      const uint64_t mask = __ballot(occ);
      if (occ) {
        const int32_t pos = written + __popcll(mask & ((1ull << lane) - 1ull));
        const int32_t x = vals[t0 + lane];
        out_col[base + pos] = d;
        out_w[base + pos] = x;
        ksum += x;
      }
      written += __popcll(mask);
    }
    ksum = wave_sum_i64(ksum);
    if (lane == 0) {
      out_len[c] = written;
      Kout[c] = ksum;
      Sout[c] = ksum;
    }
  }
}

__device__ __forceinline__ int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kBlock) k_merge_block(
    const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len, const int32_t* __restrict__ col,
    const int32_t* __restrict__ wt, const int32_t* __restrict__ C, const int32_t* __restrict__ coff,
    const int32_t* __restrict__ cmem, const int32_t* __restrict__ list, const int64_t* __restrict__ big_off,
    int64_t* __restrict__ ctr, int32_t* __restrict__ pool_keys, int32_t* __restrict__ pool_vals, int64_t pool_slots,
    const int64_t* __restrict__ out_start, int32_t* __restrict__ out_len, int32_t* __restrict__ out_col,
    int32_t* __restrict__ out_w, int64_t* __restrict__ Kout, int64_t* __restrict__ Sout) {
  __shared__ int32_t s_cnt[kBlock / kWave];
  __shared__ int64_t s_sum[kBlock / kWave];
  const int64_t count = ctr[CTR_AUX2];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t c = list[idx];
    const int64_t vol = out_start[c + 1] - out_start[c];
    const int64_t tsz64 = 2 * vol;
    if (big_off[idx] + tsz64 > pool_slots || tsz64 > 0x7fffffff) {
      if (threadIdx.x == 0) set_error(ctr, LV_EWORKSPACE);
      continue;
    }
    const uint32_t tsz = static_cast<uint32_t>(tsz64);
    int32_t* keys = pool_keys + big_off[idx];
    int32_t* vals = pool_vals + big_off[idx];
    for (uint32_t t = threadIdx.x; t < tsz; t += kBlock) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __threadfence_block();
    __syncthreads();
    const int32_t m0 = coff[c], m1 = coff[c + 1];
    for (int32_t m = m0; m < m1; ++m) {
      const int32_t i = cmem[m];
      const int64_t s = row_start[i];
      const int32_t l = row_len[i];
      for (int32_t k = threadIdx.x; k < l; k += kBlock) {
        const int32_t d = C[col[s + k]];
        const int32_t x = wt[s + k];
        uint32_t h = hash_slot(static_cast<uint32_t>(d), tsz);
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, d);
          if (old == -1 || old == d) {
            atomicAdd(&vals[h], x);
            break;
          }
          h = (h + 1 == tsz) ? 0 : h + 1;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    const int64_t base = out_start[c];
    int32_t written = 0;
    int64_t ksum = 0;
    for (uint32_t t0 = 0; t0 < tsz; t0 += kBlock) {
      const uint32_t t = t0 + threadIdx.x;
      int32_t d = -1, x = 0;
      if (t < tsz) {
        d = ld_relaxed(&keys[t]);
        if (d >= 0) x = ld_relaxed(&vals[t]);
      }
      const bool occ = d >= 0;
      const uint64_t mask = __ballot(occ);
      if (lane == 0) s_cnt[wid] = __popcll(mask);
      __syncthreads();
      int32_t before = 0, total = 0;
      for (int q = 0; q < kBlock / kWave; ++q) {
        if (q < wid) before += s_cnt[q];
        total += s_cnt[q];
      }
      if (occ) {
        const int32_t pos = written + before + __popcll(mask & ((1ull << lane) - 1ull));
        out_col[base + pos] = d;
        out_w[base + pos] = x;
        ksum += x;
      }
      written += total;
      __syncthreads();
    }
    ksum = wave_sum_i64(ksum);
    if (lane == 0) s_sum[wid] = ksum;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int q = 0; q < kBlock / kWave; ++q) tot += s_sum[q];
      out_len[c] = written;
      Kout[c] = tot;
      Sout[c] = tot;
    }
    __syncthreads();
  }
}

__global__ void k_sigma_from_members(const int32_t* __restrict__ C, const int64_t* __restrict__ K, int32_t n,
                                     int64_t* __restrict__ Sigma) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t k = K[i];
    if (k) atomic_add_i64(&Sigma[C[i]], k);
  }
}

}  // namespace

void launch_mark_exists(const int32_t* C, int32_t n, int32_t* flags, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mark_exists, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, C, n, flags);
}

void launch_relabel(int32_t* C, int32_t n, const int32_t* newid, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, C, n, newid);
}

void launch_lookup(int32_t* Ctop, int32_t n, const int32_t* Cl, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_lookup, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, Ctop, n, Cl);
}

// Community-vertex CSR (coff, cmem) and community volumes (vol).
void launch_community_members(const int32_t* C, const LevelGraph& g, int32_t nc, Workspace& ws, hipStream_t st) {
  (void)hipMemsetAsync(ws.ccount, 0, sizeof(int32_t) * (static_cast<size_t>(nc) + 1), st);
  (void)hipMemsetAsync(ws.vol, 0, sizeof(int64_t) * (static_cast<size_t>(nc) + 1), st);
  hipLaunchKernelGGL(k_count_members, dim3(grid_for(g.n, kBlock, 8192)), dim3(kBlock), 0, st, C, g.row_len, g.n,
                     ws.ccount, ws.vol);
  exclusive_scan_i32(ws.ccount, ws.coff, nc, ws, st);
  hipLaunchKernelGGL(k_fill_members, dim3(grid_for(g.n, kBlock, 8192)), dim3(kBlock), 0, st, C, g.n, ws.coff,
                     ws.ccount, ws.cmem);
}

void launch_aggregate(const LevelGraph& g, const int32_t* C, int32_t nc, LevelGraph& out, int64_t* Kout,
                      int64_t* Sout, int32_t* Cout, int32_t* sizeout, Workspace& ws, const lv_tuning& tu,
                      hipStream_t st) {
  launch_community_members(C, g, nc, ws, st);
  // super-vertex row offsets = exclusive scan of community volumes
  exclusive_scan_i64(ws.vol, out.row_start, nc, ws, st);
  out.n = nc;
  (void)hipMemsetAsync(ws.ctr + CTR_AUX1, 0, 2 * sizeof(int64_t), st);
  (void)hipMemsetAsync(ws.ctr + CTR_POOL, 0, sizeof(int64_t), st);
  hipLaunchKernelGGL(k_bin_communities, dim3(grid_for(nc, kBlock, 4096)), dim3(kBlock), 0, st, out.row_start, nc,
                     ws.bins[0], ws.bins[1], ws.hub_off, out.row_len, Kout, Sout, ws.ctr);
  hipLaunchKernelGGL(k_merge_wave, dim3(tu.blocks_wave), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col,
                     g.w, C, ws.coff, ws.cmem, ws.bins[0], ws.ctr, out.row_start, out.row_len, out.col, out.w,
                     Kout, Sout);
  hipLaunchKernelGGL(k_merge_block, dim3(tu.blocks_hub), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col,
                     g.w, C, ws.coff, ws.cmem, ws.bins[1], ws.hub_off, ws.ctr, ws.pool_keys, ws.pool_vals,
                     ws.pool_slots, out.row_start, out.row_len, out.col, out.w, Kout, Sout);
  // the next level starts from singletons; written only after the merges,
  // which still read the current membership (the same array from pass 1 on)
  launch_iota_i32(Cout, nc, st);
  if (sizeout) launch_fill_i32(sizeout, 1, nc, st);
}

void launch_sigma_from_members(const int32_t* C, const int64_t* K, int32_t n, int64_t* Sigma, hipStream_t st) {
  (void)hipMemsetAsync(Sigma, 0, sizeof(int64_t) * static_cast<size_t>(n), st);
  if (n == 0) return;
  hipLaunchKernelGGL(k_sigma_from_members, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, C, K, n, Sigma);
}

}  // namespace lv
