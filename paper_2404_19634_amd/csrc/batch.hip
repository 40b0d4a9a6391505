// In-place batch update of the slack CSR (Section 3.4: a batch holds edge
// deletions Δ- and insertions Δ+; Section 5.1.4: batches are undirected).
//
// Phase 1 (no writes to the graph): validate ids, weights and repeated
//   pairs; locate every deletion's two arcs; classify every insertion arc
//   as a merge into a surviving arc or an append; check row capacities and
//   the 2m bound.  The host reads the error slot once.
// Phase 2 (only when phase 1 found nothing): subtract deletions, compact
//   the rows that lost arcs (stable, one wavefront per row), add merges,
//   append new arcs into the slack, update 2m.
#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t canon(int32_t a, int32_t b) {
  const uint32_t lo = static_cast<uint32_t>(min(a, b)), hi = static_cast<uint32_t>(max(a, b));
  return (static_cast<uint64_t>(lo) << 32) | hi;
}

__device__ __forceinline__ uint32_t hash64(uint64_t key, uint32_t mask) {
  key ^= key >> 33;
  key *= 0xff51afd7ed558ccdull;
  key ^= key >> 33;
  return static_cast<uint32_t>(key) & mask;
}

// Inserts key; returns false when it was already present.
__device__ __forceinline__ bool set_insert(uint64_t* keys, uint32_t size, uint64_t key, uint32_t* slot) {
  const uint32_t mask = size - 1;
  uint32_t h = hash64(key, mask);
  while (true) {
    const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&keys[h]), kEmpty, key);
    if (old == kEmpty) {
      *slot = h;
      return true;
    }
    if (old == key) {
      *slot = h;
      return false;
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int64_t set_find(const uint64_t* keys, uint32_t size, uint64_t key) {
  const uint32_t mask = size - 1;
  uint32_t h = hash64(key, mask);
  while (true) {
    const uint64_t k = keys[h];
    if (k == key) return h;
    if (k == kEmpty) return -1;
    h = (h + 1) & mask;
  }
}

__global__ void k_validate(const int32_t* __restrict__ du, const int32_t* __restrict__ dv,
                           const int32_t* __restrict__ dw, int64_t nd, const int32_t* __restrict__ iu,
                           const int32_t* __restrict__ iv, const int32_t* __restrict__ iw, int64_t ni, int32_t n,
                           BatchScratch b, int64_t* __restrict__ ctr) {
  int64_t si = 0, sd = 0;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < nd + ni;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const bool del = k < nd;
    const int32_t a = del ? du[k] : iu[k - nd];
    const int32_t c = del ? dv[k] : iv[k - nd];
    const int32_t x = del ? dw[k] : iw[k - nd];
    if (a < 0 || c < 0 || a >= n || c >= n || a == c || x <= 0) {
      set_error(ctr, LV_EINVAL);
      continue;
    }
    uint32_t slot;
    if (del) {
      if (!set_insert(b.del_keys, b.del_size, canon(a, c), &slot)) set_error(ctr, LV_EINVAL);
      else b.del_vals[slot] = x;
      sd += x;
    } else {
      if (!set_insert(b.ins_keys, b.ins_size, canon(a, c), &slot)) set_error(ctr, LV_EINVAL);
      si += x;
    }
  }
  si = wave_sum_i64(si);
  sd = wave_sum_i64(sd);
  if (lane_id() == 0) {
    if (si) atomic_add_i64(&ctr[CTR_AUX2], si);
    if (sd) atomic_add_i64(&ctr[CTR_AUX3], sd);
  }
}

// Position of arc (a -> c) in row a, or -1; one wavefront scans the row.
__device__ __forceinline__ int64_t wave_find_arc(const int64_t* row_start, const int32_t* row_len,
                                                 const int32_t* col, int32_t a, int32_t c) {
  const int lane = lane_id();
  const int64_t s = row_start[a];
  const int32_t l = row_len[a];
  for (int32_t b0 = 0; b0 < l; b0 += kWave) {
    const int32_t k = b0 + lane;
    const uint64_t m = __ballot(k < l && col[s + k] == c);
    if (m) return s + b0 + (__ffsll(static_cast<unsigned long long>(m)) - 1);
  }
  return -1;
}

// one wavefront per (update, direction)
__global__ void k_find(const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len,
                       const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                       const int32_t* __restrict__ du, const int32_t* __restrict__ dv, const int32_t* __restrict__ dw,
                       int64_t nd, const int32_t* __restrict__ iu, const int32_t* __restrict__ iv, int64_t ni,
                       BatchScratch b, int64_t* __restrict__ ctr) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  const int64_t total = 2 * (nd + ni);
  for (int64_t e = wave; e < total; e += nwaves) {
    const int64_t k = e >> 1;
    const bool del = k < nd;
    int32_t a, c;
    if (del) {
      a = (e & 1) ? dv[k] : du[k];
      c = (e & 1) ? du[k] : dv[k];
    } else {
      a = (e & 1) ? iv[k - nd] : iu[k - nd];
      c = (e & 1) ? iu[k - nd] : iv[k - nd];
    }
    const int64_t pos = wave_find_arc(row_start, row_len, col, a, c);
    if (lane != 0) continue;
    if (del) {
      if (pos < 0 || wt[pos] < dw[k]) {
        set_error(ctr, LV_ENOEDGE);
        b.del_pos[e] = -1;
        continue;
      }
      b.del_pos[e] = pos;
      if (wt[pos] == dw[k]) atomicAdd(&b.row_zeroed[a], 1);
    } else {
      bool merge = pos >= 0;
      if (merge) {  // an arc removed whole by this batch's deletions is re-appended
        const int64_t h = set_find(b.del_keys, b.del_size, canon(a, c));
        if (h >= 0 && b.del_vals[h] == wt[pos]) merge = false;
      }
      b.ins_kind[e - 2 * nd] = merge ? 1 : 0;
      if (!merge) atomicAdd(&b.row_app[a], 1);
    }
  }
}

__global__ void k_capacity(const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len,
                           const int32_t* __restrict__ du, const int32_t* __restrict__ dv, int64_t nd,
                           const int32_t* __restrict__ iu, const int32_t* __restrict__ iv, int64_t ni,
                           const int64_t* __restrict__ two_m, BatchScratch b, int64_t* __restrict__ ctr) {
  const int64_t total = 2 * (nd + ni);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t nm = *two_m + 2 * ctr[CTR_AUX2] - 2 * ctr[CTR_AUX3];
    if (nm >= (int64_t(1) << 31)) set_error(ctr, LV_EOVERFLOW);
  }
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t k = e >> 1;
    int32_t a;
    if (k < nd)
      a = (e & 1) ? dv[k] : du[k];
    else
      a = (e & 1) ? iv[k - nd] : iu[k - nd];
    const int64_t need = static_cast<int64_t>(row_len[a]) - b.row_zeroed[a] + b.row_app[a];
    if (need > row_start[a + 1] - row_start[a]) set_error(ctr, LV_ENOSLACK);
  }
}

__global__ void k_apply_del(int32_t* __restrict__ wt, const int32_t* __restrict__ dw, int64_t nd, BatchScratch b) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < 2 * nd;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    wt[b.del_pos[e]] -= dw[e >> 1];
}

// stable removal of zero-weight arcs; the first wavefront that claims a row
// compacts it
__global__ void k_compact(const int64_t* __restrict__ row_start, int32_t* __restrict__ row_len,
                          int32_t* __restrict__ col, int32_t* __restrict__ wt, const int32_t* __restrict__ du,
                          const int32_t* __restrict__ dv, int64_t nd, BatchScratch b) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t e = wave; e < 2 * nd; e += nwaves) {
    const int64_t k = e >> 1;
    const int32_t a = (e & 1) ? dv[k] : du[k];
    int32_t claim = 0;
    if (lane == 0) claim = atomicExch(&b.row_zeroed[a], 0);
    claim = __shfl(claim, 0);
    if (claim == 0) continue;
    const int64_t s = row_start[a];
    const int32_t l = row_len[a];
    int32_t out = 0;
    for (int32_t b0 = 0; b0 < l; b0 += kWave) {
      const int32_t k2 = b0 + lane;
      int32_t cc = 0, ww = 0;
      if (k2 < l) {
        cc = col[s + k2];
        ww = wt[s + k2];
      }
      const bool keep = k2 < l && ww > 0;
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int32_t p = out + __popcll(m & ((1ull << lane) - 1ull));
        col[s + p] = cc;
        wt[s + p] = ww;
      }
      out += __popcll(m);
    }
    if (lane == 0) row_len[a] = out;
  }
}

__global__ void k_merge_ins(const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len,
                            const int32_t* __restrict__ col, int32_t* __restrict__ wt, const int32_t* __restrict__ iu,
                            const int32_t* __restrict__ iv, const int32_t* __restrict__ iw, int64_t ni,
                            BatchScratch b) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t e = wave; e < 2 * ni; e += nwaves) {
    if (b.ins_kind[e] != 1) continue;
    const int64_t k = e >> 1;
    const int32_t a = (e & 1) ? iv[k] : iu[k];
    const int32_t c = (e & 1) ? iu[k] : iv[k];
    const int64_t pos = wave_find_arc(row_start, row_len, col, a, c);
    if (lane == 0 && pos >= 0) wt[pos] += iw[k];
  }
}

__global__ void k_append_ins(const int64_t* __restrict__ row_start, int32_t* __restrict__ row_len,
                             int32_t* __restrict__ col, int32_t* __restrict__ wt, const int32_t* __restrict__ iu,
                             const int32_t* __restrict__ iv, const int32_t* __restrict__ iw, int64_t ni,
                             BatchScratch b) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < 2 * ni;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (b.ins_kind[e] != 0) continue;
    const int64_t k = e >> 1;
    const int32_t a = (e & 1) ? iv[k] : iu[k];
    const int32_t c = (e & 1) ? iu[k] : iv[k];
    const int64_t p = row_start[a] + atomicAdd(&row_len[a], 1);
    col[p] = c;
    wt[p] = iw[k];
  }
}

__global__ void k_update_two_m(int64_t* __restrict__ two_m, const int64_t* __restrict__ ctr) {
  *two_m += 2 * ctr[CTR_AUX2] - 2 * ctr[CTR_AUX3];
}

}  // namespace

void launch_batch_validate(const lv_edges& del, const lv_edges& ins, int32_t n, const BatchScratch& b, int64_t* ctr,
                           hipStream_t st) {
  const int64_t total = del.count + ins.count;
  if (total == 0) return;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(total, kBlock, 4096)), dim3(kBlock), 0, st, del.u, del.v, del.w,
                     del.count, ins.u, ins.v, ins.w, ins.count, n, b, ctr);
}

void launch_batch_find(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                       int64_t* ctr, hipStream_t st) {
  const int64_t total = 2 * (del.count + ins.count);
  if (total == 0) return;
  hipLaunchKernelGGL(k_find, dim3(grid_for(total * kWave, kBlock, 8192)), dim3(kBlock), 0, st, g.row_start,
                     g.row_len, g.col, g.w, del.u, del.v, del.w, del.count, ins.u, ins.v, ins.count, b, ctr);
}

void launch_batch_capacity(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                           int64_t* ctr, hipStream_t st) {
  const int64_t total = 2 * (del.count + ins.count);
  hipLaunchKernelGGL(k_capacity, dim3(grid_for(total, kBlock, 4096)), dim3(kBlock), 0, st, g.row_start, g.row_len,
                     del.u, del.v, del.count, ins.u, ins.v, ins.count, g.two_m, b, ctr);
}

void launch_batch_apply(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                        int64_t* ctr, hipStream_t st) {
  if (del.count) {
    hipLaunchKernelGGL(k_apply_del, dim3(grid_for(2 * del.count, kBlock, 4096)), dim3(kBlock), 0, st, g.w, del.w,
                       del.count, b);
    hipLaunchKernelGGL(k_compact, dim3(grid_for(2 * del.count * kWave, kBlock, 8192)), dim3(kBlock), 0, st,
                       g.row_start, g.row_len, g.col, g.w, del.u, del.v, del.count, b);
  }
  if (ins.count) {
    hipLaunchKernelGGL(k_merge_ins, dim3(grid_for(2 * ins.count * kWave, kBlock, 8192)), dim3(kBlock), 0, st,
                       g.row_start, g.row_len, g.col, g.w, ins.u, ins.v, ins.w, ins.count, b);
    hipLaunchKernelGGL(k_append_ins, dim3(grid_for(2 * ins.count, kBlock, 4096)), dim3(kBlock), 0, st, g.row_start,
                       g.row_len, g.col, g.w, ins.u, ins.v, ins.w, ins.count, b);
  }
  hipLaunchKernelGGL(k_update_two_m, dim3(1), dim3(1), 0, st, g.two_m, ctr);
}

}  // namespace lv
