// Initial marking of affected vertices and the auxiliary-information update.
//   DF (Alg. 1): endpoints of intra-community deletions and cross-community
//                insertions (both endpoints, the batch being undirected).
//   ND (Alg. 2): every vertex (a bitmask fill on the host side).
//   DS (Alg. 3): δV/δE/δC from intra-community deletions and, per insertion
//                source, the best linked community; then neighbours of δE
//                vertices and members of δC communities.  The per-source
//                hashtable is a global open-addressing table keyed by
//                (source, community), and the per-source best by a second
//                table keyed by source, so no sort of the batch is needed.
//   updateWeights (Alg. 7): K and Σ adjusted by the batch, keyed by the
//                previous community; int64 atomics replace the paper's
//                per-thread work lists.
#include <climits>

#include "lv_internal.hpp"

namespace lv {
namespace {


// Alg. 7: K_u, K_v += w and Sigma[C_u], Sigma[C_v] += w per update (minus
// for deletions).  Large communities take many of the Sigma updates of a
// batch, and device atomics on one address serialise, so each workgroup
// first sums its updates' Sigma deltas per community in LDS and then
// issues one atomic per distinct community.
// A batch entry names two distinct vertices of the graph.
__device__ __forceinline__ bool update_ok(int32_t a, int32_t b, int32_t n) {
  return a >= 0 && b >= 0 && a < n && b < n && a != b;
}

constexpr int kUwItems = 4;                         // updates per thread
constexpr int kUwSlots = 2048;                      // LDS table slots
constexpr int kUwProbes = 16;
// With `fr` given, the same pass also does DF's initial marking (both read
// the previous memberships C^{t-1}).  Nothing is done when the call's error
// slot is already set (2m out of range).  An update naming a vertex outside
// [0, n) or a self-loop (a batch apply_batch would have refused) is skipped
// and flags LV_EINVAL, so a mismatched batch is reported, never applied out
// of bounds.
__global__ void __launch_bounds__(kBlock) k_update_weights(const int32_t* __restrict__ du, const int32_t* __restrict__ dv,
                                 const int32_t* __restrict__ dw, int64_t nd, const int32_t* __restrict__ iu,
                                 const int32_t* __restrict__ iv, const int32_t* __restrict__ iw, int64_t ni,
                                 int32_t n, const int32_t* __restrict__ C, int64_t* __restrict__ K,
                                 int64_t* __restrict__ Sigma, uint32_t* __restrict__ fr, FrontList fl,
                                 int64_t* __restrict__ ctr) {
  if (ctr[CTR_ERR]) return;
  __shared__ int32_t tk[kUwSlots];
  __shared__ unsigned long long tv[kUwSlots];
  for (int q = threadIdx.x; q < kUwSlots; q += kBlock) {
    tk[q] = -1;
    tv[q] = 0;
  }
  __syncthreads();
  const int64_t total = nd + ni;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock * kUwItems;
  // all of a thread's updates are loaded, then their communities gathered,
  // so the memory latencies overlap
  int32_t ea[kUwItems], eb[kUwItems], ca[kUwItems], cb[kUwItems];
  int64_t ex[kUwItems];
  bool del[kUwItems], ok[kUwItems];
#pragma unroll
  for (int it = 0; it < kUwItems; ++it) {
    const int64_t k = base + static_cast<int64_t>(it) * kBlock + threadIdx.x;
    ok[it] = k < total;
    del[it] = k < nd;
    ea[it] = !ok[it] ? 0 : (del[it] ? du[k] : iu[k - nd]);
    eb[it] = !ok[it] ? 0 : (del[it] ? dv[k] : iv[k - nd]);
    ex[it] = !ok[it] ? 0 : (del[it] ? -static_cast<int64_t>(dw[k]) : static_cast<int64_t>(iw[k - nd]));
    if (ok[it] && !update_ok(ea[it], eb[it], n)) {
      set_error(ctr, LV_EINVAL);
      ok[it] = false;
    }
  }
#pragma unroll
  for (int it = 0; it < kUwItems; ++it) {
    ca[it] = ok[it] ? C[ea[it]] : 0;
    cb[it] = ok[it] ? C[eb[it]] : 0;
  }
  if (fr) {  // deletion inside a community, or insertion across (every lane takes part in the appends)
    int32_t vs[2 * kUwItems];
    bool hits[2 * kUwItems];
#pragma unroll
    for (int it = 0; it < kUwItems; ++it) {
      const bool hit = ok[it] && (ca[it] == cb[it]) == del[it];
      vs[2 * it] = ea[it];
      vs[2 * it + 1] = eb[it];
      hits[2 * it] = hits[2 * it + 1] = hit;
    }
    front_mark_n(fr, fl, vs, hits);
  }
#pragma unroll
  for (int it = 0; it < kUwItems; ++it) {
    if (!ok[it]) continue;
    const int32_t a = ea[it], b = eb[it];
    const int64_t x = ex[it];
    atomic_add_i64(&K[a], x);
    atomic_add_i64(&K[b], x);
    for (int side = 0; side < 2; ++side) {
      const int32_t c = side ? cb[it] : ca[it];
      uint32_t h = hash_slot(static_cast<uint32_t>(c), kUwSlots);
      bool done = false;
      for (int p = 0; p < kUwProbes; ++p) {
        const int32_t old = atomicCAS(&tk[h], -1, c);
        if (old == -1 || old == c) {
          atomicAdd(&tv[h], static_cast<unsigned long long>(x));
          done = true;
          break;
        }
        h = (h + 1) & (kUwSlots - 1);
      }
      if (!done) atomic_add_i64(&Sigma[c], x);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kUwSlots; q += kBlock)
    if (tk[q] >= 0 && tv[q]) atomic_add_i64(&Sigma[tk[q]], static_cast<int64_t>(tv[q]));
}

// ctr[CTR_AUX2] += Σ w of insertions, ctr[CTR_AUX3] += Σ w of deletions
__global__ void k_batch_weight_sums(const int32_t* __restrict__ dw, int64_t nd, const int32_t* __restrict__ iw,
                                    int64_t ni, int64_t* __restrict__ ctr) {
  int64_t si = 0, sd = 0;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < nd + ni;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (k < nd)
      sd += dw[k];
    else
      si += iw[k - nd];
  }
  si = wave_sum_i64(si);
  sd = wave_sum_i64(sd);
  if (lane_id() == 0) {
    if (si) atomic_add_i64(&ctr[CTR_AUX2], si);
    if (sd) atomic_add_i64(&ctr[CTR_AUX3], sd);
  }
}

__global__ void k_ds_deletions(const int32_t* __restrict__ du, const int32_t* __restrict__ dv, int64_t nd, int32_t n,
                               const int32_t* __restrict__ C, uint32_t* __restrict__ dV, uint32_t* __restrict__ dE,
                               uint32_t* __restrict__ dC, int64_t* __restrict__ ctr) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < nd;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t a = du[k], b = dv[k];
    if (!update_ok(a, b, n)) {
      set_error(ctr, LV_EINVAL);
      continue;
    }
    if (C[a] != C[b]) continue;
    set_bit(dV, a);
    set_bit(dV, b);
    set_bit(dE, a);
    set_bit(dE, b);
    set_bit(dC, C[a]);
  }
}

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint32_t hash64(uint64_t key, uint32_t mask) {
  key ^= key >> 33;
  key *= 0xff51afd7ed558ccdull;
  key ^= key >> 33;
  return static_cast<uint32_t>(key) & mask;
}

// find-or-insert; returns the slot
__device__ __forceinline__ uint32_t table_slot(uint64_t* keys, uint32_t size, uint64_t key) {
  const uint32_t mask = size - 1;
  uint32_t h = hash64(key, mask);
  while (true) {
    const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&keys[h]), kEmpty, key);
    if (old == kEmpty || old == key) return h;
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ uint32_t table_find(const uint64_t* keys, uint32_t size, uint64_t key) {
  const uint32_t mask = size - 1;
  uint32_t h = hash64(key, mask);
  while (true) {
    const uint64_t k = keys[h];
    if (k == key) return h;
    if (k == kEmpty) return 0xffffffffu;
    h = (h + 1) & mask;
  }
}

// H[(source, C[target])] += w over cross-community insertion arcs (both
// directions of every insertion)
__global__ void k_ds_insert_pairs(const int32_t* __restrict__ iu, const int32_t* __restrict__ iv,
                                  const int32_t* __restrict__ iw, int64_t ni, int32_t n, const int32_t* __restrict__ C,
                                  uint64_t* __restrict__ keys, int64_t* __restrict__ vals, uint32_t size,
                                  int64_t* __restrict__ ctr) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < 2 * ni;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t e = k >> 1;
    const int32_t s = (k & 1) ? iv[e] : iu[e];
    const int32_t t = (k & 1) ? iu[e] : iv[e];
    if (!update_ok(s, t, n)) {
      set_error(ctr, LV_EINVAL);
      continue;
    }
    const int32_t cs = C[s], ct = C[t];
    if (cs == ct) continue;
    const uint64_t key = (static_cast<uint64_t>(static_cast<uint32_t>(s)) << 32) | static_cast<uint32_t>(ct);
    const uint32_t h = table_slot(keys, size, key);
    atomic_add_i64(&vals[h], iw[e]);
  }
}

// pass 0: per source, the largest score 2m_prev H[c] - K_s Σ_c (Eq. 2 with
// K_{s->c} := H[c], terms independent of c dropped); pass 1: lowest c
// attaining it
__global__ void k_ds_best(const uint64_t* __restrict__ keys, const int64_t* __restrict__ vals, uint32_t size,
                          const int64_t* __restrict__ K, const int64_t* __restrict__ Sigma,
                          const int64_t* __restrict__ two_m_dev, const int64_t* __restrict__ ctr,
                          uint64_t* __restrict__ skeys, int64_t* __restrict__ sbest, int32_t* __restrict__ sbestc,
                          uint32_t ssize, int pass) {
  const int64_t two_m_prev = *two_m_dev - 2 * ctr[CTR_AUX2] + 2 * ctr[CTR_AUX3];
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < size;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t key = keys[k];
    if (key == kEmpty) continue;
    const int32_t s = static_cast<int32_t>(key >> 32);
    const int32_t c = static_cast<int32_t>(key & 0xffffffffu);
    const int64_t score = two_m_prev * vals[k] - K[s] * Sigma[c];
    if (pass == 0) {
      const uint32_t h = table_slot(skeys, ssize, static_cast<uint64_t>(s));
      atomicMax(reinterpret_cast<long long*>(&sbest[h]), static_cast<long long>(score));
    } else {
      const uint32_t h = table_find(skeys, ssize, static_cast<uint64_t>(s));
      if (h != 0xffffffffu && sbest[h] == score) atomicMin(&sbestc[h], c);
    }
  }
}

__global__ void k_ds_mark_sources(const uint64_t* __restrict__ skeys, const int32_t* __restrict__ sbestc,
                                  uint32_t ssize, uint32_t* __restrict__ dV, uint32_t* __restrict__ dE,
                                  uint32_t* __restrict__ dC) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < ssize;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t key = skeys[k];
    if (key == kEmpty) continue;
    const int32_t s = static_cast<int32_t>(key);
    set_bit(dV, s);
    set_bit(dE, s);
    set_bit(dC, sbestc[k]);
  }
}

// members of affected communities join δV
__global__ void k_ds_community_members(const int32_t* __restrict__ C, int32_t n, const uint32_t* __restrict__ dC,
                                       uint32_t* __restrict__ dV) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (test_bit(dC, C[i])) set_bit(dV, static_cast<int32_t>(i));
}

// neighbours of δE vertices join δV; δE vertices are batch endpoints, so
// one wavefront per endpoint of every update
__global__ void k_ds_expand(const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len,
                            const int32_t* __restrict__ col, int32_t n, const int32_t* __restrict__ du,
                            const int32_t* __restrict__ dv, int64_t nd, const int32_t* __restrict__ iu,
                            const int32_t* __restrict__ iv, int64_t ni, const uint32_t* __restrict__ dE,
                            uint32_t* __restrict__ dV) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  const int64_t total = 2 * (nd + ni);
  for (int64_t e = wave; e < total; e += nwaves) {
    const int64_t k = e >> 1;
    int32_t v;
    if (k < nd)
      v = (e & 1) ? dv[k] : du[k];
    else
      v = (e & 1) ? iv[k - nd] : iu[k - nd];
    if (v < 0 || v >= n || !test_bit(dE, v)) continue;  // (ids out of range are flagged by the other kernels)
    const int64_t s = row_start[v];
    const int32_t l = row_len[v];
    for (int32_t t = lane; t < l; t += kWave) set_bit(dV, col[s + t]);
  }
}

}  // namespace


void launch_update_weights(const lv_edges& del, const lv_edges& ins, int32_t n, const int32_t* C, int64_t* K,
                           int64_t* Sigma, uint32_t* df_frontier, const FrontList& df_list, int64_t* ctr,
                           hipStream_t st) {
  const int64_t total = del.count + ins.count;
  if (total == 0) return;
  const int blocks = static_cast<int>((total + kBlock * kUwItems - 1) / (kBlock * kUwItems));
  hipLaunchKernelGGL(k_update_weights, dim3(blocks), dim3(kBlock), 0, st, del.u, del.v,
                     del.w, del.count, ins.u, ins.v, ins.w, ins.count, n, C, K, Sigma, df_frontier, df_list, ctr);
}

void launch_batch_weight_sums(const lv_edges& del, const lv_edges& ins, int64_t* ctr, hipStream_t st) {
  const int64_t total = del.count + ins.count;
  if (total == 0) return;
  hipLaunchKernelGGL(k_batch_weight_sums, dim3(grid_for(total, kBlock, 1024)), dim3(kBlock), 0, st, del.w,
                     del.count, ins.w, ins.count, ctr);
}

void launch_community_sizes(const int32_t* C, int32_t n, int32_t* size, hipStream_t st) {
  (void)hipMemsetAsync(size, 0, sizeof(int32_t) * static_cast<size_t>(n), st);
  launch_accumulate(C, n, nullptr, nullptr, size, nullptr, st);
}

void launch_ds_deletions(const lv_edges& del, int32_t n, const int32_t* C, uint32_t* dV, uint32_t* dE, uint32_t* dC,
                         int64_t* ctr, hipStream_t st) {
  if (del.count == 0) return;
  hipLaunchKernelGGL(k_ds_deletions, dim3(grid_for(del.count, kBlock, 4096)), dim3(kBlock), 0, st, del.u, del.v,
                     del.count, n, C, dV, dE, dC, ctr);
}

void launch_ds_insert_pairs(const lv_edges& ins, int32_t n, const int32_t* C, uint64_t* keys, int64_t* vals,
                            uint32_t size, int64_t* ctr, hipStream_t st) {
  if (ins.count == 0) return;
  hipLaunchKernelGGL(k_ds_insert_pairs, dim3(grid_for(2 * ins.count, kBlock, 4096)), dim3(kBlock), 0, st, ins.u,
                     ins.v, ins.w, ins.count, n, C, keys, vals, size, ctr);
}

void launch_ds_best(const uint64_t* keys, const int64_t* vals, uint32_t size, const int64_t* K, const int64_t* Sigma,
                    const int64_t* two_m_dev, const int64_t* ctr, uint64_t* skeys, int64_t* sbest, int32_t* sbestc,
                    uint32_t ssize, int pass, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_best, dim3(grid_for(size, kBlock, 4096)), dim3(kBlock), 0, st, keys, vals, size, K, Sigma,
                     two_m_dev, ctr, skeys, sbest, sbestc, ssize, pass);
}

void launch_ds_mark_sources(const uint64_t* skeys, const int32_t* sbestc, uint32_t ssize, uint32_t* dV,
                            uint32_t* dE, uint32_t* dC, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_mark_sources, dim3(grid_for(ssize, kBlock, 4096)), dim3(kBlock), 0, st, skeys, sbestc,
                     ssize, dV, dE, dC);
}

void launch_ds_expand(const LevelGraph& g, const lv_edges& del, const lv_edges& ins, const int32_t* C,
                      const uint32_t* dE, const uint32_t* dC, uint32_t* dV, hipStream_t st) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_ds_community_members, dim3(grid_for(g.n, kBlock, 8192)), dim3(kBlock), 0, st, C, g.n, dC,
                     dV);
  const int64_t total = 2 * (del.count + ins.count);
  if (total == 0) return;
  hipLaunchKernelGGL(k_ds_expand, dim3(grid_for(total * kWave, kBlock, 4096)), dim3(kBlock), 0, st, g.row_start,
                     g.row_len, g.col, g.n, del.u, del.v, del.count, ins.u, ins.v, ins.count, dE, dV);
}

}  // namespace lv
