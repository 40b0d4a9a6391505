// Local-moving phase (Alg. 5): frontier compaction into degree bins, the
// neighbour-community scan with the integer ΔQ argmax, and the moves with
// incremental frontier expansion (the vertex-pruning marking that DF relies
// on, Section 4.1).
//
// Gain of moving i from d = C_i to a neighbouring community c (Eq. 2 times
// 2m^2, exact in int64 while 2m < 2^31):
//     g(c) = 2m (K_{i->c} - K_{i->d}) - K_i (Σ_c - Σ_d + K_i)
// The target is the c != d with the largest g, lowest id on ties; i moves
// only when that gain is positive.  Self-loops are not scanned.
//
// Work mapping (wave64, CDNA):
//   rows of 1..4/5..8/9..16/17..32 arcs: groups of 4/8/16/32 lanes, one arc
//     per lane; community weights are summed by all-pairs lane exchange
//     within the group (no memory traffic, no atomics, conflict free);
//   rows up to the wave threshold: one wavefront with an open-addressing
//     table in LDS; arcs into the vertex's own community are summed in
//     registers, which keeps the most common key out of the LDS atomics;
//   longer rows: one workgroup with an open-addressing table in global
//     memory (a slice of the workspace pool sized 2*deg).
// SYNC mode reads the iteration-start state and records movers; a separate
// kernel applies them.  ASYNC mode applies each move at once.  Both expand
// the next frontier from the kernel that holds the mover's arcs.
#include <climits>

#include "lv_internal.hpp"

namespace lv {
namespace {

struct Dev {
  const int64_t* row_start;
  const int32_t* row_len;
  const int32_t* col;
  const int32_t* wt;
  int32_t* C;
  const int64_t* K;
  int64_t* Sigma;
  int32_t* size;
  uint32_t* next;
  int32_t* mv_v;
  int32_t* mv_c;
  int64_t* ctr;
  int64_t two_m;
  int32_t mode;
  int32_t guard;
};

Dev make_dev(const MoveArgs& a, Workspace& ws) {
  Dev d;
  d.row_start = a.g.row_start;
  d.row_len = a.g.row_len;
  d.col = a.g.col;
  d.wt = a.g.w;
  d.C = a.C;
  d.K = a.K;
  d.Sigma = a.Sigma;
  d.size = a.size;
  d.next = a.next;
  d.mv_v = ws.mv_v;
  d.mv_c = ws.mv_c;
  d.ctr = ws.ctr;
  d.two_m = a.two_m;
  d.mode = a.mode;
  d.guard = a.guard;
  return d;
}

__device__ __forceinline__ bool better(int64_t g1, int32_t c1, int64_t g0, int32_t c0) {
  return g1 > g0 || (g1 == g0 && c1 < c0);
}

__device__ __forceinline__ int64_t gain_of(int64_t two_m, int64_t kic, int64_t kid, int64_t Ki, int64_t Sc,
                                           int64_t Sd) {
  return two_m * (kic - kid) - Ki * (Sc - Sd + Ki);
}

// Final decision with the optional swap guard (singleton into a singleton
// of larger id is vetoed).  Reads sizes of the current state.
__device__ __forceinline__ bool decide_move(const Dev& D, int32_t d, int32_t c, int64_t g) {
  if (c == INT_MAX || g <= 0) return false;
  if (D.guard && D.size[d] == 1 && D.size[c] == 1 && c > d) return false;
  return true;
}

// Applies a move immediately (ASYNC) -- one lane per mover.
__device__ __forceinline__ void apply_now(const Dev& D, int32_t i, int32_t d, int32_t c, int64_t Ki) {
  D.C[i] = c;
  atomic_add_i64(&D.Sigma[d], -Ki);
  atomic_add_i64(&D.Sigma[c], Ki);
  if (D.size) {
    atomicSub(&D.size[d], 1);
    atomicAdd(&D.size[c], 1);
  }
}

// Vertices of word k that belong to sub-round `round` (ASYNC mode splits
// each iteration into 2^(32 - shift) sub-rounds by a multiplicative hash of
// the vertex id, so that a vertex sees most neighbours' moves already
// applied; shift = 32 means a single round).
__device__ __forceinline__ uint32_t round_mask(uint32_t k, uint32_t round, uint32_t shift) {
  uint32_t m = 0;
#pragma unroll 8
  for (uint32_t b = 0; b < 32; ++b) {
    const uint32_t i = k * 32 + b;
    if (((i * 0x9E3779B1u) >> shift) == round) m |= 1u << b;
  }
  return m;
}

// --------------------------------------------------------------------------
// Frontier -> degree bins.  One lane per 32-vertex bitmask word; set bits
// are peeled one per step so the wavefront stays converged for the
// aggregated appends.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_bin_frontier(const uint32_t* __restrict__ cur,
                                                        const uint32_t* __restrict__ range,
                                                        uint32_t* __restrict__ ever,
                                                        const int32_t* __restrict__ row_len, int32_t n,
                                                        int32_t wave_max, uint32_t round, uint32_t round_shift,
                                                        int32_t* b0, int32_t* b1,
                                                        int32_t* b2, int32_t* b3, int32_t* b4, int32_t* b5,
                                                        int64_t* __restrict__ hub_off, int64_t* __restrict__ ctr) {
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  int64_t arcs = 0, processed = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t w0 = blockIdx.x * static_cast<int64_t>(blockDim.x); w0 < words; w0 += stride) {
    const int64_t k = w0 + threadIdx.x;
    uint32_t bits = 0;
    if (k < words) {
      bits = cur[k];
      if (range) bits &= range[k];
      if (round_shift < 32 && bits) bits &= round_mask(static_cast<uint32_t>(k), round, round_shift);
      if (ever && bits) ever[k] |= bits;
    }
    while (__ballot(bits != 0)) {
      const bool has = bits != 0;
      int32_t i = 0, deg = 0;
      if (has) {
        i = static_cast<int32_t>(k * 32 + (__ffs(bits) - 1));
        bits &= bits - 1;
        deg = row_len[i];
        processed += 1;
        arcs += deg;
      }
      int bin = -1;
      if (has && deg > 0) {
        if (deg <= 4) bin = BIN_G4;
        else if (deg <= 8) bin = BIN_G8;
        else if (deg <= 16) bin = BIN_G16;
        else if (deg <= 32) bin = BIN_G32;
        else if (deg <= wave_max) bin = BIN_WAVE;
        else bin = BIN_HUB;
      }
      int32_t* lists[NBINS] = {b0, b1, b2, b3, b4, b5};
#pragma unroll
      for (int b = 0; b < NBINS; ++b) {
        const int64_t pos = wave_append(bin == b, &ctr[CTR_BIN0 + b]);
        if (pos >= 0) {
          lists[b][pos] = i;
          if (b == BIN_HUB)
            hub_off[pos] = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_POOL]),
                                                          2ull * static_cast<unsigned long long>(deg)));
        }
      }
    }
  }
  processed = wave_sum_i64(processed);
  arcs = wave_sum_i64(arcs);
  if (lane_id() == 0) {
    if (processed) atomic_add_i64(&ctr[CTR_PROCESSED], processed);
    if (arcs) atomic_add_i64(&ctr[CTR_ARCS], arcs);
  }
}

// --------------------------------------------------------------------------
// Rows of at most G arcs: groups of G lanes, one arc per lane.
// --------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(kBlock) k_move_small(Dev D, const int32_t* __restrict__ list, int bin) {
  constexpr int VPW = kWave / G;
  const int64_t count = D.ctr[CTR_BIN0 + bin];
  const int lane = lane_id();
  const int sub = lane / G;
  const int k = lane % G;
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  int64_t gain_acc = 0, moved = 0;
  for (int64_t base = wave * VPW; base < count; base += nwaves * VPW) {
    const int64_t idx = base + sub;
    const bool valid = idx < count;
    int32_t i = 0, deg = 0, d = -1;
    int64_t start = 0;
    if (valid) {
      i = list[idx];
      start = D.row_start[i];
      deg = D.row_len[i];
      d = D.C[i];
    }
    bool has = valid && k < deg;
    int32_t j = -1, x = 0, c = -1;
    if (has) {
      j = D.col[start + k];
      x = D.wt[start + k];
      if (j == i) has = false;  // self-loop: not a neighbour
    }
    if (has) c = D.C[j];
    // K_{i->c} for this lane's community: all-pairs exchange inside the group
    int32_t kc = has ? x : 0;
    const int32_t xe = has ? x : 0;
#pragma unroll
    for (int s = 1; s < G; ++s) {
      const int32_t c2 = __shfl_xor(c, s);
      const int32_t x2 = __shfl_xor(xe, s);
      if (has && c2 == c) kc += x2;
    }
    int32_t kid = (has && c == d) ? kc : 0;
#pragma unroll
    for (int s = 1; s < G; s <<= 1) kid = max(kid, __shfl_xor(kid, s));
    const bool cand = has && c != d;
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    int64_t Ki = 0;
    if (valid) Ki = D.K[i];
    if (cand) {
      const int64_t Sd = D.Sigma[d];
      bg = gain_of(D.two_m, kc, kid, Ki, D.Sigma[c], Sd);
      bc = c;
    }
#pragma unroll
    for (int s = 1; s < G; s <<= 1) {
      const int64_t og = __shfl_xor(bg, s);
      const int32_t oc = __shfl_xor(bc, s);
      if (better(og, oc, bg, bc)) {
        bg = og;
        bc = oc;
      }
    }
    const bool lead = valid && k == 0;
    bool mv = false;
    if (valid) mv = decide_move(D, d, bc, bg);
    if (D.mode == LV_SYNC) {
      const int64_t pos = wave_append(lead && mv, &D.ctr[CTR_MOVERS]);
      if (pos >= 0) {
        D.mv_v[pos] = i;
        D.mv_c[pos] = bc;
      }
    } else if (lead && mv) {
      apply_now(D, i, d, bc, Ki);
    }
    if (lead && mv) {
      gain_acc += bg;
      moved += 1;
    }
    if (mv && has) set_bit(D.next, j);
  }
  gain_acc = wave_sum_i64(gain_acc);
  moved = wave_sum_i64(moved);
  if (lane == 0 && moved) {
    atomic_add_i64(&D.ctr[CTR_GAIN], gain_acc);
    if (D.mode != LV_SYNC) atomic_add_i64(&D.ctr[CTR_MOVERS], moved);
  }
}

// --------------------------------------------------------------------------
// Rows up to the wave threshold: one wavefront, LDS table of TS slots.
// --------------------------------------------------------------------------
template <int TS>
__global__ void __launch_bounds__(kBlock) k_move_wave(Dev D, const int32_t* __restrict__ list) {
  __shared__ int32_t s_keys[kBlock / kWave][TS];
  __shared__ int32_t s_vals[kBlock / kWave][TS];
  const int64_t count = D.ctr[CTR_BIN0 + BIN_WAVE];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int32_t* keys = s_keys[wid];
  int32_t* vals = s_vals[wid];
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  int64_t gain_acc = 0, moved = 0;
  for (int64_t idx = wave; idx < count; idx += nwaves) {
    const int32_t i = list[idx];
    const int64_t start = D.row_start[i];
    const int32_t deg = D.row_len[i];
    const int32_t d = D.C[i];
    for (int t = lane; t < TS; t += kWave) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int32_t kid = 0;
    for (int32_t b = 0; b < deg; b += kWave) {
      const int32_t k = b + lane;
      if (k < deg) {
        const int32_t j = D.col[start + k];
        const int32_t x = D.wt[start + k];
        if (j != i) {
          const int32_t c = D.C[j];
          if (c == d) {
            kid += x;
          } else {
            uint32_t h = hash_slot(static_cast<uint32_t>(c), TS);
            while (true) {
              const int32_t old = atomicCAS(&keys[h], -1, c);
              if (old == -1 || old == c) {
                atomicAdd(&vals[h], x);
                break;
              }
              h = (h + 1) & (TS - 1);
            }
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    kid = wave_sum_i32(kid);
    const int64_t Ki = D.K[i];
    const int64_t Sd = D.Sigma[d];
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    for (int t = lane; t < TS; t += kWave) {
      const int32_t c = keys[t];
      if (c >= 0) {
        const int64_t g = gain_of(D.two_m, vals[t], kid, Ki, D.Sigma[c], Sd);
        if (better(g, c, bg, bc)) {
          bg = g;
          bc = c;
        }
      }
    }
    for (int s = 1; s < kWave; s <<= 1) {
      const int64_t og = __shfl_xor(bg, s);
      const int32_t oc = __shfl_xor(bc, s);
      if (better(og, oc, bg, bc)) {
        bg = og;
        bc = oc;
      }
    }
    const bool mv = decide_move(D, d, bc, bg);
    if (mv) {
      if (lane == 0) {
        if (D.mode == LV_SYNC) {
          const int64_t pos = static_cast<int64_t>(
              atomicAdd(reinterpret_cast<unsigned long long*>(&D.ctr[CTR_MOVERS]), 1ull));
          D.mv_v[pos] = i;
          D.mv_c[pos] = bc;
        } else {
          apply_now(D, i, d, bc, Ki);
        }
        gain_acc += bg;
        moved += 1;
      }
      for (int32_t b = lane; b < deg; b += kWave) {
        const int32_t j = D.col[start + b];
        if (j != i) set_bit(D.next, j);
      }
    }
  }
  gain_acc = wave_sum_i64(gain_acc);
  moved = wave_sum_i64(moved);
  if (lane == 0 && moved) {
    atomic_add_i64(&D.ctr[CTR_GAIN], gain_acc);
    if (D.mode != LV_SYNC) atomic_add_i64(&D.ctr[CTR_MOVERS], moved);
  }
}

// --------------------------------------------------------------------------
// Long rows: one workgroup, global-memory table of 2*deg slots.
// --------------------------------------------------------------------------
__device__ __forceinline__ int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kBlock) k_move_hub(Dev D, const int32_t* __restrict__ list,
                                                    const int64_t* __restrict__ hub_off,
                                                    int32_t* __restrict__ pool_keys,
                                                    int32_t* __restrict__ pool_vals, int64_t pool_slots) {
  __shared__ int64_t r_g[kBlock / kWave];
  __shared__ int32_t r_c[kBlock / kWave];
  __shared__ int32_t r_k[kBlock / kWave];
  const int64_t count = D.ctr[CTR_BIN0 + BIN_HUB];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int64_t gain_acc = 0, moved = 0;
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t i = list[idx];
    const int64_t start = D.row_start[i];
    const int32_t deg = D.row_len[i];
    const int32_t d = D.C[i];
    const uint32_t tsz = 2u * static_cast<uint32_t>(deg);
    if (hub_off[idx] + tsz > pool_slots) {  // cannot happen with the workspace bound; never write past it
      if (threadIdx.x == 0) set_error(D.ctr, LV_EWORKSPACE);
      continue;
    }
    int32_t* keys = pool_keys + hub_off[idx];
    int32_t* vals = pool_vals + hub_off[idx];
    for (uint32_t t = threadIdx.x; t < tsz; t += kBlock) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __threadfence_block();
    __syncthreads();
    int32_t kid = 0;
    for (int32_t k = threadIdx.x; k < deg; k += kBlock) {
      const int32_t j = D.col[start + k];
      const int32_t x = D.wt[start + k];
      if (j == i) continue;
      const int32_t c = D.C[j];
      if (c == d) {
        kid += x;
        continue;
      }
      uint32_t h = hash_slot(static_cast<uint32_t>(c), tsz);
      while (true) {
        const int32_t old = atomicCAS(&keys[h], -1, c);
        if (old == -1 || old == c) {
          atomicAdd(&vals[h], x);
          break;
        }
        h = (h + 1 == tsz) ? 0 : h + 1;
      }
    }
    kid = wave_sum_i32(kid);
    if (lane == 0) r_k[wid] = kid;
    __threadfence_block();
    __syncthreads();
    kid = 0;
    for (int t = 0; t < kBlock / kWave; ++t) kid += r_k[t];
    const int64_t Ki = D.K[i];
    const int64_t Sd = D.Sigma[d];
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    for (uint32_t t = threadIdx.x; t < tsz; t += kBlock) {
      const int32_t c = ld_relaxed(&keys[t]);
      if (c >= 0) {
        const int64_t g = gain_of(D.two_m, ld_relaxed(&vals[t]), kid, Ki, D.Sigma[c], Sd);
        if (better(g, c, bg, bc)) {
          bg = g;
          bc = c;
        }
      }
    }
    for (int s = 1; s < kWave; s <<= 1) {
      const int64_t og = __shfl_xor(bg, s);
      const int32_t oc = __shfl_xor(bc, s);
      if (better(og, oc, bg, bc)) {
        bg = og;
        bc = oc;
      }
    }
    if (lane == 0) {
      r_g[wid] = bg;
      r_c[wid] = bc;
    }
    __syncthreads();
    for (int t = 0; t < kBlock / kWave; ++t)
      if (better(r_g[t], r_c[t], bg, bc)) {
        bg = r_g[t];
        bc = r_c[t];
      }
    const bool mv = decide_move(D, d, bc, bg);
    if (mv) {
      if (threadIdx.x == 0) {
        if (D.mode == LV_SYNC) {
          const int64_t pos = static_cast<int64_t>(
              atomicAdd(reinterpret_cast<unsigned long long*>(&D.ctr[CTR_MOVERS]), 1ull));
          D.mv_v[pos] = i;
          D.mv_c[pos] = bc;
        } else {
          apply_now(D, i, d, bc, Ki);
        }
        gain_acc += bg;
        moved += 1;
      }
      for (int32_t k = threadIdx.x; k < deg; k += kBlock) {
        const int32_t j = D.col[start + k];
        if (j != i) set_bit(D.next, j);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && moved) {
    atomic_add_i64(&D.ctr[CTR_GAIN], gain_acc);
    if (D.mode != LV_SYNC) atomic_add_i64(&D.ctr[CTR_MOVERS], moved);
  }
}

// --------------------------------------------------------------------------
// SYNC: apply the recorded moves after every decision was taken.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_apply_moves(int32_t* __restrict__ C, const int64_t* __restrict__ K,
                                                       int64_t* __restrict__ Sigma, int32_t* __restrict__ size,
                                                       const int32_t* __restrict__ mv_v,
                                                       const int32_t* __restrict__ mv_c,
                                                       const int64_t* __restrict__ ctr) {
  const int64_t count = ctr[CTR_MOVERS];
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < count;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t i = mv_v[t];
    const int32_t c = mv_c[t];
    const int32_t d = C[i];
    const int64_t Ki = K[i];
    C[i] = c;
    atomic_add_i64(&Sigma[d], -Ki);
    atomic_add_i64(&Sigma[c], Ki);
    if (size) {
      atomicSub(&size[d], 1);
      atomicAdd(&size[c], 1);
    }
  }
}

int table_slots_for(int wave_max) {
  int ts = 64;
  while (ts < 2 * wave_max) ts <<= 1;
  return ts;
}

}  // namespace

void launch_bin_frontier(const MoveArgs& a, Workspace& ws, int round, int rounds_log2, hipStream_t st) {
  const int64_t words = (static_cast<int64_t>(a.g.n) + 31) / 32;
  const uint32_t shift = rounds_log2 > 0 ? 32u - static_cast<uint32_t>(rounds_log2) : 32u;
  hipLaunchKernelGGL(k_bin_frontier, dim3(grid_for(words, kBlock, 4096)), dim3(kBlock), 0, st, a.cur,
                     a.range, a.ever, a.g.row_len, a.g.n, a.wave_max, static_cast<uint32_t>(round), shift,
                     ws.bins[0], ws.bins[1], ws.bins[2], ws.bins[3], ws.bins[4], ws.bins[5], ws.hub_off, ws.ctr);
}

void launch_move(const MoveArgs& a, Workspace& ws, const lv_tuning& tu, hipStream_t st) {
  const Dev D = make_dev(a, ws);
  const int bs = tu.blocks_small, bw = tu.blocks_wave, bh = tu.blocks_hub;
  hipLaunchKernelGGL(k_move_small<4>, dim3(bs), dim3(kBlock), 0, st, D, ws.bins[BIN_G4], int(BIN_G4));
  hipLaunchKernelGGL(k_move_small<8>, dim3(bs), dim3(kBlock), 0, st, D, ws.bins[BIN_G8], int(BIN_G8));
  hipLaunchKernelGGL(k_move_small<16>, dim3(bs), dim3(kBlock), 0, st, D, ws.bins[BIN_G16], int(BIN_G16));
  hipLaunchKernelGGL(k_move_small<32>, dim3(bs), dim3(kBlock), 0, st, D, ws.bins[BIN_G32], int(BIN_G32));
  const int ts = table_slots_for(a.wave_max);
  if (ts <= 128)
    hipLaunchKernelGGL(k_move_wave<128>, dim3(bw), dim3(kBlock), 0, st, D, ws.bins[BIN_WAVE]);
  else if (ts <= 256)
    hipLaunchKernelGGL(k_move_wave<256>, dim3(bw), dim3(kBlock), 0, st, D, ws.bins[BIN_WAVE]);
  else if (ts <= 512)
    hipLaunchKernelGGL(k_move_wave<512>, dim3(bw), dim3(kBlock), 0, st, D, ws.bins[BIN_WAVE]);
  else
    hipLaunchKernelGGL(k_move_wave<1024>, dim3(bw), dim3(kBlock), 0, st, D, ws.bins[BIN_WAVE]);
  hipLaunchKernelGGL(k_move_hub, dim3(bh), dim3(kBlock), 0, st, D, ws.bins[BIN_HUB], ws.hub_off,
                     ws.pool_keys, ws.pool_vals, ws.pool_slots);
}

void launch_apply_moves(const MoveArgs& a, Workspace& ws, hipStream_t st) {
  hipLaunchKernelGGL(k_apply_moves, dim3(grid_for(a.g.n, kBlock, 2048)), dim3(kBlock), 0, st, a.C, a.K,
                     a.Sigma, a.size, ws.mv_v, ws.mv_c, ws.ctr);
}

}  // namespace lv
