// In-place batch update of the slack CSR (Section 3.4: a batch holds edge
// deletions Δ- and insertions Δ+; Section 5.1.4: batches are undirected, so
// every update touches the arc in both directions).
//
// The work is organised by ROW, not by update: rows are unsorted, so
// finding an arc means scanning its row, and in a skewed graph many updates
// land on the same hub rows.  Each touched row is therefore scanned once,
// in chunks of kChunk arcs, against a small per-chunk filter of the
// partners the batch names for that row; filter hits are resolved in a
// hashtable of the batch's undirected pairs.
//
// Phase 1 (reads the graph only): validate ids, weights and repeated pairs;
//   collect the touched rows; locate every update's two arcs; classify
//   insertion arcs as merges (the arc survives the deletions) or appends;
//   check row capacities and the 2m bound.  Errors go to the error counter.
// Phase 2 (every kernel returns at once if phase 1 set an error, so a bad
//   batch leaves the graph untouched without a host round trip in between):
//   subtract deletions and add merges at the located positions; refill the
//   holes left by arcs that reached weight 0 with the surviving arcs of the
//   row's tail (O(holes) per row, not O(row length); rows stay unsorted);
//   append new arcs into the slack; update 2m.
#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr int kChunk = 1024;        // arcs per scan unit (one wavefront)
constexpr int kFilterBits = 4096;   // per-wavefront partner filter
constexpr int kScanWaves = kBlock / kWave;

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

// Inserts key; returns its slot.
__device__ __forceinline__ uint32_t pair_insert(uint64_t* keys, uint32_t size, uint64_t key) {
  const uint32_t mask = size - 1;
  uint32_t h = hash64(key, mask);
  while (true) {
    const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&keys[h]), kEmpty, key);
    if (old == kEmpty || old == key) return h;
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int32_t pair_find(const uint64_t* keys, uint32_t size, uint64_t key) {
  const uint32_t mask = size - 1;
  uint32_t h = hash64(key, mask);
  while (true) {
    const uint64_t k = keys[h];
    if (k == key) return static_cast<int32_t>(h);
    if (k == kEmpty) return -1;
    h = (h + 1) & mask;
  }
}

// Endpoints of direction e: directions 2k, 2k+1 belong to deletion k
// (k < nd), then 2(nd + k), 2(nd + k) + 1 to insertion k.  Direction
// 2k is the arc u -> v, 2k + 1 the arc v -> u.
struct Upd {
  const int32_t *du, *dv, *dw;
  int64_t nd;
  const int32_t *iu, *iv, *iw;
  int64_t ni;
  __device__ __forceinline__ bool is_del(int64_t e) const { return e < 2 * nd; }
  __device__ __forceinline__ int64_t update(int64_t e) const { return e >> 1; }  // index into [del | ins]
  __device__ __forceinline__ void ends(int64_t e, int32_t& a, int32_t& c) const {
    const int64_t k = e >> 1;
    const int32_t x = k < nd ? du[k] : iu[k - nd];
    const int32_t y = k < nd ? dv[k] : iv[k - nd];
    a = (e & 1) ? y : x;
    c = (e & 1) ? x : y;
  }
  __device__ __forceinline__ int32_t weight(int64_t e) const {
    const int64_t k = e >> 1;
    return k < nd ? dw[k] : iw[k - nd];
  }
};

__device__ __forceinline__ bool failed(const int64_t* ctr) {
  return *reinterpret_cast<const volatile int64_t*>(&ctr[CTR_ERR]) != 0;
}

__global__ void k_init(BatchScratch b, int64_t words, int64_t* __restrict__ ctr) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (int64_t i = t0; i < b.size; i += stride) {
    b.keys[i] = kEmpty;
    b.dw[i] = 0;
    b.iw[i] = 0;
    b.pos[2 * i] = -1;
    b.pos[2 * i + 1] = -1;
  }
  for (int64_t i = t0; i < b.dirs; i += stride) {
    b.r_cnt[i] = 0;
    b.r_zero[i] = 0;
    b.r_app[i] = 0;
    b.r_hole[i] = 0;
  }
  for (int64_t i = t0; i < words; i += stride) b.tag[i] = 0;
  for (int64_t i = t0; i < CTR_COUNT; i += stride) ctr[i] = 0;
}

// Validation, the pair table, and the touched rows.  A row is listed
// under the first direction that reaches it: row_slot[vertex] = that
// direction's index e, row_of[e] = vertex (-1 for every other direction).
constexpr uint64_t kTagMul = 2654435761ull;  // a prime above any tag bit count
__global__ void __launch_bounds__(kBlock) k_validate(Upd U, int32_t n, BatchScratch b, int64_t* __restrict__ ctr,
                                                    uint64_t tag_bits) {
  __shared__ int64_t lds[kBlock / kWave];
  int64_t si = 0, sd = 0;
  const int64_t total = U.nd + U.ni;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < total;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const bool del = k < U.nd;
    const int32_t a = del ? U.du[k] : U.iu[k - U.nd];
    const int32_t c = del ? U.dv[k] : U.iv[k - U.nd];
    const int32_t x = del ? U.dw[k] : U.iw[k - U.nd];
    bool ok = a >= 0 && c >= 0 && a < n && c < n && a != c && x > 0;
    int32_t h = -1;
    if (ok) {
      h = static_cast<int32_t>(pair_insert(b.keys, b.size, canon(a, c)));
      if (atomicCAS(del ? &b.dw[h] : &b.iw[h], 0, x) != 0) ok = false;  // pair repeated on this side
    }
    if (ok) {
      if (del)
        sd += x;
      else
        si += x;
    } else {
      set_error(ctr, LV_EINVAL);
      h = -1;
    }
    b.slot[k] = h;
    for (int side = 0; side < 2; ++side) {
      const int32_t r = side ? c : a;
      const int64_t e = 2 * k + side;
      int32_t head = -1;
      if (ok) {
        // Row r's tag is bit (r * kTagMul) mod tag_bits: a bijection (the
        // prime kTagMul exceeds tag_bits), which scatters the rows of
        // neighbouring ids -- in a skewed graph often all hubs, touched by
        // many updates -- over many lines instead of one, whose atomics
        // would queue.
        const int64_t t = static_cast<int64_t>((static_cast<uint64_t>(r) * kTagMul) % tag_bits);
        const uint32_t bit = 1u << (t & 31);
        if ((atomicOr(&b.tag[t >> 5], bit) & bit) == 0) {
          b.row_slot[r] = static_cast<int32_t>(e);
          head = r;
        }
      }
      b.row_of[e] = head;
    }
  }
  si = block_sum(si, lds);
  sd = block_sum(sd, lds);
  if (threadIdx.x == 0) {  // (replicated counters: one address per workgroup would serialise)
    if (si) stat_add(ctr + CTR_STATS0, ST_W_INS, si);
    if (sd) stat_add(ctr + CTR_STATS0, ST_W_DEL, sd);
  }
}

// rank of every direction among the directions of its row
__global__ void k_rank(Upd U, BatchScratch b) {
  const int64_t dirs = 2 * (U.nd + U.ni);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < dirs;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (b.slot[U.update(e)] < 0) {
      b.d_rank[e] = -1;
      continue;
    }
    int32_t a, c;
    U.ends(e, a, c);
    b.d_rank[e] = atomicAdd(&b.r_cnt[b.row_slot[a]], 1);
  }
}

// per touched row: its length, its range in the partner list, its chunks
// (one packed reservation, chunks << 32 | partners, per workgroup and pass
// of kRowsPer rows per thread: the reservations all hit one counter).
constexpr int kRowsPer = 4;
__global__ void __launch_bounds__(kBlock) k_rows(const int64_t* __restrict__ row_start,
                                                 const int32_t* __restrict__ row_len, BatchScratch b,
                                                 int64_t* __restrict__ ctr) {
  __shared__ int64_t lds[kBlock / kWave + 1];
  const int64_t per_pass = static_cast<int64_t>(kBlock) * kRowsPer;
  for (int64_t r0 = blockIdx.x * per_pass; r0 < b.dirs; r0 += static_cast<int64_t>(gridDim.x) * per_pass) {
    int32_t a[kRowsPer], len[kRowsPer], cnt[kRowsPer];
    int64_t rs[kRowsPer];
    int64_t packed = 0;
#pragma unroll
    for (int j = 0; j < kRowsPer; ++j) {
      const int64_t r = r0 + static_cast<int64_t>(j) * kBlock + threadIdx.x;
      a[j] = r < b.dirs ? b.row_of[r] : -1;
    }
#pragma unroll
    for (int j = 0; j < kRowsPer; ++j) {  // (all loads issued together)
      const int64_t r = r0 + static_cast<int64_t>(j) * kBlock + threadIdx.x;
      const bool on = a[j] >= 0;
      len[j] = on ? row_len[a[j]] : 0;
      cnt[j] = on ? b.r_cnt[r] : 0;
      rs[j] = on ? row_start[a[j]] : 0;
    }
#pragma unroll
    for (int j = 0; j < kRowsPer; ++j) {
      if (a[j] < 0) continue;
      const int64_t r = r0 + static_cast<int64_t>(j) * kBlock + threadIdx.x;
      b.r_len[r] = len[j];
      packed += ((static_cast<int64_t>(len[j]) + kChunk - 1) / kChunk << 32) | cnt[j];
    }
    int64_t at = block_reserve(packed, &ctr[CTR_B_RESV], lds);
#pragma unroll
    for (int j = 0; j < kRowsPer; ++j) {
      if (a[j] < 0) continue;
      const int64_t r = r0 + static_cast<int64_t>(j) * kBlock + threadIdx.x;
      const int64_t nch = (static_cast<int64_t>(len[j]) + kChunk - 1) / kChunk;
      const int32_t pbase = static_cast<int32_t>(at & 0xffffffffll);
      const int64_t cbase = at >> 32;
      const int64_t s = rs[j];
      b.r_pbase[r] = pbase;
      for (int64_t q = 0; q < nch; ++q) {
        BatchScratch::Chunk c;
        c.s = s;
        c.a = a[j];
        c.off = static_cast<int32_t>(q * kChunk);
        c.end = static_cast<int32_t>(min(static_cast<int64_t>(len[j]), (q + 1) * kChunk));
        c.cnt = cnt[j];
        c.pbase = pbase;
        c.pad = 0;
        b.chunk[cbase + q] = c;
      }
      at += (nch << 32) | cnt[j];
    }
  }
}

__global__ void k_place(Upd U, BatchScratch b) {
  const int64_t dirs = 2 * (U.nd + U.ni);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < dirs;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t rk = b.d_rank[e];
    if (rk < 0) continue;
    int32_t a, c;
    U.ends(e, a, c);
    b.part[b.r_pbase[b.row_slot[a]] + rk] = c;
  }
}

// One wavefront per chunk: filter of the row's partners in LDS, then every
// arc of the chunk is tested; hits are looked up in the pair table and
// their positions recorded per (pair, direction).
__global__ void __launch_bounds__(kBlock) k_scan(const int64_t* __restrict__ row_start,
                                                 const int32_t* __restrict__ col, BatchScratch b,
                                                 const int64_t* __restrict__ ctr) {
  __shared__ uint32_t filt[kScanWaves][kFilterBits / 32];
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  uint32_t* F = filt[wv];
  const int64_t chunks = ctr[CTR_B_RESV] >> 32;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kScanWaves;
  for (int64_t ch = blockIdx.x * static_cast<int64_t>(kScanWaves) + wv; ch < chunks; ch += nwaves) {
    const BatchScratch::Chunk c = b.chunk[ch];
    const int32_t a = c.a, cnt = c.cnt, pbase = c.pbase, off = c.off, end = c.end;
    const int64_t s = c.s;
    if (end - off <= kWave) {
      // a chunk of at most one arc per lane looks every arc up directly
      // (the filter would cost more round trips than it saves)
      const int32_t k = off + lane;
      if (k < end) {
        const int32_t cc = col[s + k];
        const int32_t p = pair_find(b.keys, b.size, canon(a, cc));
        if (p >= 0) b.pos[2 * static_cast<int64_t>(p) + (a > cc ? 1 : 0)] = s + k;
      }
      continue;
    }
    for (int i = lane; i < kFilterBits / 32; i += kWave) F[i] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int32_t j = lane; j < cnt; j += kWave) {
      const uint32_t h = hash_slot(static_cast<uint32_t>(b.part[pbase + j]), kFilterBits);
      atomicOr(&F[h >> 5], 1u << (h & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // four arcs per lane in flight per step (the loads are independent)
    for (int32_t k0 = off + lane; k0 < end; k0 += 4 * kWave) {
      int32_t cc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t k = k0 + q * kWave;
        cc[q] = k < end ? col[s + k] : -1;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t c = cc[q];
        if (c < 0) continue;
        const uint32_t h = hash_slot(static_cast<uint32_t>(c), kFilterBits);
        if (!((F[h >> 5] >> (h & 31)) & 1u)) continue;
        const int32_t p = pair_find(b.keys, b.size, canon(a, c));
        if (p >= 0) b.pos[2 * static_cast<int64_t>(p) + (a > c ? 1 : 0)] = s + k0 + q * kWave;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Deletions must find their arc with enough weight; insertions merge into
// an arc that survives the deletions, else append.
__global__ void k_check(Upd U, const int32_t* __restrict__ wt, BatchScratch b, int64_t* __restrict__ ctr) {
  const int64_t dirs = 2 * (U.nd + U.ni);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < dirs;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t h = b.slot[U.update(e)];
    if (h < 0) continue;
    int32_t a, c;
    U.ends(e, a, c);
    const int64_t p = b.pos[2 * static_cast<int64_t>(h) + (a > c ? 1 : 0)];
    const int32_t r = b.row_slot[a];
    const int32_t dwh = b.dw[h];
    if (U.is_del(e)) {
      if (p < 0 || wt[p] < dwh) {
        set_error(ctr, LV_ENOEDGE);
        continue;
      }
      if (wt[p] == dwh) atomicAdd(&b.r_zero[r], 1);
    } else {
      const bool merge = p >= 0 && !(dwh > 0 && dwh == wt[p]);
      b.kind[e - 2 * U.nd] = merge ? 1 : 0;
      if (!merge) atomicAdd(&b.r_app[r], 1);
    }
  }
}

__global__ void k_capacity(const int64_t* __restrict__ row_start, const int64_t* __restrict__ two_m, BatchScratch b,
                           int64_t* __restrict__ ctr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t nm = *two_m + 2 * stat_total(ctr + CTR_STATS0, ST_W_INS) - 2 * stat_total(ctr + CTR_STATS0, ST_W_DEL);
    if (nm >= (int64_t(1) << 31)) set_error(ctr, LV_EOVERFLOW);
  }
  for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < b.dirs;
       r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t a = b.row_of[r];
    if (a < 0) continue;
    const int64_t need = static_cast<int64_t>(b.r_len[r]) - b.r_zero[r] + b.r_app[r];
    if (need > row_start[a + 1] - row_start[a]) set_error(ctr, LV_ENOSLACK);
  }
}

// ---- phase 2 ---------------------------------------------------------------

__global__ void k_apply(Upd U, int32_t* __restrict__ wt, int64_t* __restrict__ two_m, BatchScratch b,
                        const int64_t* __restrict__ ctr) {
  if (failed(ctr)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    *two_m += 2 * stat_total(ctr + CTR_STATS0, ST_W_INS) - 2 * stat_total(ctr + CTR_STATS0, ST_W_DEL);
  const int64_t dirs = 2 * (U.nd + U.ni);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < dirs;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t h = b.slot[U.update(e)];
    int32_t a, c;
    U.ends(e, a, c);
    const int64_t p = b.pos[2 * static_cast<int64_t>(h) + (a > c ? 1 : 0)];
    if (U.is_del(e))
      atomicSub(&wt[p], U.weight(e));  // a pair deleted and merged back gets two updates
    else if (b.kind[e - 2 * U.nd])
      atomicAdd(&wt[p], U.weight(e));
  }
}

// Rows with zeroed arcs: the new length is L' = L - zeroed; the arcs of
// the tail [L', L) that survive are copied out (they refill the holes of
// the head [0, L') in k_fill) and the row is cut to L'.  The copies go to
// the row's partner range (zeroed <= partners).  A lane handles a row whose
// tail is short; longer tails take the whole wavefront.
constexpr int kTailLane = 16;
__global__ void __launch_bounds__(kBlock) k_tail(const int64_t* __restrict__ row_start, int32_t* __restrict__ row_len,
                                                 const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                 BatchScratch b, const int64_t* __restrict__ ctr) {
  if (failed(ctr)) return;
  const int lane = lane_id();
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
  for (int64_t s0 = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave * kWave; s0 < b.dirs;
       s0 += nwaves * kWave) {
    const int64_t e = s0 + lane;
    const int32_t a = e < b.dirs ? b.row_of[e] : -1;
    const int32_t z = a >= 0 ? b.r_zero[e] : 0;
    if (z > 0 && z <= kTailLane) {
      const int32_t L = b.r_len[e], Lp = L - z;
      const int64_t s = row_start[a];
      int64_t q = b.r_pbase[e];
      for (int32_t k = Lp; k < L; ++k) {
        const int32_t x = wt[s + k];
        if (x > 0) {
          b.tcol[q] = col[s + k];
          b.tw[q] = x;
          ++q;
        }
      }
      row_len[a] = Lp;
    }
    for (uint64_t m = __ballot(z > kTailLane); m; m &= m - 1) {
      const int64_t r = s0 + (__ffsll(static_cast<unsigned long long>(m)) - 1);
      const int32_t ra = b.row_of[r];
      const int32_t L = b.r_len[r], Lp = L - b.r_zero[r];
      const int64_t s = row_start[ra];
      const int64_t base = b.r_pbase[r];
      int32_t out = 0;
      for (int32_t k0 = Lp; k0 < L; k0 += kWave) {
        const int32_t k = k0 + lane;
        const bool keep = k < L && wt[s + k] > 0;
        const uint64_t km = __ballot(keep);
        if (keep) {
          const int64_t q = base + out + __popcll(km & ((1ull << lane) - 1ull));
          b.tcol[q] = col[s + k];
          b.tw[q] = wt[s + k];
        }
        out += __popcll(km);
      }
      if (lane == 0) row_len[ra] = Lp;
    }
  }
}

// Zeroed head arcs take the row's tail survivors; insertions that do not
// merge are appended after the (cut) row.
__global__ void k_fill(Upd U, const int64_t* __restrict__ row_start, int32_t* __restrict__ row_len,
                       int32_t* __restrict__ col, int32_t* __restrict__ wt, BatchScratch b,
                       const int64_t* __restrict__ ctr) {
  if (failed(ctr)) return;
  const int64_t dirs = 2 * (U.nd + U.ni);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < dirs;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int32_t a, c;
    U.ends(e, a, c);
    const int32_t r = b.row_slot[a];
    const int64_t s = row_start[a];
    if (U.is_del(e)) {
      const int32_t h = b.slot[U.update(e)];
      const int64_t p = b.pos[2 * static_cast<int64_t>(h) + (a > c ? 1 : 0)];
      const int32_t Lp = b.r_len[r] - b.r_zero[r];
      if (p - s >= Lp || wt[p] != 0) continue;  // tail arc, or weight left
      const int32_t j = atomicAdd(&b.r_hole[r], 1);
      col[p] = b.tcol[b.r_pbase[r] + j];
      wt[p] = b.tw[b.r_pbase[r] + j];
    } else if (!b.kind[e - 2 * U.nd]) {
      const int64_t q = s + atomicAdd(&row_len[a], 1);
      col[q] = c;
      wt[q] = U.weight(e);
    }
  }
}

Upd upd(const lv_edges& del, const lv_edges& ins) {
  return Upd{del.u, del.v, del.w, del.count, ins.u, ins.v, ins.w, ins.count};
}

}  // namespace

int64_t batch_chunks_bound(int64_t dirs, int64_t cap) { return dirs + cap / kChunk + 1; }

void launch_batch_phase1(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                         int64_t words, int64_t* ctr, hipStream_t st) {
  const Upd U = upd(del, ins);
  const int64_t total = del.count + ins.count, dirs = 2 * total;
  hipLaunchKernelGGL(k_init, dim3(grid_for(std::max<int64_t>(std::max<int64_t>(b.size, dirs), words), kBlock, 2048)),
                     dim3(kBlock), 0, st, b, words, ctr);
  hipLaunchKernelGGL(k_validate, dim3(grid_for(total, kBlock, 256)), dim3(kBlock), 0, st, U, g.n, b, ctr,
                     static_cast<uint64_t>(words) * 32);
  hipLaunchKernelGGL(k_rank, dim3(grid_for(dirs, kBlock, 4096)), dim3(kBlock), 0, st, U, b);
  hipLaunchKernelGGL(k_rows, dim3(grid_for(dirs, kBlock * kRowsPer, 4096)), dim3(kBlock), 0, st, g.row_start,
                     g.row_len, b, ctr);
  hipLaunchKernelGGL(k_place, dim3(grid_for(dirs, kBlock, 4096)), dim3(kBlock), 0, st, U, b);
  // chunks: one per touched row plus one per kChunk arcs of long rows; the
  // grid covers a few per touched row and strides over the rest
  hipLaunchKernelGGL(k_scan, dim3(grid_for(std::min<int64_t>(4 * dirs + 64, 32768) * kWave, kBlock, 8192)),
                     dim3(kBlock), 0, st, g.row_start, g.col, b, ctr);
  hipLaunchKernelGGL(k_check, dim3(grid_for(dirs, kBlock, 4096)), dim3(kBlock), 0, st, U, g.w, b, ctr);
  hipLaunchKernelGGL(k_capacity, dim3(grid_for(dirs, kBlock, 4096)), dim3(kBlock), 0, st, g.row_start, g.two_m, b,
                     ctr);
}

void launch_batch_phase2(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                         int64_t* ctr, hipStream_t st) {
  const Upd U = upd(del, ins);
  const int64_t dirs = 2 * (del.count + ins.count);
  hipLaunchKernelGGL(k_apply, dim3(grid_for(dirs, kBlock, 4096)), dim3(kBlock), 0, st, U, g.w, g.two_m, b, ctr);
  if (del.count)
    hipLaunchKernelGGL(k_tail, dim3(grid_for(dirs, kBlock, 1024)), dim3(kBlock), 0, st, g.row_start,
                       g.row_len, g.col, g.w, b, ctr);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(dirs, kBlock, 4096)), dim3(kBlock), 0, st, U, g.row_start, g.row_len,
                     g.col, g.w, b, ctr);
}

}  // namespace lv
