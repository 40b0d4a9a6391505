// DF Louvain for many independent graphs in one persistent launch.
//
// One workgroup takes one graph (item) at a time from the descriptor array
// and runs, inside the workgroup, what the single-graph path spreads over
// many launches:
//   A. the batch edit in place (Section 3.4; both arc directions), with
//      all-or-nothing validation (ids, weights, repeated pairs, missing
//      edges, row capacity, 2m bound) before anything is written;
//   B. updateWeights (Alg. 7) and DF's initial marking (Alg. 1);
//   C. the local-moving iterations of pass 0 (Alg. 5): frontier list from
//      the bitmask, one wavefront per vertex with an LDS table (rows up to
//      kManyWaveDeg arcs) or the whole workgroup (rows up to
//      kManyBlockDeg), SYNC (decide all, then apply) or ASYNC (apply at
//      once), expansion to the neighbours of movers, and the convergence
//      test 2 * Σg <= τ (2m)^2.
// A graph whose pass 0 does not converge within one iteration (l_i > 1)
// needs aggregation and more passes (Alg. 4); its item is marked and the
// host continues it on the single-graph path from that state.
//
// The graphs are small (one workgroup each) and thousands of them fill the
// GPU together, so the per-graph work is serial inside the workgroup:
// shared data is read with agent-scope atomic loads after other lanes of
// the workgroup wrote it with device atomics, and phases are separated by
// workgroup barriers.
#include <algorithm>
#include <climits>

#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int64_t kTwoMLimit = int64_t(1) << 31;
constexpr int kNW = kBlock / kWave;

template <class T>
__device__ __forceinline__ T ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t pair_key(int32_t a, int32_t b) {  // never 0 (a != b)
  const uint32_t lo = static_cast<uint32_t>(min(a, b)), hi = static_cast<uint32_t>(max(a, b));
  return ((static_cast<uint64_t>(lo) << 32) | hi) + 1;
}

__device__ __forceinline__ uint32_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return static_cast<uint32_t>(k);
}

__device__ __forceinline__ bool better(int64_t g1, int32_t c1, int64_t g0, int32_t c0) {
  return g1 > g0 || (g1 == g0 && c1 < c0);
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* r) {
  v = wave_sum_i64(v);
  __syncthreads();
  if (lane_id() == 0) r[threadIdx.x / kWave] = v;
  __syncthreads();
  int64_t s = 0;
  for (int t = 0; t < kNW; ++t) s += r[t];
  return s;
}

__device__ __forceinline__ int64_t block_max(int64_t v, int64_t* r) {
  for (int s = 32; s > 0; s >>= 1) v = max(v, __shfl_xor(v, s));
  __syncthreads();
  if (lane_id() == 0) r[threadIdx.x / kWave] = v;
  __syncthreads();
  int64_t m = r[0];
  for (int t = 1; t < kNW; ++t) m = max(m, r[t]);
  return m;
}

__device__ __forceinline__ void block_best(int64_t& bg, int32_t& bc, int64_t* rg, int32_t* rc) {
  for (int s = 1; s < kWave; s <<= 1) {
    const int64_t og = __shfl_xor(bg, s);
    const int32_t oc = __shfl_xor(bc, s);
    if (better(og, oc, bg, bc)) {
      bg = og;
      bc = oc;
    }
  }
  __syncthreads();
  if (lane_id() == 0) {
    rg[threadIdx.x / kWave] = bg;
    rc[threadIdx.x / kWave] = bc;
  }
  __syncthreads();
  for (int t = 0; t < kNW; ++t)
    if (better(rg[t], rc[t], bg, bc)) {
      bg = rg[t];
      bc = rc[t];
    }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Shared {
  union {
    struct {
      int32_t keys[kNW][2 * kManyWaveDeg];
      int32_t vals[kNW][2 * kManyWaveDeg];
    } w;
    struct {
      int32_t keys[2 * kManyBlockDeg];
      int32_t vals[2 * kManyBlockDeg];
    } b;
    int32_t scan[kBlock];
  } u;
  int64_t red[kNW];
  int32_t redc[kNW];
  int32_t err;
  int32_t nlist;
  int32_t nbig;
};

// Scratch of one item.  The bitmasks and the two tables are zero on entry
// and left zero; the arrays are written before they are read.
//   cur, next, ever: frontier bitmasks; list: frontier list (and, after it,
//   the workgroup-row list); tgt: SYNC targets; pairs: table of the batch's
//   pairs; rows: table of touched rows; pos: per update direction, the arc's
//   offset in its row (or -1) and whether an insertion merges.
struct ItemScratch {
  uint32_t* cur;
  uint32_t* next;
  uint32_t* ever;
  int32_t* list;
  int32_t* tgt;
  uint64_t* pkey;
  int32_t* pdw;
  int32_t* piw;
  int32_t* rkey;
  int32_t* rzero;
  int32_t* rapp;
  int32_t* pos;
  int32_t* kind;
  int32_t psize;  // power of two
  int32_t rsize;
};

__device__ __forceinline__ ItemScratch carve(const ManyItem& it) {
  ItemScratch s;
  const int64_t words = (static_cast<int64_t>(it.n) + 31) / 32 + 1;
  const int32_t cap = it.max_updates;
  int32_t ps = 64;
  while (ps < 2 * cap) ps <<= 1;
  int32_t rs = 64;
  while (rs < 4 * cap) rs <<= 1;
  char* p = static_cast<char*>(it.scratch);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~size_t(255);
    return q;
  };
  s.cur = reinterpret_cast<uint32_t*>(take(4 * words));
  s.next = reinterpret_cast<uint32_t*>(take(4 * words));
  s.ever = reinterpret_cast<uint32_t*>(take(4 * words));
  s.list = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(it.n) + 4));
  s.tgt = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(it.n) + 4));
  s.pkey = reinterpret_cast<uint64_t*>(take(8 * static_cast<size_t>(ps)));
  s.pdw = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(ps)));
  s.piw = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(ps)));
  s.rkey = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(rs)));
  s.rzero = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(rs)));
  s.rapp = reinterpret_cast<int32_t*>(take(4 * static_cast<size_t>(rs)));
  s.pos = reinterpret_cast<int32_t*>(take(8 * static_cast<size_t>(cap) + 4));
  s.kind = reinterpret_cast<int32_t*>(take(8 * static_cast<size_t>(cap) + 4));
  s.psize = ps;
  s.rsize = rs;
  return s;
}

// slot of the pair key (inserting it); the table never fills (2x updates)
__device__ __forceinline__ int32_t pair_slot(const ItemScratch& s, uint64_t key) {
  uint32_t h = mix64(key) & (s.psize - 1);
  while (true) {
    const unsigned long long old =
        atomicCAS(reinterpret_cast<unsigned long long*>(&s.pkey[h]), 0ull, static_cast<unsigned long long>(key));
    if (old == 0 || old == key) return static_cast<int32_t>(h);
    h = (h + 1) & (s.psize - 1);
  }
}

__device__ __forceinline__ int32_t row_slot(const ItemScratch& s, int32_t row) {  // key row + 1
  uint32_t h = hash_slot(static_cast<uint32_t>(row), s.rsize);
  while (true) {
    const int32_t old = atomicCAS(&s.rkey[h], 0, row + 1);
    if (old == 0 || old == row + 1) return static_cast<int32_t>(h);
    h = (h + 1) & (s.rsize - 1);
  }
}

__device__ __forceinline__ void set_err(Shared& sh, int32_t code) { atomicCAS(&sh.err, 0, code); }

// ---- A: the batch edit ------------------------------------------------------
// Returns the status; on error nothing of the graph was written.
__device__ int32_t edit_graph(const ManyItem& it, const ItemScratch& s, Shared& sh) {
  const int32_t nd = it.nd, ni = it.ni, U = nd + ni, n = it.n;
  if (threadIdx.x == 0) sh.err = 0;
  __syncthreads();
  int64_t si = 0, sd = 0;
  // A1: ids, weights, repeated pairs
  for (int32_t k = threadIdx.x; k < U; k += kBlock) {
    const bool del = k < nd;
    const int32_t a = del ? it.du[k] : it.iu[k - nd];
    const int32_t c = del ? it.dv[k] : it.iv[k - nd];
    const int32_t x = del ? it.dw[k] : it.iw[k - nd];
    if (a < 0 || c < 0 || a >= n || c >= n || a == c || x <= 0) {
      set_err(sh, LV_EINVAL);
      continue;
    }
    const int32_t h = pair_slot(s, pair_key(a, c));
    if (atomicCAS(del ? &s.pdw[h] : &s.piw[h], 0, x) != 0) set_err(sh, LV_EINVAL);
    if (del)
      sd += x;
    else
      si += x;
  }
  si = block_sum(si, sh.red);
  sd = block_sum(sd, sh.red);
  // A2: arc positions, deletion checks, merge or append
  if (sh.err == 0) {
    for (int32_t e = threadIdx.x; e < 2 * U; e += kBlock) {
      const int32_t k = e >> 1;
      const bool del = k < nd;
      const int32_t x0 = del ? it.du[k] : it.iu[k - nd];
      const int32_t y0 = del ? it.dv[k] : it.iv[k - nd];
      const int32_t a = (e & 1) ? y0 : x0, c = (e & 1) ? x0 : y0;
      const int64_t rs = it.row_start[a];
      const int32_t len = it.row_len[a];
      int32_t p = -1;
      for (int32_t q = 0; q < len; ++q)
        if (it.col[rs + q] == c) {
          p = q;
          break;
        }
      s.pos[e] = p;
      const int32_t h = pair_slot(s, pair_key(a, c));
      const int32_t dwp = s.pdw[h];
      if (del) {
        if (p < 0 || it.w[rs + p] < dwp) {
          set_err(sh, LV_ENOEDGE);
        } else if (it.w[rs + p] == dwp) {
          atomicAdd(&s.rzero[row_slot(s, a)], 1);
        }
      } else {
        const bool merge = p >= 0 && !(dwp > 0 && dwp == it.w[rs + p]);
        s.kind[e] = merge ? 1 : 0;
        if (!merge) atomicAdd(&s.rapp[row_slot(s, a)], 1);
      }
    }
  }
  __syncthreads();
  // A3: capacities, the 2m bound, and the longest row after the edit (a
  // row longer than a workgroup's table is left to the single-graph path)
  int64_t longest = 0;
  if (sh.err == 0) {
    if (threadIdx.x == 0 && *it.two_m + 2 * si - 2 * sd >= kTwoMLimit) set_err(sh, LV_EOVERFLOW);
    for (int32_t h = threadIdx.x; h < s.rsize; h += kBlock) {
      const int32_t key = ld(&s.rkey[h]);
      if (!key) continue;
      const int32_t a = key - 1;
      const int64_t need = static_cast<int64_t>(it.row_len[a]) - ld(&s.rzero[h]) + ld(&s.rapp[h]);
      if (need > it.row_start[a + 1] - it.row_start[a]) set_err(sh, LV_ENOSLACK);
      longest = max(longest, need);
    }
    for (int32_t v = threadIdx.x; v < n; v += kBlock) longest = max(longest, static_cast<int64_t>(it.row_len[v]));
  }
  longest = block_max(longest, sh.red);
  if (longest > kManyBlockDeg && threadIdx.x == 0) set_err(sh, LV_ETOOLARGE);
  __syncthreads();
  const int32_t status = sh.err;
  if (status == 0) {
    // A4: weights of deletions and merges
    for (int32_t e = threadIdx.x; e < 2 * U; e += kBlock) {
      const int32_t k = e >> 1;
      const bool del = k < nd;
      const int32_t x0 = del ? it.du[k] : it.iu[k - nd];
      const int32_t y0 = del ? it.dv[k] : it.iv[k - nd];
      const int32_t a = (e & 1) ? y0 : x0;
      const int32_t p = ld(&s.pos[e]);
      if (del)
        atomicSub(&it.w[it.row_start[a] + p], it.dw[k]);
      else if (ld(&s.kind[e]))
        atomicAdd(&it.w[it.row_start[a] + p], it.iw[k - nd]);
    }
    __syncthreads();
    // A5: rows that lost arcs are compacted (one lane per row, rows are short)
    for (int32_t h = threadIdx.x; h < s.rsize; h += kBlock) {
      const int32_t key = ld(&s.rkey[h]);
      if (!key || ld(&s.rzero[h]) == 0) continue;
      const int32_t a = key - 1;
      const int64_t rs = it.row_start[a];
      const int32_t len = ld(&it.row_len[a]);
      int32_t o = 0;
      for (int32_t q = 0; q < len; ++q) {
        const int32_t x = ld(&it.w[rs + q]);
        if (x > 0) {
          it.col[rs + o] = ld(&it.col[rs + q]);
          it.w[rs + o] = x;
          ++o;
        }
      }
      it.row_len[a] = o;
    }
    __syncthreads();
    // A6: appends
    for (int32_t e = threadIdx.x; e < 2 * ni; e += kBlock) {
      const int32_t k = nd + (e >> 1);
      const int32_t ed = 2 * nd + e;
      if (ld(&s.kind[ed])) continue;
      const int32_t x0 = it.iu[k - nd], y0 = it.iv[k - nd];
      const int32_t a = (e & 1) ? y0 : x0, c = (e & 1) ? x0 : y0;
      const int64_t q = it.row_start[a] + atomicAdd(&it.row_len[a], 1);
      it.col[q] = c;
      it.w[q] = it.iw[k - nd];
    }
    if (threadIdx.x == 0) *it.two_m += 2 * si - 2 * sd;
  }
  __syncthreads();
  // tables back to zero
  for (int32_t h = threadIdx.x; h < s.psize; h += kBlock) {
    s.pkey[h] = 0;
    s.pdw[h] = 0;
    s.piw[h] = 0;
  }
  for (int32_t h = threadIdx.x; h < s.rsize; h += kBlock) {
    s.rkey[h] = 0;
    s.rzero[h] = 0;
    s.rapp[h] = 0;
  }
  __syncthreads();
  return status;
}

// ---- B: updateWeights and DF marking ----------------------------------------
__device__ void update_and_mark(const ManyItem& it, const ItemScratch& s) {
  const int32_t nd = it.nd, U = nd + it.ni;
  for (int32_t k = threadIdx.x; k < U; k += kBlock) {
    const bool del = k < nd;
    const int32_t a = del ? it.du[k] : it.iu[k - nd];
    const int32_t b = del ? it.dv[k] : it.iv[k - nd];
    const int64_t x = del ? -static_cast<int64_t>(it.dw[k]) : static_cast<int64_t>(it.iw[k - nd]);
    const int32_t ca = it.C[a], cb = it.C[b];
    atomic_add_i64(&it.K[a], x);
    atomic_add_i64(&it.K[b], x);
    atomic_add_i64(&it.Sigma[ca], x);
    atomic_add_i64(&it.Sigma[cb], x);
    if ((ca == cb) == del) {
      set_bit(s.cur, a);
      set_bit(s.cur, b);
    }
  }
  __syncthreads();
}

// ---- C: local moving, pass 0 ------------------------------------------------
struct MoveCfg {
  int64_t two_m;
  int32_t mode;
  int32_t guard;
};

__device__ __forceinline__ bool decide(const ManyItem& it, const MoveCfg& m, int32_t d, int32_t c, int64_t g) {
  if (c == INT_MAX || g <= 0) return false;
  if (m.guard && ld(&it.size[d]) == 1 && ld(&it.size[c]) == 1 && c > d) return false;
  return true;
}

__device__ __forceinline__ void apply_move(const ManyItem& it, int32_t v, int32_t d, int32_t c) {
  const int64_t Kv = ld(&it.K[v]);
  it.C[v] = c;
  atomic_add_i64(&it.Sigma[d], -Kv);
  atomic_add_i64(&it.Sigma[c], Kv);
  atomicSub(&it.size[d], 1);
  atomicAdd(&it.size[c], 1);
}

__device__ __forceinline__ void push_neighbours(const ManyItem& it, const ItemScratch& s, int32_t v, int32_t from,
                                                int32_t step) {
  const int64_t rs = it.row_start[v];
  const int32_t len = ld(&it.row_len[v]);
  for (int32_t q = from; q < len; q += step) {
    const int32_t j = ld(&it.col[rs + q]);
    if (j != v) set_bit(s.next, j);
  }
}

// One vertex by one wavefront (table of 2*kManyWaveDeg slots).  Returns the
// gain of the move it decided (lane 0), 0 otherwise.
__device__ int64_t scan_wave(const ManyItem& it, const ItemScratch& s, const MoveCfg& m, int32_t v, int32_t* keys,
                             int32_t* vals) {
  const int lane = lane_id();
  const int64_t rs = it.row_start[v];
  const int32_t deg = ld(&it.row_len[v]);
  const int32_t d = ld(&it.C[v]);
  const uint32_t ts = max(64u, 1u << (32 - __clz(static_cast<uint32_t>(2 * max(deg, 1) - 1))));
  for (uint32_t t = lane; t < ts; t += kWave) {
    keys[t] = -1;
    vals[t] = 0;
  }
  wave_sync();
  int32_t kid = 0;
  for (int32_t q = lane; q < deg; q += kWave) {
    const int32_t j = ld(&it.col[rs + q]);
    const int32_t x = ld(&it.w[rs + q]);
    if (j == v) continue;
    const int32_t c = ld(&it.C[j]);
    if (c == d) {
      kid += x;
      continue;
    }
    uint32_t h = hash_slot(static_cast<uint32_t>(c), ts);
    while (true) {
      const int32_t old = atomicCAS(&keys[h], -1, c);
      if (old == -1 || old == c) {
        atomicAdd(&vals[h], x);
        break;
      }
      h = (h + 1) & (ts - 1);
    }
  }
  wave_sync();
  kid = wave_sum_i32(kid);
  const int64_t Kv = ld(&it.K[v]);
  const int64_t Sd = ld(&it.Sigma[d]);
  // candidates whose gain bound K_{v->c} (2m - K_v) - tb is not positive
  // (Σ_c >= K_{v->c}) cannot be chosen; their Σ_c is not read
  const int64_t tb = m.two_m * kid - Kv * (Sd - Kv), dm = m.two_m - Kv;
  int64_t bg = LLONG_MIN;
  int32_t bc = INT_MAX;
  for (uint32_t t = lane; t < ts; t += kWave) {
    const int32_t c = keys[t];
    if (c < 0 || static_cast<int64_t>(vals[t]) * dm <= tb) continue;
    const int64_t g = m.two_m * (static_cast<int64_t>(vals[t]) - kid) - Kv * (ld(&it.Sigma[c]) - Sd + Kv);
    if (better(g, c, bg, bc)) {
      bg = g;
      bc = c;
    }
  }
  for (int sft = 1; sft < kWave; sft <<= 1) {
    const int64_t og = __shfl_xor(bg, sft);
    const int32_t oc = __shfl_xor(bc, sft);
    if (better(og, oc, bg, bc)) {
      bg = og;
      bc = oc;
    }
  }
  wave_sync();  // the table is reused by the wavefront's next vertex
  const bool mv = decide(it, m, d, bc, bg);
  if (m.mode == LV_SYNC) {
    if (lane == 0) s.tgt[v] = mv ? bc : -1;
    return (mv && lane == 0) ? bg : 0;
  }
  if (mv) {
    if (lane == 0) apply_move(it, v, d, bc);
    push_neighbours(it, s, v, lane, kWave);
  }
  return (mv && lane == 0) ? bg : 0;
}

// One vertex by the whole workgroup (table of 2*kManyBlockDeg slots).
__device__ int64_t scan_block(const ManyItem& it, const ItemScratch& s, const MoveCfg& m, int32_t v, Shared& sh) {
  const int64_t rs = it.row_start[v];
  const int32_t deg = ld(&it.row_len[v]);
  const int32_t d = ld(&it.C[v]);
  int32_t* keys = sh.u.b.keys;
  int32_t* vals = sh.u.b.vals;
  const uint32_t ts = max(256u, 1u << (32 - __clz(static_cast<uint32_t>(2 * deg - 1))));
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
    keys[t] = -1;
    vals[t] = 0;
  }
  __syncthreads();
  int64_t kid = 0;
  for (int32_t q = threadIdx.x; q < deg; q += kBlock) {
    const int32_t j = ld(&it.col[rs + q]);
    const int32_t x = ld(&it.w[rs + q]);
    if (j == v) continue;
    const int32_t c = ld(&it.C[j]);
    if (c == d) {
      kid += x;
      continue;
    }
    uint32_t h = hash_slot(static_cast<uint32_t>(c), ts);
    while (true) {
      const int32_t old = atomicCAS(&keys[h], -1, c);
      if (old == -1 || old == c) {
        atomicAdd(&vals[h], x);
        break;
      }
      h = (h + 1) & (ts - 1);
    }
  }
  kid = block_sum(kid, sh.red);
  const int64_t Kv = ld(&it.K[v]);
  const int64_t Sd = ld(&it.Sigma[d]);
  const int64_t tb = m.two_m * kid - Kv * (Sd - Kv), dm = m.two_m - Kv;  // as in scan_wave
  int64_t bg = LLONG_MIN;
  int32_t bc = INT_MAX;
  for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
    const int32_t c = keys[t];
    if (c < 0 || static_cast<int64_t>(vals[t]) * dm <= tb) continue;
    const int64_t g = m.two_m * (static_cast<int64_t>(vals[t]) - kid) - Kv * (ld(&it.Sigma[c]) - Sd + Kv);
    if (better(g, c, bg, bc)) {
      bg = g;
      bc = c;
    }
  }
  block_best(bg, bc, sh.red, sh.redc);
  const bool mv = decide(it, m, d, bc, bg);
  if (m.mode == LV_SYNC) {
    if (threadIdx.x == 0) s.tgt[v] = mv ? bc : -1;
  } else if (mv) {
    if (threadIdx.x == 0) apply_move(it, v, d, bc);
    push_neighbours(it, s, v, threadIdx.x, kBlock);
  }
  __syncthreads();
  return (mv && threadIdx.x == 0) ? bg : 0;
}

// Frontier bitmask -> list (clearing the words), with the degree split:
// rows up to wave_deg (at most kManyWaveDeg: the LDS tables hold twice
// that) from the front of the list, longer ones from the back.  Counts first-time vertices and scanned arcs.
__device__ void build_list(const ManyItem& it, const ItemScratch& s, Shared& sh, int32_t wave_deg, int64_t& affected,
                           int64_t& arcs) {
  const int64_t words = (static_cast<int64_t>(it.n) + 31) / 32;
  if (threadIdx.x == 0) {
    sh.nlist = 0;
    sh.nbig = 0;
  }
  __syncthreads();
  for (int64_t k = threadIdx.x; k < words; k += kBlock) {
    const uint32_t bits = ld(&s.cur[k]);
    if (!bits) continue;
    s.cur[k] = 0;
    const uint32_t old = s.ever[k];
    affected += __popc(bits & ~old);
    s.ever[k] = old | bits;
    for (uint32_t r = bits; r; r &= r - 1) {
      const int32_t v = static_cast<int32_t>(k * 32 + (__ffs(r) - 1));
      const int32_t deg = ld(&it.row_len[v]);
      arcs += deg;
      if (deg <= wave_deg)
        s.list[atomicAdd(&sh.nlist, 1)] = v;
      else
        s.list[it.n - 1 - atomicAdd(&sh.nbig, 1)] = v;
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBlock) k_many_df(const int32_t* __restrict__ count_ptr,
                                                   ManyItem* __restrict__ items, double tol, int32_t max_iterations,
                                                   int32_t mode, int32_t guard, int32_t wave_deg) {
  __shared__ Shared sh;
  const int32_t count = *count_ptr;  // the descriptor header: a captured launch serves any count
  for (int32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const ManyItem& it = items[idx];  // uniform: fields come through the scalar cache
    if (it.status != 0) continue;      // rejected by the host (sizes)
    const ItemScratch s = carve(it);
    int32_t status = edit_graph(it, s, sh);
    if (status == LV_ETOOLARGE) {  // nothing written: the single-graph path takes it
      if (threadIdx.x == 0) items[idx].status = status;
      continue;
    }
    int64_t two_m = ld(it.two_m);
    if (status == 0 && two_m <= 0) status = LV_EEMPTY;
    if (status != 0) {
      if (threadIdx.x == 0) items[idx].status = status;
      continue;
    }
    update_and_mark(it, s);
    const MoveCfg m{two_m, mode, guard};
    int64_t moves = 0, arcs_total = 0, affected_total = 0;
    int32_t li = max_iterations;
    uint32_t* cur = s.cur;
    uint32_t* next = s.next;
    for (int32_t iter = 0; iter < max_iterations; ++iter) {
      ItemScratch si = s;
      si.cur = cur;
      si.next = next;
      int64_t affected = 0, arcs = 0;
      build_list(it, si, sh, wave_deg, affected, arcs);
      const int32_t nsmall = sh.nlist, nbig = sh.nbig;
      int64_t gain = 0, movers = 0;
      // wavefront rows
      const int wv = threadIdx.x / kWave;
      for (int32_t q = wv; q < nsmall; q += kNW) {
        const int32_t v = s.list[q];
        const int64_t g = scan_wave(it, si, m, v, sh.u.w.keys[wv], sh.u.w.vals[wv]);
        gain += g;
        movers += g > 0 ? 1 : 0;
      }
      __syncthreads();
      // workgroup rows
      for (int32_t q = 0; q < nbig; ++q) {
        const int32_t v = s.list[it.n - 1 - q];
        const int64_t g = scan_block(it, si, m, v, sh);
        gain += g;
        movers += g > 0 ? 1 : 0;
      }
      __syncthreads();
      if (mode == LV_SYNC) {  // apply every recorded move, then expand
        for (int32_t q = threadIdx.x; q < nsmall + nbig; q += kBlock) {
          const int32_t v = q < nsmall ? s.list[q] : s.list[it.n - 1 - (q - nsmall)];
          const int32_t c = ld(&s.tgt[v]);
          if (c >= 0) apply_move(it, v, ld(&it.C[v]), c);
        }
        __syncthreads();
        for (int32_t q = threadIdx.x; q < nsmall + nbig; q += kBlock) {
          const int32_t v = q < nsmall ? s.list[q] : s.list[it.n - 1 - (q - nsmall)];
          if (ld(&s.tgt[v]) >= 0) push_neighbours(it, si, v, 0, 1);
        }
        __syncthreads();
      }
      gain = block_sum(gain, sh.red);
      movers = block_sum(movers, sh.red);
      affected = block_sum(affected, sh.red);
      arcs = block_sum(arcs, sh.red);
      moves += movers;
      arcs_total += arcs;
      affected_total += affected;
      if (threadIdx.x == 0 && iter < kManyIters) {
        items[idx].iter_moves[iter] = movers;
        items[idx].iter_gain[iter] = gain;
      }
      const uint32_t* t = cur;
      cur = next;
      next = const_cast<uint32_t*>(t);
      const double tm = static_cast<double>(two_m);
      if (2.0 * static_cast<double>(gain) / (tm * tm) <= tol) {
        li = iter + 1;
        break;
      }
    }
    // frontier and visited bitmasks back to zero
    const int64_t words = (static_cast<int64_t>(it.n) + 31) / 32;
    for (int64_t k = threadIdx.x; k < words; k += kBlock) {
      cur[k] = 0;
      next[k] = 0;
      s.ever[k] = 0;
    }
    if (threadIdx.x == 0) {
      items[idx].iterations = li;
      items[idx].moves = moves;
      items[idx].arcs_scanned = arcs_total;
      items[idx].vertices_affected = affected_total;
      items[idx].status = 0;
    }
    __syncthreads();
  }
}

}  // namespace

size_t many_scratch_bytes(int32_t n, int32_t max_updates) {
  const size_t words = (static_cast<size_t>(n > 0 ? n : 1) + 31) / 32 + 1;
  const size_t cap = static_cast<size_t>(max_updates > 0 ? max_updates : 1);
  size_t ps = 64;
  while (ps < 2 * cap) ps <<= 1;
  size_t rs = 64;
  while (rs < 4 * cap) rs <<= 1;
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t un = static_cast<size_t>(n > 0 ? n : 1);
  return 3 * a(4 * words) + 2 * a(4 * un + 4) + a(8 * ps) + 2 * a(4 * ps) + 3 * a(4 * rs) + 2 * a(8 * cap + 4);
}

void launch_many_df(const int32_t* count, ManyItem* items, int32_t grid, const lv_params& p, int32_t wave_deg,
                    hipStream_t st) {
  wave_deg = std::max(1, std::min(wave_deg, kManyWaveDeg));
  hipLaunchKernelGGL(k_many_df, dim3(grid), dim3(kBlock), 0, st, count, items, p.tolerance, p.max_iterations,
                     p.mode, p.swap_guard, wave_deg);
}

}  // namespace lv
