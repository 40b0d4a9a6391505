// Internal declarations shared by the library's HIP translation units:
// workspace layout, device helpers and the host-side launchers of every
// kernel.  Not part of the public interface (see include/louvain.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "louvain.h"

namespace lv {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // 4 wavefronts

// Degree bins of the local-moving phase.  Rows of length 1..32 are handled
// by groups of 4/8/16/32 lanes (one arc per lane), longer rows up to the
// wave threshold by one wavefront with an LDS hashtable, rows up to
// kBlockMaxDegree by one workgroup with an LDS hashtable, and the rest (hub
// rows) by many workgroups sharing a global-memory hashtable.
enum Bin { BIN_G4 = 0, BIN_G8, BIN_G16, BIN_G32, BIN_WAVE, BIN_BLOCK, BIN_HUB, NBINS };

constexpr int kWaveTableMaxDegree = 512;  // largest wave-bin row the LDS table supports
constexpr int kBlockMaxDegree = 2048;     // largest workgroup-bin row (LDS table of 4096 slots)
constexpr int kHubUnitArcs = 2048;        // arcs per work unit of a hub row (8 per thread)
constexpr int kHubClearSlots = 4096;      // table slots per clear unit of a hub row

// Device counters (int64 slots of Workspace::ctr).  Device-scope atomics
// on MI355X are executed at the memory side and serialise per 128-byte line
// (about 12 ns each), so every counter owns a line of its own, and the
// statistics summed by every workgroup are spread over kStatReplicas
// replicas (replica = workgroup id mod kStatReplicas) that the host adds up.
//
// Sub-round counters (bin sizes, hub units) and per-iteration statistics
// each come in two sets used alternately, so no clear has to be launched
// between rounds or iterations: the first kernel of a round zeroes the set
// the next round will use (the previous round's, already consumed), and the
// first kernel of an iteration zeroes the statistics set of the iteration
// after it (the host read it at the end of the previous iteration).
constexpr int kCtrLine = 16;        // int64 slots per 128-byte line
constexpr int64_t kRowListPad = 8192;  // bin lists hold n + this many entries (row-sum region lists)
constexpr int kStatReplicas = 32;
constexpr int kStatStride = 2 * kCtrLine;  // slots per replica (two lines)
constexpr int kStatSet = kStatReplicas * kStatStride;
constexpr int kHotRegions = 16;     // reservation counters of the deferred-total records
constexpr int kRoundSet = (10 + kHotRegions) * kCtrLine;
enum Ctr {
  CTR_ERR = 0 * kCtrLine,        // error code (first nonzero wins)
  CTR_TOTAL = 1 * kCtrLine,      // generic total (scans, counts)
  CTR_AUX0 = 2 * kCtrLine,
  CTR_AUX1 = 3 * kCtrLine,
  CTR_AUX2 = 4 * kCtrLine,
  CTR_AUX3 = 5 * kCtrLine,
  CTR_TWO_M = 6 * kCtrLine,      // 2m as read by the first kernel of a louvain call
  CTR_AGG_SMALL = 7 * kCtrLine,  // aggregation: communities per tier, unit counts, pool
  CTR_AGG_MEDIUM = 8 * kCtrLine,
  CTR_AGG_BIG = 9 * kCtrLine,
  CTR_UNITS_INS = 10 * kCtrLine,
  CTR_UNITS_EMIT = 11 * kCtrLine,
  CTR_AGG_POOL = 12 * kCtrLine,
  CTR_B_RESV = 13 * kCtrLine,    // apply_batch: packed (chunks << 32 | partners) reserved
  CTR_STATS0 = 16 * kCtrLine,    // two statistics sets of kStatSet slots
  CTR_ROUND0 = CTR_STATS0 + 2 * kStatSet,  // two sub-round sets of kRoundSet slots
  CTR_FL0 = CTR_ROUND0 + 2 * kRoundSet,    // two frontier-list count sets of kFlSet slots
  CTR_COUNT = CTR_FL0 + 2 * (32 * kCtrLine)
};
// Frontier lists.  Next to each frontier bitmask the vertices whose bit is
// set are listed, so that binning reads the frontier rather than every
// bitmask word.  A list has kFlRegions regions (writers append to the region
// of their workgroup id modulo kFlRegions, one counter line each, so the
// appends of many workgroups do not queue on one address).  The list is
// valid while every region count is at most its capacity; a count above it
// (an overfull region, or kFlInvalid written by a kernel that sets bits
// without listing them) makes binning walk the bitmask words instead.
constexpr int kFlRegions = 32;
constexpr int kFlSet = kFlRegions * kCtrLine;
constexpr int64_t kFlInvalid = int64_t(1) << 60;
static_assert(CTR_COUNT == CTR_FL0 + 2 * kFlSet, "frontier-list counters");
struct FrontList {
  int32_t* list;   // kFlRegions regions of capr entries
  int64_t* cnt;    // region r's count at cnt[r * kCtrLine]
  int64_t capr;
};
// sub-round counters, offsets inside a round set
enum RoundCtr {
  RC_BIN0 = 0,                   // lines 0 .. NBINS-1: items per bin (rc_bin)
  RC_POOL = 7 * kCtrLine,        // hub table slots handed out
  RC_HUB_UNITS = 8 * kCtrLine,   // hub insert units
  RC_HUB_CUNITS = 9 * kCtrLine,  // hub table-slot (clear / decide) units
  RC_HOT = 10 * kCtrLine         // lines 10 .. 10+kHotRegions-1: deferred-total records per region
};
// per-iteration statistics, slots of every replica
enum Stat {
  ST_MOVERS = 0,  // moves decided
  ST_GAIN,        // sum of the movers' gains
  ST_ARCS,        // arcs of processed vertices (edges scanned)
  ST_PROCESSED,   // vertices processed
  ST_EXPAND,      // arcs of movers (bound on the next frontier)
  ST_AFFECTED,    // vertices processed for the first time in the call
  ST_INTRA,       // modularity: weight of arcs inside communities
  ST_BIN_V0,      // .. + NBINS - 1: vertices processed per bin
  ST_BIN_A0 = ST_BIN_V0 + 7,  // .. + NBINS - 1: arcs scanned per bin
  ST_W_INS = ST_BIN_A0 + 7,   // batch edit (first set): total weight of the insertions
  ST_W_DEL,                   // ... and of the deletions
  NSTATS
};
static_assert(NSTATS <= kStatStride, "statistics exceed a replica");
constexpr int rc_bin(int b) { return RC_BIN0 + b * kCtrLine; }


struct LevelGraph {
  int32_t n = 0;
  int64_t* row_start = nullptr;  // n + 1
  int32_t* row_len = nullptr;    // n
  int32_t* col = nullptr;
  int32_t* w = nullptr;
};

// Carving of the caller's workspace.  Every region is 256-byte aligned.
// A move role's change to a large community's total and size, applied after
// the scan launch (k_hot_apply) instead of by device atomics at the end of
// every workgroup.
struct HotRec {
  int32_t c;
  int32_t ds;
  int64_t dk;
};
constexpr int64_t kHotCap = 8192;  // records per region

struct Workspace {
  int32_t n = 0;
  int64_t cap = 0;
  int64_t words = 0;
  uint32_t* fr_a = nullptr;   // frontier bitmasks (current / next)
  uint32_t* fr_b = nullptr;
  uint32_t* ever = nullptr;   // vertices processed in pass 0
  uint32_t* range = nullptr;  // DS affected range
  uint32_t* dE = nullptr;     // DS: neighbours-affected flags
  uint32_t* dC = nullptr;     // DS: community-affected flags
  uint32_t* moved = nullptr;  // vertices moved in this iteration (pull expansion)
  uint8_t* push_flags = nullptr;  // one byte per vertex (32 per frontier word) for the push expansion
  int32_t* fl[2] = {};        // frontier lists of fr_a and fr_b (kFlRegions regions of fl_capr)
  int64_t fl_capr = 0;
  int32_t* bins[NBINS] = {};
  int64_t* hub_off = nullptr;  // global-table offset of each hub item
  int64_t* hub_kid = nullptr;  // hub items: weight into the vertex's own community
  int32_t* hub_moved = nullptr;
  int64_t* hub_cbase = nullptr;  // hub items: first table-slot unit and unit count
  int32_t* hub_cnum = nullptr;
  int64_t* unit_g = nullptr;     // per table-slot unit: best gain and community
  int32_t* unit_c = nullptr;
  int32_t* mv_c = nullptr;     // SYNC: target community of each mover (by vertex)
  int32_t* size = nullptr;     // community sizes (swap guard)
  int32_t* lC = nullptr;       // level >= 1 membership, weights, totals
  int64_t* lK = nullptr;
  int64_t* lS = nullptr;
  int32_t* flags = nullptr;    // n + 1
  int32_t* newid = nullptr;    // n + 1
  int32_t* ccount = nullptr;   // n + 1
  int32_t* coff = nullptr;     // n + 1
  int32_t* cmem = nullptr;     // n
  int64_t* vol = nullptr;      // n + 1
  int64_t* i64tmp = nullptr;   // n + 1 (scans over int64, community sums)
  LevelGraph lg[2];
  int32_t* u_ins_b = nullptr;    // work units of big items (item, first arc)
  int64_t* u_ins_a = nullptr;
  int32_t* u_emit_b = nullptr;   // table-slot units of big items (item, first slot)
  int64_t* u_emit_s = nullptr;
  int64_t units_max = 0;
  int32_t* pool_keys = nullptr;  // global hashtables: keys then values, or
  int32_t* pool_vals = nullptr;  // (as pool_pairs) packed key:value slots
  uint64_t* pool_pairs = nullptr;
  int64_t pool_slots = 0;
  HotRec* hot = nullptr;         // deferred totals of large communities (kHotRegions x kHotCap)
  int64_t* scan_part = nullptr;  // per-block partial sums of the scans
  int64_t scan_part_len = 0;
  int64_t* ctr = nullptr;        // CTR_COUNT counters
  size_t bytes = 0;
};

// Computes the layout; with base == nullptr only the size is computed.
size_t carve_workspace(Workspace& ws, void* base, int32_t n, int64_t cap);

// --------------------------------------------------------------------------
// Device helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ bool test_bit(const uint32_t* bm, int32_t i) {
  return (bm[i >> 5] >> (i & 31)) & 1u;
}

__device__ __forceinline__ void set_bit(uint32_t* bm, int32_t i) {
  atomicOr(&bm[i >> 5], 1u << (i & 31));
}

__device__ __forceinline__ void atomic_add_i64(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
}

__device__ __forceinline__ void set_error(int64_t* ctr, int64_t code) {
  atomicCAS(reinterpret_cast<unsigned long long*>(&ctr[CTR_ERR]), 0ull,
            static_cast<unsigned long long>(code));
}

// Adds v to statistic `st` in this workgroup's replica of the set `sc`.
__device__ __forceinline__ void stat_add(int64_t* sc, int st, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(&sc[(blockIdx.x % kStatReplicas) * kStatStride + st]),
            static_cast<unsigned long long>(v));
}

// A statistic of one set summed over its replicas (on the device).
__device__ __forceinline__ int64_t stat_total(const int64_t* sc, int st) {
  int64_t v = 0;
  for (int r = 0; r < kStatReplicas; ++r) v += sc[r * kStatStride + st];
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}

// Wave-aggregated append: lanes with `pred` get consecutive slots of
// `list` after atomically bumping *count.  Returns the slot or -1.
__device__ __forceinline__ int64_t wave_append(bool pred, int64_t* count) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return -1;
  const int lane = lane_id();
  const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
  int64_t base = 0;
  if (lane == leader)
    base = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(count),
                                          static_cast<unsigned long long>(__popcll(mask))));
  base = __shfl(base, leader);
  const uint64_t below = mask & ((1ull << lane) - 1ull);
  return pred ? base + __popcll(below) : -1;
}

// Workgroup-aggregated reservation of `count` consecutive entries of
// *total (one device atomic per workgroup); every thread of the workgroup
// must call it.  `lds` holds kBlock / kWave + 1 entries.
__device__ __forceinline__ int64_t block_reserve(int64_t count, int64_t* total, int64_t* lds) {
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  constexpr int nw = kBlock / kWave;
  int64_t incl = count;
  for (int s = 1; s < kWave; s <<= 1) {
    const int64_t t = __shfl_up(incl, s);
    if (lane >= s) incl += t;
  }
  if (lane == kWave - 1) lds[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int w = 0; w < nw; ++w) {
      const int64_t x = lds[w];
      lds[w] = run;
      run += x;
    }
    lds[nw] = run ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(total),
                                                   static_cast<unsigned long long>(run)))
                  : 0;
  }
  __syncthreads();
  const int64_t base = lds[nw] + lds[wv] + incl - count;
  __syncthreads();
  return base;
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* lds) {
  v = wave_sum_i64(v);
  if (lane_id() == 0) lds[threadIdx.x / kWave] = v;
  __syncthreads();
  int64_t t = 0;
  for (int w = 0; w < kBlock / kWave; ++w) t += lds[w];
  __syncthreads();
  return t;
}

// Sets frontier bit i when `pred`; a vertex whose bit was clear is appended
// to the frontier list (list may be null: bitmask only).  Every active lane
// of the wavefront calls it together; they share one counter atomic.
// The word is read first and the atomic issued only while the bit is clear:
// the neighbours of movers in a skewed graph are mostly the same few hubs,
// and device atomics on one line serialise, while reads of it do not.  (A
// stale read of a clear bit only costs the atomic; bits are not cleared
// while a kernel marks.)
__device__ __forceinline__ void front_mark(uint32_t* bm, const FrontList& F, int32_t i, bool pred) {
  bool fresh = false;
  if (pred) {
    const uint32_t bit = 1u << (i & 31);
    if (!(bm[i >> 5] & bit)) fresh = !(atomicOr(&bm[i >> 5], bit) & bit);
  }
  if (!F.list) return;
  const int r = static_cast<int>(blockIdx.x % kFlRegions);
  const int64_t pos = wave_append(fresh, &F.cnt[r * kCtrLine]);
  if (fresh && pos < F.capr) F.list[r * F.capr + pos] = i;
}

// front_mark of N vertices per lane: the N bitmask atomics are issued
// together (one memory round trip, not N), and one counter atomic per
// wavefront reserves the list slots of all fresh vertices.
template <int N>
__device__ __forceinline__ void front_mark_n(uint32_t* bm, const FrontList& F, const int32_t (&v)[N],
                                             const bool (&pred)[N]) {
  uint32_t old[N];  // (no read first: a batch's endpoints are mostly fresh)
#pragma unroll
  for (int q = 0; q < N; ++q) old[q] = pred[q] ? atomicOr(&bm[v[q] >> 5], 1u << (v[q] & 31)) : ~0u;
  if (!F.list) return;
  uint64_t mask[N];
  int64_t total = 0;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const bool fresh = pred[q] && !((old[q] >> (v[q] & 31)) & 1u);
    mask[q] = __ballot(fresh);
    total += __popcll(mask[q]);
  }
  if (total == 0) return;
  const int lane = lane_id();
  const int r = static_cast<int>(blockIdx.x % kFlRegions);
  int64_t base = 0;
  if (lane == 0)
    base = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&F.cnt[r * kCtrLine]),
                                          static_cast<unsigned long long>(total)));
  base = __shfl(base, 0);
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    if ((mask[q] >> lane) & 1ull) {
      const int64_t pos = base + __popcll(mask[q] & below);
      if (pos < F.capr) F.list[r * F.capr + pos] = v[q];
    }
    base += __popcll(mask[q]);
  }
}

// Hash of a community id into [0, size) for the open-addressing tables.
__device__ __forceinline__ uint32_t hash_slot(uint32_t key, uint32_t size) {
  const uint32_t h = key * 0x9E3779B1u;
  return static_cast<uint32_t>((static_cast<uint64_t>(h) * size) >> 32);
}

// MurmurHash3's 32-bit finalizer: a second hash, independent of hash_slot's
// ordering, for tables whose keys may arrive sorted by hash_slot (the hub
// segments chosen by hash_slot, the rows an aggregation emits in
// hash_slot order).
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// --------------------------------------------------------------------------
// Launchers (host).  All enqueue on `st`; none synchronises.
// --------------------------------------------------------------------------
int grid_for(int64_t items, int per_block, int max_blocks = 65535 * 4);
// Workgroups of `kernel` (with `lds` bytes of dynamic LDS) that the current
// device holds at once: occupancy per compute unit times the unit count.
int64_t resident_blocks(const void* kernel, int block, size_t lds);

// scan.hip
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, Workspace& ws, hipStream_t st);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, Workspace& ws, hipStream_t st);
int64_t scan_parts_needed(int64_t n);

// hist.hip
void launch_accumulate(const int32_t* C, int32_t n, const int32_t* v32, const int64_t* v64, int32_t* out_count,
                       int64_t* out_val, hipStream_t st);
void launch_fill_members(const int32_t* C, int32_t n, const int32_t* coff, int32_t* cursor, int32_t* cmem,
                         hipStream_t st);

// graph.hip
void launch_build_count(const lv_edges& e, int32_t n, int32_t* deg, int64_t* ctr, hipStream_t st);
void launch_row_capacity(const int32_t* deg, int64_t* capv, int32_t n, float frac, int32_t smin,
                         hipStream_t st);
void launch_build_scatter(const lv_edges& e, const int64_t* row_start, int32_t* row_len, int32_t* col,
                          int32_t* w, int64_t* two_m, hipStream_t st);
void launch_relayout_copy(const lv_graph& src, const int64_t* dst_start, int32_t* dst_len,
                          int32_t* dst_col, int32_t* dst_w, hipStream_t st);
struct Workspace;
void launch_row_sums(const LevelGraph& g, const int32_t* C_mod, int64_t* K, int64_t* Sigma, int32_t* Cinit,
                     int32_t* size, Workspace& ws, hipStream_t st);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
void launch_iota_i32(int32_t* p, int64_t n, hipStream_t st);
void launch_set_all_bits(uint32_t* bm, int32_t n, hipStream_t st);
void launch_copy_bits(const uint32_t* src, uint32_t* dst, int64_t words, hipStream_t st);
void launch_sum_squares(const int64_t* v, int32_t n, int64_t* out, hipStream_t st);

// batch.hip
struct BatchScratch {
  // table of the batch's undirected pairs (canonical key lo << 32 | hi)
  uint64_t* keys;
  int32_t* dw;      // deletion weight of the pair, 0 if none
  int32_t* iw;      // insertion weight of the pair, 0 if none
  int64_t* pos;     // 2 per slot: arc positions of lo -> hi and hi -> lo, -1 if absent
  int64_t size;     // slots (power of two)
  int32_t* slot;    // per update (deletions, then insertions): pair slot, -1 if invalid
  int64_t dirs;     // 2 * updates: arc directions
  // touched rows, each listed under the first direction e that reaches it
  // (per-row arrays below are indexed by that e; dirs entries each)
  uint32_t* tag;    // n bits: row already listed
  int32_t* row_slot;  // n: e of a listed row (read only where tagged)
  int32_t* row_of;  // e -> vertex if e lists a row, else -1
  int32_t* r_len;   // length before the batch
  int32_t* r_cnt;   // update directions on the row
  int32_t* r_pbase; // first partner in `part` (also first tail survivor in tcol / tw)
  int32_t* r_zero;  // arcs reaching weight 0
  int32_t* r_app;   // arcs appended
  int32_t* r_hole;  // head holes refilled so far
  int32_t* d_rank;  // per direction: rank among its row's directions, -1 if invalid
  int32_t* part;    // partners (other endpoints) grouped by row
  int32_t* kind;    // per insertion direction: 1 merge, 0 append
  struct Chunk {     // scan unit: arcs [off, end) of the row of vertex a
    int64_t s;        // row start
    int32_t a, off, end, cnt, pbase, pad;
  };
  Chunk* chunk;
  int32_t* tcol;    // tail survivors, in the row's partner range (dirs entries)
  int32_t* tw;
};
int64_t batch_chunks_bound(int64_t dirs, int64_t cap);
void launch_batch_phase1(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                         int64_t words, int64_t* ctr, hipStream_t st);
void launch_batch_phase2(const lv_graph& g, const lv_edges& del, const lv_edges& ins, const BatchScratch& b,
                         int64_t* ctr, hipStream_t st);

// mark.hip
// updateWeights (Alg. 7); with df_frontier given it also marks DF's initial
// frontier (Alg. 1) in the same pass.  Does nothing if ctr[CTR_ERR] is set;
// flags LV_EINVAL for (and skips) updates outside [0, n) or self-loops.
void launch_update_weights(const lv_edges& del, const lv_edges& ins, int32_t n, const int32_t* C, int64_t* K,
                           int64_t* Sigma, uint32_t* df_frontier, const FrontList& df_list, int64_t* ctr,
                           hipStream_t st);
void launch_batch_weight_sums(const lv_edges& del, const lv_edges& ins, int64_t* ctr, hipStream_t st);
void launch_community_sizes(const int32_t* C, int32_t n, int32_t* size, hipStream_t st);
void launch_ds_deletions(const lv_edges& del, int32_t n, const int32_t* C, uint32_t* dV, uint32_t* dE,
                         uint32_t* dC, int64_t* ctr, hipStream_t st);
void launch_ds_insert_pairs(const lv_edges& ins, int32_t n, const int32_t* C, uint64_t* keys, int64_t* vals,
                            uint32_t size, int64_t* ctr, hipStream_t st);
void launch_ds_best(const uint64_t* keys, const int64_t* vals, uint32_t size, const int64_t* K,
                    const int64_t* Sigma, const int64_t* two_m_dev, const int64_t* ctr, uint64_t* skeys,
                    int64_t* sbest, int32_t* sbestc, uint32_t ssize, int pass, hipStream_t st);
void launch_ds_mark_sources(const uint64_t* skeys, const int32_t* sbestc, uint32_t ssize, uint32_t* dV,
                            uint32_t* dE, uint32_t* dC, hipStream_t st);
void launch_ds_expand(const LevelGraph& g, const lv_edges& del, const lv_edges& ins, const int32_t* C,
                      const uint32_t* dE, const uint32_t* dC, uint32_t* dV, hipStream_t st);

// many.hip -- DF for many graphs in one persistent launch
constexpr int kManyWaveDeg = 256;    // rows up to this length: one wavefront
constexpr int kManyBlockDeg = 2048;  // rows up to this length: one workgroup (longer: not batched)
constexpr int kManyIters = 32;
struct ManyItem {
  int64_t* row_start;
  int32_t* row_len;
  int32_t* col;
  int32_t* w;
  int64_t* two_m;
  int32_t n;
  int32_t max_updates;  // capacity of the scratch
  int32_t* C;
  int64_t* K;
  int64_t* Sigma;
  int32_t* size;
  const int32_t* du;
  const int32_t* dv;
  const int32_t* dw;
  const int32_t* iu;
  const int32_t* iv;
  const int32_t* iw;
  int32_t nd;
  int32_t ni;
  void* scratch;
  // results
  int32_t status;
  int32_t iterations;  // pass 0 (l_i)
  int64_t moves;
  int64_t arcs_scanned;
  int64_t vertices_affected;
  int64_t iter_moves[kManyIters];
  int64_t iter_gain[kManyIters];
};
size_t many_scratch_bytes(int32_t n, int32_t max_updates);
// The descriptor buffer: an int32 item count in a header of kManyHeader
// bytes, then the items.  The kernel reads the count there.
constexpr size_t kManyHeader = 256;
// wave_deg: rows up to this many arcs take one wavefront (at most
// kManyWaveDeg), longer ones the whole workgroup.
void launch_many_df(const int32_t* count, ManyItem* items, int32_t grid, const lv_params& p, int32_t wave_deg,
                    hipStream_t st);

// move.hip
struct MoveArgs {
  LevelGraph g;
  int32_t* C;
  const int64_t* K;
  int64_t* Sigma;
  int32_t* size;
  const uint32_t* cur;
  uint32_t* next;
  FrontList cur_fl;       // the list of cur (read by binning)
  FrontList next_fl;      // the list of next (appended to by the pushes; its counts are zeroed by the
                          // first round's binning)
  const uint32_t* range;  // nullptr: every vertex in range
  uint32_t* ever;         // nullptr: not tracked
  uint32_t* moved;        // movers bitmask (SYNC always; ASYNC when pulling)
  int32_t push;           // 1: movers push the next frontier; 0: it is pulled afterwards
  const int64_t* two_m;   // device copy of 2m (kernels do nothing unless 0 < 2m < 2^31)
  int64_t* rc;            // this sub-round's counter set
  int64_t* rc_next;       // the other set, zeroed by this round's binning for the next round
  int64_t* sc;            // this iteration's statistics set
  int64_t* sc_next;       // the other set; zeroed by the first round's binning when non-null
  int32_t clear_cur;      // 1: binning clears the current frontier as it reads it (last round)
  int32_t sparse;         // 1: the scan may run as one fused launch (a frontier bound that is a small
                          // share of the level's vertices, or a small aggregated level)
  int64_t est;            // upper bound of the vertices processed (grid sizes)
  int32_t mode;
  int32_t guard;
  int32_t wave_max;
};
// One ASYNC sub-round: vertices whose id hash matches (hash_shift = 32: all),
// ids in [id_lo, id_hi), row lengths in [deg_lo, deg_hi].
struct SubRound {
  uint32_t hash_round = 0;
  uint32_t hash_shift = 32;
  int32_t id_lo = 0;
  int32_t id_hi = 0;
  int32_t deg_lo = 0;
  int32_t deg_hi = 0x7fffffff;
};
// Measurement hook (lv_set_timing): the start and stop events of one launch
// of a timed kernel, for hipExtLaunchKernelGGL, which stamps them with the
// kernel's own begin and end times from its dispatch (both null when the
// kernel is not timed); collected after the stream is synchronised.
struct TimerPair {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
TimerPair timer_pair(int kernel);
void timer_collect(int32_t* launches, double* ms);  // adds per kernel, resets

// One sub-round: binning, hub table clear, the fused scan over the bins in
// `bin_mask` (and hub inserts), hub decisions.  Four launches.
uint32_t bins_for_degrees(int32_t lo, int32_t hi, int32_t wave_max);
void launch_round(const MoveArgs& a, Workspace& ws, const lv_tuning& tu, const SubRound& r, uint32_t bin_mask,
                  hipStream_t st);
void launch_apply_moves(const MoveArgs& a, Workspace& ws, bool clear_moved, hipStream_t st);
void launch_pull_expand(const MoveArgs& a, Workspace& ws, hipStream_t st);
// Host helpers shared with the paper-precision path (fp.hip): the error
// message of lv_last_error, the tuning in force, and the sub-rounds of an
// ASYNC iteration.
lv_status lv_fail(lv_status code, const char* msg);
lv_tuning lv_effective_tuning();
std::vector<SubRound> lv_sub_rounds(int32_t mode, int32_t pass, int64_t est_frontier, int32_t n,
                                    const lv_tuning& tu);

// First kernel of a louvain call: zeroes the counters and the frontier
// bitmasks, copies 2m into CTR_TWO_M and flags LV_EEMPTY / LV_EOVERFLOW.
// The frontier lists start empty and valid, or with `dense_a` the list of
// fr_a starts invalid (its bitmask is about to be filled without listing).
void launch_call_begin(Workspace& ws, const int64_t* two_m, bool dense_a, bool keep_err, hipStream_t st);
FrontList front_list(const Workspace& ws, int k);
// Marks a frontier list invalid (its bitmask was filled without listing).
void launch_list_invalid(const FrontList& f, hipStream_t st);

// aggregate.hip
void launch_mark_exists(const int32_t* C, int32_t n, int32_t* flags, hipStream_t st);
void launch_relabel(int32_t* C, int32_t n, const int32_t* newid, hipStream_t st);
void launch_lookup(int32_t* Ctop, int32_t n, const int32_t* Clevel, hipStream_t st);
void launch_community_members(const int32_t* C, const LevelGraph& g, int32_t nc, Workspace& ws,
                              hipStream_t st);
void launch_aggregate(const LevelGraph& g, const int32_t* C, int32_t nc, LevelGraph& out, int64_t* Kout,
                      int64_t* Sout, int32_t* Cout, int32_t* sizeout, Workspace& ws, const lv_tuning& tu,
                      hipStream_t st);
void launch_sigma_from_members(const int32_t* C, const int64_t* K, int32_t n, int64_t* Sigma,
                               hipStream_t st);

}  // namespace lv
