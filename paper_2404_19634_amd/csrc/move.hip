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
//   rows up to the wave threshold: one wavefront, open-addressing table in
//     LDS;
//   rows up to 2048 arcs: one workgroup, open-addressing table in LDS;
//   hub rows: units of 2048 arcs spread over workgroups; each unit
//     pre-aggregates in LDS and flushes into the row's global table
//     (2 x deg slots from the workspace pool); units of 4096 table slots
//     take partial argmaxes, one wavefront per hub picks the move, and
//     insert-sized units expand the frontier of moved hubs.
// Arcs into the vertex's own community d are summed in registers in every
// tier, which keeps the most frequent key out of the hashtable atomics.
//
// A sub-round is binning, then (with hub rows) a hub table clear, the scan,
// then (with hub rows) hub partial argmaxes, decisions and expansion.  For small
// frontiers the scan is one fused kernel whose workgroups take the roles
// of the per-bin kernels (the block ranges of the roles laid end to end in
// one grid): such launches are bound by launch latency, so the count
// matters.  Large frontiers run the same kernel once per bin, in order of
// degree, so that ASYNC moves of one bin are seen by the next.
//
// SYNC mode reads the iteration-start state and records movers; a separate
// kernel applies them.  ASYNC mode applies each move's membership at once.
// Both expand the next frontier from the kernel that holds the mover's arcs
// (or leave it to the pull kernels when the frontier is large).
#include <climits>

#include <hip/hip_ext.h>

#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int64_t kTwoMLimit = int64_t(1) << 31;

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
  FrontList nl;  // the list of next
  uint32_t* moved;
  int32_t* mv_c;
  int32_t push;
  int64_t* rc;  // sub-round counters
  int64_t* sc;  // statistics set
  int64_t* ctr;
  const int64_t* two_m;
  int32_t mode;
  int32_t guard;
  int32_t defer;  // ASYNC: Sigma / size changes through the workgroup aggregate
  HotRec* hot;    // ASYNC with defer: record buffer of large communities' changes (else null)
};

Dev make_dev(const MoveArgs& a, Workspace& ws, const lv_tuning& tu) {
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
  d.nl = a.next_fl;
  d.moved = a.moved;
  d.mv_c = ws.mv_c;
  d.push = a.push;
  d.rc = a.rc;
  d.sc = a.sc;
  d.ctr = ws.ctr;
  d.two_m = a.two_m;
  d.mode = a.mode;
  d.guard = a.guard;
  d.defer = tu.defer_totals;
  d.hot = (a.mode == LV_ASYNC && tu.defer_totals) ? ws.hot : nullptr;
  return d;
}

// 2m of the call; 0 when it is out of range (the first kernel of the call
// has flagged the error and every move kernel then does nothing).
__device__ __forceinline__ int64_t load_two_m(const Dev& D) {
  const int64_t t = *D.two_m;
  return (t > 0 && t < kTwoMLimit) ? t : 0;
}

__device__ __forceinline__ bool better(int64_t g1, int32_t c1, int64_t g0, int32_t c0) {
  return g1 > g0 || (g1 == g0 && c1 < c0);
}

__device__ __forceinline__ int64_t gain_of(int64_t two_m, int64_t kic, int64_t kid, int64_t Ki, int64_t Sc,
                                           int64_t Sd) {
  return two_m * (kic - kid) - Ki * (Sc - Sd + Ki);
}

// Exact pruning of candidates before their total is read.  The gain of a
// move to c != d is 2m K_{i->c} - K_i Σ_c - t with
// t = 2m K_{i->d} - K_i (Σ_d - K_i).  Every member j of c counts the arc
// j -> i in K_j, so Σ_c >= K_{i->c}, and the gain is at most
// K_{i->c} (2m - K_i) - t.  A community that fails open() cannot gain, so
// it is never the target of a move and its Σ_c (a random 8-byte gather)
// is skipped; the move decided is the same.  (Under ASYNC a total that
// lags its membership can undercut K_{i->c}; such a candidate's gain is
// then inflated by the lag, and the bound leaves it out.)
struct GainBar {
  int64_t t, dm;
  __device__ __forceinline__ bool open(int64_t kic) const { return kic * dm > t; }
};
__device__ __forceinline__ GainBar gain_bar(int64_t two_m, int64_t kid, int64_t Ki, int64_t Sd) {
  return GainBar{two_m * kid - Ki * (Sd - Ki), two_m - Ki};
}

// Final decision with the optional swap guard (singleton into a singleton
// of larger id is vetoed).  Reads sizes of the current state.
__device__ __forceinline__ bool decide_move(const Dev& D, int32_t d, int32_t c, int64_t g) {
  if (c == INT_MAX || g <= 0) return false;
  if (D.guard && D.size[d] == 1 && D.size[c] == 1 && c > d) return false;
  return true;
}

// Community-total updates of moves, summed per workgroup in LDS and
// applied with one device atomic per distinct community when the workgroup
// ends (agg_end).  Movers crowd into few large communities, and device
// atomics on one address serialise, so per-move atomics on Sigma and size
// would queue behind each other.  In ASYNC mode a move's new membership is
// visible at once; its effect on Sigma and size becomes visible when the
// workgroup that made it finishes.
constexpr int kAggProbes = 8;
template <int SLOTS>
struct MoveAggT {
  static constexpr int kSlots = SLOTS;
  int32_t key[SLOTS];
  int32_t dsize[SLOTS];
  unsigned long long dsig[SLOTS];
};
using MoveAgg = MoveAggT<512>;       // roles with many movers per workgroup
using MoveAggSmall = MoveAggT<128>;  // the workgroup-per-row role

template <class A>
__device__ __forceinline__ void agg_begin(A* a) {
  for (int s = threadIdx.x; s < A::kSlots; s += blockDim.x) {
    a->key[s] = -1;
    a->dsize[s] = 0;
    a->dsig[s] = 0;
  }
  __syncthreads();
}

template <class A>
__device__ __forceinline__ void agg_add(A* a, int64_t* Sigma, int32_t* size, int32_t c, int64_t dk, int32_t ds) {
  uint32_t h = hash_slot(static_cast<uint32_t>(c), A::kSlots);
  for (int p = 0; p < kAggProbes; ++p) {
    const int32_t old = atomicCAS(&a->key[h], -1, c);
    if (old == -1 || old == c) {
      atomicAdd(&a->dsig[h], static_cast<unsigned long long>(dk));
      if (size) atomicAdd(&a->dsize[h], ds);
      return;
    }
    h = (h + 1) & (A::kSlots - 1);
  }
  atomic_add_i64(&Sigma[c], dk);
  if (size) atomicAdd(&size[c], ds);
}

// every thread of the workgroup calls it once, after its last agg_add
template <class A>
__device__ __forceinline__ void agg_end(A* a, int64_t* Sigma, int32_t* size) {
  __syncthreads();
  for (int s = threadIdx.x; s < A::kSlots; s += blockDim.x) {
    const int32_t c = a->key[s];
    if (c < 0) continue;
    if (a->dsig[s]) atomic_add_i64(&Sigma[c], static_cast<int64_t>(a->dsig[s]));
    if (size && a->dsize[s]) atomicAdd(&size[c], a->dsize[s]);
  }
}

// Records (SYNC: target by vertex plus the movers bitmask) or applies
// (ASYNC: membership now, totals through the workgroup's aggregate, or
// directly when A is null) one move -- one lane per mover.
template <class Agg>
__device__ __forceinline__ void commit_move(const Dev& D, Agg* A, int32_t i, int32_t d, int32_t c, int64_t Ki) {
  if (D.moved) set_bit(D.moved, i);
  if (D.mode == LV_SYNC) {
    D.mv_c[i] = c;
    return;
  }
  D.C[i] = c;
  if (A && D.defer) {
    agg_add(A, D.Sigma, D.size, d, -Ki, -1);
    agg_add(A, D.Sigma, D.size, c, Ki, 1);
  } else {
    atomic_add_i64(&D.Sigma[d], -Ki);
    atomic_add_i64(&D.Sigma[c], Ki);
    if (D.size) {
      atomicSub(&D.size[d], 1);
      atomicAdd(&D.size[c], 1);
    }
  }
}

// End of a move role's workgroup: its aggregate is flushed.  The
// communities whose total is at least 2m / 1024 (at most 1024 of them) are
// the ones that most workgroups of a launch move vertices into or out of:
// device atomics on their lines queue at the memory side, one at a time,
// and reads of the same lines wait behind them.  Their changes are written
// as records instead (one counter atomic per workgroup) and k_hot_apply adds
// them after the launch, one atomic per community; every other community is
// updated here.  Within the launch this only delays what other workgroups
// see of the changes, which they did not see before their own end either.
template <class A>
__device__ __forceinline__ void agg_end_moves(A* a, const Dev& D, int64_t two_m) {
  if (!D.hot) {
    agg_end(a, D.Sigma, D.size);
    return;
  }
  constexpr int kPer = (A::kSlots + kBlock - 1) / kBlock;
  __shared__ int32_t s_n;
  __shared__ int64_t s_base;
  __syncthreads();  // every agg_add of the workgroup is done
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const int64_t hmin = two_m >> 10;
  int32_t pos[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    pos[q] = -1;
    const int sl = threadIdx.x + q * kBlock;
    if (sl >= A::kSlots) continue;
    const int32_t c = a->key[sl];
    if (c < 0) continue;
    const int64_t dk = static_cast<int64_t>(a->dsig[sl]);
    const int32_t ds = a->dsize[sl];
    if (!dk && !ds) continue;
    if (D.Sigma[c] >= hmin) {
      pos[q] = atomicAdd(&s_n, 1);
      continue;
    }
    if (dk) atomic_add_i64(&D.Sigma[c], dk);
    if (D.size && ds) atomicAdd(&D.size[c], ds);
  }
  __syncthreads();
  const int region = static_cast<int>(blockIdx.x % kHotRegions);
  if (threadIdx.x == 0 && s_n)
    s_base = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&D.rc[RC_HOT + region * kCtrLine]),
                                            static_cast<unsigned long long>(s_n)));
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (pos[q] < 0) continue;
    const int sl = threadIdx.x + q * kBlock;
    const int32_t c = a->key[sl];
    const int64_t dk = static_cast<int64_t>(a->dsig[sl]);
    const int32_t ds = a->dsize[sl];
    const int64_t at = s_base + pos[q];
    if (at < kHotCap) {
      D.hot[region * kHotCap + at] = HotRec{c, ds, dk};
    } else {  // the region is full: added here after all
      if (dk) atomic_add_i64(&D.Sigma[c], dk);
      if (D.size && ds) atomicAdd(&D.size[c], ds);
    }
  }
}

// The records of one scan launch: workgroup r sums region r's records per
// community in LDS (four records per thread in flight) and adds each sum
// with one atomic, so a community gets at most kHotRegions atomics.
constexpr int64_t kHotMinFrontier = 1 << 16;  // frontier estimate of a launch that defers
constexpr int kHotSlots = 2048;
__global__ void __launch_bounds__(kBlock) k_hot_apply(const int64_t* __restrict__ rc, const HotRec* __restrict__ hot,
                                                     int64_t* __restrict__ Sigma, int32_t* __restrict__ size) {
  __shared__ int32_t key[kHotSlots];
  __shared__ unsigned long long dk[kHotSlots];
  __shared__ int32_t ds[kHotSlots];
  for (int t = threadIdx.x; t < kHotSlots; t += kBlock) {
    key[t] = -1;
    dk[t] = 0;
    ds[t] = 0;
  }
  __syncthreads();
  const int64_t cnt = min(rc[RC_HOT + blockIdx.x * kCtrLine], kHotCap);
  const HotRec* src = hot + blockIdx.x * kHotCap;
  constexpr int U = 4;
  for (int64_t k0 = 0; k0 < cnt; k0 += U * kBlock) {
    HotRec h[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t k = k0 + q * kBlock + threadIdx.x;
      h[q] = k < cnt ? src[k] : HotRec{-1, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (h[q].c < 0) continue;
      uint32_t t = hash_slot(static_cast<uint32_t>(h[q].c), kHotSlots);
      bool done = false;
      for (int p = 0; p < kHotSlots; ++p) {
        const int32_t old = atomicCAS(&key[t], -1, h[q].c);
        if (old == -1 || old == h[q].c) {
          atomicAdd(&dk[t], static_cast<unsigned long long>(h[q].dk));
          atomicAdd(&ds[t], h[q].ds);
          done = true;
          break;
        }
        t = (t + 1) & (kHotSlots - 1);
      }
      if (!done) {  // (more communities in the region than slots)
        atomic_add_i64(&Sigma[h[q].c], h[q].dk);
        if (size) atomicAdd(&size[h[q].c], h[q].ds);
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHotSlots; t += kBlock) {
    const int32_t c = key[t];
    if (c < 0) continue;
    if (dk[t]) atomic_add_i64(&Sigma[c], static_cast<int64_t>(dk[t]));
    if (size && ds[t]) atomicAdd(&size[c], ds[t]);
  }
}

// Wavefront totals of gains, moves and mover arcs into the statistics.
__device__ __forceinline__ void flush_totals(const Dev& D, int64_t gain, int64_t moved, int64_t arcs) {
  gain = wave_sum_i64(gain);
  moved = wave_sum_i64(moved);
  arcs = wave_sum_i64(arcs);
  if (lane_id() == 0 && moved) {
    stat_add(D.sc, ST_GAIN, gain);
    stat_add(D.sc, ST_EXPAND, arcs);
    stat_add(D.sc, ST_MOVERS, moved);
  }
}

// Vertices of word k that belong to sub-round `round` (ASYNC mode splits
// each iteration into 2^(32 - shift) sub-rounds by a multiplicative hash of
// the vertex id, or by contiguous id ranges, so that a vertex sees most
// neighbours' moves already applied; shift = 32 means a single round).
__device__ __forceinline__ uint32_t round_mask(uint32_t k, uint32_t round, uint32_t shift) {
  uint32_t m = 0;
#pragma unroll 8
  for (uint32_t b = 0; b < 32; ++b) {
    const uint32_t i = k * 32 + b;
    if (((i * 0x9E3779B1u) >> shift) == round) m |= 1u << b;
  }
  return m;
}

// Vertices of word k with ids in [lo, hi) (ASYNC sub-rounds over id ranges).
__device__ __forceinline__ uint32_t range_mask(int64_t k, int32_t lo, int32_t hi) {
  const int64_t first = k * 32;
  const int64_t a = max(static_cast<int64_t>(lo) - first, int64_t(0));
  const int64_t b = min(static_cast<int64_t>(hi) - first, int64_t(32));
  if (a >= b) return 0u;
  const uint32_t upto_b = b >= 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
  const uint32_t upto_a = (1u << a) - 1u;
  return upto_b & ~upto_a;
}

struct Bins {
  int32_t* list[NBINS];
};

__device__ __forceinline__ int bin_of(int32_t deg, int32_t wave_max) {
  if (deg <= 0) return -1;
  if (deg <= 4) return BIN_G4;
  if (deg <= 8) return BIN_G8;
  if (deg <= 16) return BIN_G16;
  if (deg <= 32) return BIN_G32;
  if (deg <= wave_max) return BIN_WAVE;
  if (deg <= kBlockMaxDegree) return BIN_BLOCK;
  return BIN_HUB;
}

struct HubOut {
  int64_t* off;    // global table offset
  int64_t* cbase;  // first clear / decide unit
  int32_t* cnum;   // number of clear / decide units
  int32_t* u_b;    // insert units: (hub item, first arc)
  int64_t* u_a;
  int32_t* c_b;    // clear / decide units: (hub item, first slot)
  int64_t* c_s;
};

__device__ __forceinline__ int64_t hub_units(int32_t deg) { return (deg + kHubUnitArcs - 1) / kHubUnitArcs; }
__device__ __forceinline__ int64_t hub_cunits(int32_t deg) {
  return (2 * static_cast<int64_t>(deg) + kHubClearSlots - 1) / kHubClearSlots;
}

// Hub rows up to kHubPartMaxDeg arcs aggregate by segment: each insert unit
// sums its arcs per community in LDS and writes the (community, weight)
// pairs grouped by segment (a hash range of community ids, one per decide
// unit); each decide unit then sums its segment's pairs from every insert
// unit in LDS.  Plain stores replace the global hashtable's atomics.
// Longer rows use the global table.  A partitioned row's pool reservation
// holds its pairs (unit u at slot u * kHubUnitArcs) and, after 2 * deg
// slots, the segment offsets of every unit (hub_cunits + 1 int32 each).
constexpr int32_t kHubPartMaxDeg = 1 << 20;
constexpr int kHubMaxSegs = (2 * kHubPartMaxDeg + kHubClearSlots - 1) / kHubClearSlots;
constexpr int kHubMaxUnits = (kHubPartMaxDeg + kHubUnitArcs - 1) / kHubUnitArcs;

static_assert(kHubMaxSegs + 1 <= 4 * kBlock && kHubMaxUnits + 1 <= 4 * kBlock,
              "segment offsets and unit counts must fit one workgroup scan");

__device__ __forceinline__ bool hub_part(int32_t deg) { return deg <= kHubPartMaxDeg; }
__device__ __forceinline__ int64_t hub_slots(int32_t deg) {
  const int64_t base = 2 * static_cast<int64_t>(deg);
  return hub_part(deg) ? base + (hub_units(deg) * (hub_cunits(deg) + 1) + 1) / 2 : base;
}

// A hub row's table offset and first clear / decide unit.
__device__ __forceinline__ void hub_head(const HubOut& H, int64_t pos, int32_t deg, int64_t off, int64_t bc) {
  H.off[pos] = off;
  H.cbase[pos] = bc;
  H.cnum[pos] = static_cast<int32_t>(hub_cunits(deg));
}

// Its unit descriptors at the given bases, entries t, t + stride, ... (a
// mega-hub has thousands: the workgroup writes them together).
__device__ __forceinline__ void hub_units_write(const HubOut& H, int64_t pos, int32_t deg, int64_t bu, int64_t bc,
                                               int t, int stride) {
  const int64_t nu = hub_units(deg), nc = hub_cunits(deg);
  for (int64_t u = t; u < nu; u += stride) {
    H.u_b[bu + u] = static_cast<int32_t>(pos);
    H.u_a[bu + u] = u * kHubUnitArcs;
  }
  for (int64_t u = t; u < nc; u += stride) {
    H.c_b[bc + u] = static_cast<int32_t>(pos);
    H.c_s[bc + u] = u * kHubClearSlots;
  }
}

__device__ __forceinline__ void hub_write(const HubOut& H, int64_t pos, int32_t deg, int64_t off, int64_t bu,
                                         int64_t bc) {
  hub_head(H, pos, deg, off, bc);
  hub_units_write(H, pos, deg, bu, bc, 0, 1);
}

// Reserves the hub row's global table (2*deg slots) and its units alone
// (three device atomics).
__device__ __forceinline__ void hub_setup(const HubOut& H, int64_t pos, int32_t deg, int64_t* rc) {
  const int64_t off = static_cast<int64_t>(
      atomicAdd(reinterpret_cast<unsigned long long*>(&rc[RC_POOL]), static_cast<unsigned long long>(hub_slots(deg))));
  const int64_t bu = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&rc[RC_HUB_UNITS]),
                                                    static_cast<unsigned long long>(hub_units(deg))));
  const int64_t bc = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&rc[RC_HUB_CUNITS]),
                                                    static_cast<unsigned long long>(hub_cunits(deg))));
  hub_write(H, pos, deg, off, bu, bc);
}

// --------------------------------------------------------------------------
// First kernel of a call: counters, frontier bitmasks, 2m.
// --------------------------------------------------------------------------
// keep_err: the call follows a batch edit enqueued on the same stream; its
// error (the edit was refused) stays in the error slot, so every later
// kernel leaves the state alone.
__global__ void k_call_begin(int64_t* __restrict__ ctr, uint32_t* __restrict__ fr_a, uint32_t* __restrict__ fr_b,
                             uint32_t* __restrict__ ever, uint32_t* __restrict__ moved, int64_t words,
                             const int64_t* __restrict__ two_m, int32_t dense_a, int32_t keep_err) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (int64_t k = t0; k < words; k += stride) {
    fr_a[k] = 0;
    fr_b[k] = 0;
    ever[k] = 0;
    moved[k] = 0;
  }
  for (int64_t k = t0; k < CTR_COUNT; k += stride) {
    int64_t v = 0;
    if (k == CTR_TWO_M) v = *two_m;
    if (k == CTR_FL0 && dense_a) v = kFlInvalid;
    if (k == CTR_ERR) {
      const int64_t t = *two_m;
      const int64_t prev = keep_err ? ctr[k] : 0;
      v = prev ? prev : (t <= 0 ? LV_EEMPTY : (t >= kTwoMLimit ? LV_EOVERFLOW : 0));
    }
    ctr[k] = v;
  }
}

constexpr int kBinStats = 3 + 2 * NBINS;  // processed, arcs, affected, per-bin vertices and arcs
constexpr int kBinPer = 4;                // items (words or listed vertices) per thread per pass
constexpr int kBinHubs = 2 * kBlock;      // hubs a workgroup reserves together per pass

// --------------------------------------------------------------------------
// Frontier -> degree bins.  Each thread takes kBinPer 32-vertex bitmask
// words (or kBinPer listed vertices) per pass.  Each workgroup counts its
// vertices per bin in LDS, reserves one range per bin with a single global
// atomic, then places them.  Block 0 zeroes the other
// round set (and, on the first round of an iteration, the other statistics
// set); on the last round of an iteration each word of the frontier is
// cleared once read.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_bin_frontier(uint32_t* __restrict__ cur, FrontList cl,
                                                        int64_t* __restrict__ next_cnt,
                                                        const uint32_t* __restrict__ range,
                                                        uint32_t* __restrict__ ever,
                                                        const int32_t* __restrict__ row_len, int32_t n,
                                                        int32_t wave_max, uint32_t round, uint32_t round_shift,
                                                        int32_t id_lo, int32_t id_hi, int32_t deg_lo, int32_t deg_hi,
                                                        int32_t clear_cur, Bins bins, HubOut H,
                                                        int64_t* __restrict__ rc, int64_t* __restrict__ sc,
                                                        int64_t* __restrict__ rc_next,
                                                        int64_t* __restrict__ sc_next) {
  __shared__ int32_t s_cnt[NBINS];
  __shared__ int64_t s_base[NBINS];
  __shared__ unsigned long long s_stat[kBinStats];  // block totals of the statistics
  __shared__ int32_t s_nh;                          // hubs placed in this pass of the block
  __shared__ int64_t s_hpos[kBinHubs];
  __shared__ int32_t s_hdeg[kBinHubs];
  __shared__ int64_t s_hoff[kBinHubs];  // inclusive sums of the queued hubs' table slots,
  __shared__ int32_t s_pu[kBinHubs];    // insert units
  __shared__ int32_t s_pc[kBinHubs];    // and clear / decide units
  __shared__ int64_t s_hbase[3];
  __shared__ int64_t s_rbase[kFlRegions + 1];  // list mode: first entry of each region
  __shared__ int32_t s_list;
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  if (threadIdx.x < kBinStats) s_stat[threadIdx.x] = 0;
  if (threadIdx.x < kWave) {  // the frontier list serves when valid and shorter than the bitmask
    const int lane = threadIdx.x;
    const int64_t c = (cl.list && lane < kFlRegions) ? cl.cnt[lane * kCtrLine] : 0;
    const bool ok = cl.list != nullptr && !__any(c > cl.capr);
    int64_t incl = c;
    for (int d = 1; d < kFlRegions; d <<= 1) {
      const int64_t u = __shfl_up(incl, d);
      if (lane >= d) incl += u;
    }
    if (lane < kFlRegions) s_rbase[lane] = ok ? incl - c : 0;
    if (lane == kFlRegions - 1) {
      s_rbase[kFlRegions] = ok ? incl : 0;
      s_list = ok && incl <= words;
    }
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < kRoundSet; k += blockDim.x) rc_next[k] = 0;
    if (next_cnt)  // the next frontier's list starts empty (first round of an iteration)
      for (int r = threadIdx.x; r < kFlRegions; r += blockDim.x) next_cnt[r * kCtrLine] = 0;
  }
  if (sc_next)
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < kStatSet;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x)
      sc_next[k] = 0;
  __syncthreads();
  const bool lm = s_list != 0;
  const int64_t items = lm ? s_rbase[kFlRegions] : words;
  int64_t arcs = 0, processed = 0, affected = 0;
  int64_t bin_verts[NBINS], bin_arcs[NBINS];
#pragma unroll
  for (int q = 0; q < NBINS; ++q) bin_verts[q] = bin_arcs[q] = 0;
  // each thread takes kBinPer items (words or listed vertices) per pass and
  // issues their loads together: a pass costs a few memory round trips,
  // not a few per item.  A listed vertex's degree is read once.
  const int64_t per_pass = static_cast<int64_t>(kBlock) * kBinPer;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * per_pass;
  const bool filter_deg = deg_lo > 0 || deg_hi < INT_MAX;
  for (int64_t w0 = blockIdx.x * per_pass; w0 < items; w0 += stride) {
    if (threadIdx.x < NBINS) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_nh = 0;
    __syncthreads();
    int64_t kv[kBinPer];   // the word of each item's vertices
    uint32_t bv[kBinPer];  // its vertices in this round
    int32_t dv[kBinPer];   // list mode: the degree of the item's vertex
    if (lm) {
      int32_t iv[kBinPer];
#pragma unroll
      for (int j = 0; j < kBinPer; ++j) {
        const int64_t e = w0 + static_cast<int64_t>(j) * kBlock + threadIdx.x;
        iv[j] = -1;
        if (e < items) {
          int r = 0;
#pragma unroll
          for (int h = kFlRegions / 2; h > 0; h >>= 1)
            if (s_rbase[r + h] <= e) r += h;
          iv[j] = cl.list[r * cl.capr + (e - s_rbase[r])];
        }
      }
#pragma unroll
      for (int j = 0; j < kBinPer; ++j) dv[j] = iv[j] >= 0 ? row_len[iv[j]] : 0;
#pragma unroll
      for (int j = 0; j < kBinPer; ++j) {
        const int32_t i = iv[j];
        const int64_t k = i >= 0 ? (i >> 5) : 0;
        uint32_t bits = i >= 0 ? 1u << (i & 31) : 0u;
        if (i >= 0 && clear_cur) cur[k] = 0;  // (every set bit of the word is listed)
        if (bits && range) bits &= range[k];
        if (bits && round_shift < 32) bits &= round_mask(static_cast<uint32_t>(k), round, round_shift);
        if (bits) bits &= range_mask(k, id_lo, id_hi);
        if (bits && filter_deg && (dv[j] < deg_lo || dv[j] > deg_hi)) bits = 0;
        kv[j] = k;
        bv[j] = bits;
      }
      if (ever) {  // (other listed vertices may share a word)
        uint32_t old[kBinPer];
#pragma unroll
        for (int j = 0; j < kBinPer; ++j) old[j] = bv[j] ? atomicOr(&ever[kv[j]], bv[j]) : ~0u;
#pragma unroll
        for (int j = 0; j < kBinPer; ++j) affected += __popc(bv[j] & ~old[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < kBinPer; ++j) {
        const int64_t e = w0 + static_cast<int64_t>(j) * kBlock + threadIdx.x;
        kv[j] = e;
        bv[j] = e < items ? cur[e] : 0u;
        dv[j] = 0;
      }
#pragma unroll
      for (int j = 0; j < kBinPer; ++j) {
        const int64_t k = kv[j];
        uint32_t bits = bv[j];
        if (clear_cur && bits) cur[k] = 0;
        if (bits && range) bits &= range[k];
        if (bits && round_shift < 32) bits &= round_mask(static_cast<uint32_t>(k), round, round_shift);
        if (bits) bits &= range_mask(k, id_lo, id_hi);
        if (bits && filter_deg) {  // this round's degree class only
          uint32_t keep = 0;
          for (uint32_t r = bits; r; r &= r - 1) {
            const int b = __ffs(r) - 1;
            const int32_t deg = row_len[k * 32 + b];
            if (deg >= deg_lo && deg <= deg_hi) keep |= 1u << b;
          }
          bits = keep;
        }
        if (ever && bits) {
          const uint32_t old = ever[k];
          affected += __popc(bits & ~old);
          ever[k] = old | bits;
        }
        bv[j] = bits;
      }
    }
    // the vertices of item j with their degrees
    auto for_each_vertex = [&](int j, auto&& f) {
      if (lm) {
        if (bv[j]) f(static_cast<int32_t>(kv[j] * 32 + (__ffs(bv[j]) - 1)), dv[j]);
      } else {
        for (uint32_t r = bv[j]; r; r &= r - 1) {
          const int32_t i = static_cast<int32_t>(kv[j] * 32 + (__ffs(r) - 1));
          f(i, row_len[i]);
        }
      }
    };
    int32_t cnt[NBINS];
#pragma unroll
    for (int q = 0; q < NBINS; ++q) cnt[q] = 0;
#pragma unroll
    for (int j = 0; j < kBinPer; ++j)
      for_each_vertex(j, [&](int32_t, int32_t deg) {
        processed += 1;
        arcs += deg;
        const int bin = bin_of(deg, wave_max);
#pragma unroll
        for (int q = 0; q < NBINS; ++q) {
          cnt[q] += (bin == q) ? 1 : 0;
          bin_arcs[q] += (bin == q) ? deg : 0;
        }
      });
#pragma unroll
    for (int q = 0; q < NBINS; ++q) bin_verts[q] += cnt[q];
#pragma unroll
    for (int q = 0; q < NBINS; ++q)
      if (cnt[q]) atomicAdd(&s_cnt[q], cnt[q]);
    __syncthreads();
    if (threadIdx.x < NBINS) {
      const int32_t c = s_cnt[threadIdx.x];
      s_base[threadIdx.x] = c ? static_cast<int64_t>(atomicAdd(
                                    reinterpret_cast<unsigned long long*>(&rc[rc_bin(threadIdx.x)]),
                                    static_cast<unsigned long long>(c)))
                              : 0;
      s_cnt[threadIdx.x] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBinPer; ++j)
      for_each_vertex(j, [&](int32_t i, int32_t deg) {
        const int bin = bin_of(deg, wave_max);
        if (bin < 0) return;
        const int64_t pos = s_base[bin] + atomicAdd(&s_cnt[bin], 1);
        bins.list[bin][pos] = i;
        if (bin == BIN_HUB) {  // queued for one reservation per workgroup
          const int q = atomicAdd(&s_nh, 1);
          if (q < kBinHubs) {
            s_hpos[q] = pos;
            s_hdeg[q] = deg;
          } else {
            hub_setup(H, pos, deg, rc);
          }
        }
      });
    __syncthreads();
    const int nh = min(s_nh, kBinHubs);
    if (nh > 0) {
      // inclusive prefix sums of the queued hubs' table slots, insert units
      // and clear units (Hillis-Steele over at most kBinHubs entries)
      for (int q = threadIdx.x; q < nh; q += kBlock) {
        s_hoff[q] = hub_slots(s_hdeg[q]);
        s_pu[q] = static_cast<int32_t>(hub_units(s_hdeg[q]));
        s_pc[q] = static_cast<int32_t>(hub_cunits(s_hdeg[q]));
      }
      __syncthreads();
      for (int d = 1; d < nh; d <<= 1) {
        int64_t a0[kBinHubs / kBlock];
        int32_t a1[kBinHubs / kBlock], a2[kBinHubs / kBlock];
#pragma unroll
        for (int t = 0; t < kBinHubs / kBlock; ++t) {
          const int q = threadIdx.x + t * kBlock;
          const bool on = q < nh && q >= d;
          a0[t] = on ? s_hoff[q - d] : 0;
          a1[t] = on ? s_pu[q - d] : 0;
          a2[t] = on ? s_pc[q - d] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kBinHubs / kBlock; ++t) {
          const int q = threadIdx.x + t * kBlock;
          if (q < nh) {
            s_hoff[q] += a0[t];
            s_pu[q] += a1[t];
            s_pc[q] += a2[t];
          }
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        s_hbase[0] = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&rc[RC_POOL]),
                                                    static_cast<unsigned long long>(s_hoff[nh - 1])));
        s_hbase[1] = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&rc[RC_HUB_UNITS]),
                                                    static_cast<unsigned long long>(s_pu[nh - 1])));
        s_hbase[2] = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&rc[RC_HUB_CUNITS]),
                                                    static_cast<unsigned long long>(s_pc[nh - 1])));
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nh; q += kBlock) {
        const int32_t deg = s_hdeg[q];
        hub_head(H, s_hpos[q], deg, s_hbase[0] + s_hoff[q] - hub_slots(deg),
                 s_hbase[2] + s_pc[q] - hub_cunits(deg));
      }
      // the unit descriptors, all queued hubs' at once: entry x of the
      // block's range belongs to the first hub whose inclusive sum exceeds x
      auto owner = [&](const int32_t* incl, int32_t x) {
        int lo = 0, hi = nh - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (incl[mid] > x) hi = mid; else lo = mid + 1;
        }
        return lo;
      };
      for (int32_t x = threadIdx.x; x < s_pu[nh - 1]; x += kBlock) {
        const int q = owner(s_pu, x);
        const int64_t u = x - (s_pu[q] - hub_units(s_hdeg[q]));
        H.u_b[s_hbase[1] + x] = static_cast<int32_t>(s_hpos[q]);
        H.u_a[s_hbase[1] + x] = u * kHubUnitArcs;
      }
      for (int32_t x = threadIdx.x; x < s_pc[nh - 1]; x += kBlock) {
        const int q = owner(s_pc, x);
        const int64_t u = x - (s_pc[q] - hub_cunits(s_hdeg[q]));
        H.c_b[s_hbase[2] + x] = static_cast<int32_t>(s_hpos[q]);
        H.c_s[s_hbase[2] + x] = u * kHubClearSlots;
      }
    }
    __syncthreads();
  }
  // statistics: wavefront sums, then workgroup sums, then one atomic each
  // (skipped by workgroups that met no vertex)
  if (__syncthreads_or(processed != 0 || affected != 0) == 0) return;
  {
    int64_t v[kBinStats];
    v[0] = processed;
    v[1] = arcs;
    v[2] = affected;
#pragma unroll
    for (int q = 0; q < NBINS; ++q) {
      v[3 + q] = bin_verts[q];
      v[3 + NBINS + q] = bin_arcs[q];
    }
#pragma unroll
    for (int q = 0; q < kBinStats; ++q) {
      const int64_t t = wave_sum_i64(v[q]);
      if (lane_id() == 0 && t) atomicAdd(&s_stat[q], static_cast<unsigned long long>(t));
    }
  }
  __syncthreads();
  if (threadIdx.x < kBinStats && s_stat[threadIdx.x]) {
    const int q = threadIdx.x;
    const int slot = q == 0 ? ST_PROCESSED : q == 1 ? ST_ARCS : q == 2 ? ST_AFFECTED
                   : q < 3 + NBINS ? ST_BIN_V0 + (q - 3) : ST_BIN_A0 + (q - 3 - NBINS);
    stat_add(sc, slot, static_cast<int64_t>(s_stat[q]));
  }
}

// --------------------------------------------------------------------------
// Roles of the fused scan kernel.  Each takes its own block index range
// (rb in [0, nb)) and the workgroup's LDS.
// --------------------------------------------------------------------------

// Rows of at most G arcs: groups of G lanes, one arc per lane.
template <int G>
__device__ __forceinline__ void role_small(const Dev& D, int64_t two_m, const int32_t* __restrict__ list, int bin,
                                           int64_t rb, int64_t nb, MoveAgg* agg) {
  constexpr int VPW = kWave / G;
  const int64_t count = D.rc[rc_bin(bin)];
  const int lane = lane_id();
  const int sub = lane / G;
  const int k = lane % G;
  const int64_t wave = (rb * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = nb * blockDim.x / kWave;
  int64_t gain_acc = 0, moved = 0, marcs = 0;
  // the next iteration's row and its metadata are loaded during this one
  int32_t n_i = 0, n_deg = 0, n_d = -1;
  int64_t n_start = 0;
  if (wave * VPW + sub < count) {
    n_i = list[wave * VPW + sub];
    n_start = D.row_start[n_i];
    n_deg = D.row_len[n_i];
    n_d = D.C[n_i];
  }
  for (int64_t base = wave * VPW; base < count; base += nwaves * VPW) {
    const int64_t idx = base + sub;
    const bool valid = idx < count;
    int32_t i = 0, deg = 0, d = -1;
    int64_t start = 0;
    if (valid) {
      i = n_i;
      start = n_start;
      deg = n_deg;
      d = n_d;
    }
    const int64_t Ki = valid ? D.K[i] : 0;
    const int64_t Sd = valid && k < deg ? D.Sigma[d] : 0;
    const int64_t nidx = idx + nwaves * VPW;
    if (nidx < count) n_i = list[nidx];
    bool has = valid && k < deg;
    int32_t j = -1, x = 0, c = -1;
    if (has) {
      j = D.col[start + k];
      x = D.wt[start + k];
      if (j == i) has = false;  // self-loop: not a neighbour
    }
    if (has) c = D.C[j];
    if (nidx < count) {
      n_start = D.row_start[n_i];
      n_deg = D.row_len[n_i];
      n_d = D.C[n_i];
    }
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
    const bool cand = has && c != d && gain_bar(two_m, kid, Ki, Sd).open(kc);
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    if (cand) {
      bg = gain_of(two_m, kc, kid, Ki, D.Sigma[c], Sd);
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
    if (lead && mv) {
      commit_move(D, agg, i, d, bc, Ki);
      gain_acc += bg;
      moved += 1;
      marcs += deg;
    }
    front_mark(D.next, D.nl, j, mv && has && D.push);
  }
  flush_totals(D, gain_acc, moved, marcs);
}

// Rows of at most 4 arcs: one lane per row, so that a wavefront keeps 64
// rows' loads in flight; K_{i->c} of the (at most four) neighbour
// communities is summed in registers, with no exchange between lanes.
__device__ __forceinline__ void role_lane4(const Dev& D, int64_t two_m, const int32_t* __restrict__ list, int64_t rb,
                                           int64_t nb, MoveAgg* agg) {
  const int64_t count = D.rc[rc_bin(BIN_G4)];
  const int64_t nt = nb * blockDim.x;
  int64_t gain_acc = 0, moved = 0, marcs = 0;
  for (int64_t idx = rb * blockDim.x + threadIdx.x; idx < count; idx += nt) {
    const int32_t i = list[idx];
    const int64_t start = D.row_start[i];
    const int32_t deg = D.row_len[i];  // 1..4
    const int32_t d = D.C[i];
    const int64_t Ki = D.K[i];
    int32_t j[4], x[4], c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      j[q] = q < deg ? D.col[start + q] : -1;
      x[q] = q < deg ? D.wt[start + q] : 0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (j[q] == i) j[q] = -1;  // self-loop: not a neighbour
      c[q] = j[q] >= 0 ? D.C[j[q]] : -1;
    }
    const int64_t Sd = D.Sigma[d];
    int32_t kid = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) kid += (c[q] == d) ? x[q] : 0;
    const GainBar bar = gain_bar(two_m, kid, Ki, Sd);
    int32_t kc[4];
    bool op[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      kc[q] = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) kc[q] += (c[r] == c[q]) ? x[r] : 0;
      op[q] = c[q] >= 0 && c[q] != d && bar.open(kc[q]);
    }
    int64_t sc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) sc[q] = op[q] ? D.Sigma[c[q]] : 0;
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!op[q]) continue;
      const int64_t g = gain_of(two_m, kc[q], kid, Ki, sc[q], Sd);
      if (better(g, c[q], bg, bc)) {
        bg = g;
        bc = c[q];
      }
    }
    const bool mv = decide_move(D, d, bc, bg);
    if (mv) {
      commit_move(D, agg, i, d, bc, Ki);
      gain_acc += bg;
      moved += 1;
      marcs += deg;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) front_mark(D.next, D.nl, j[q], mv && D.push && j[q] >= 0);
  }
  flush_totals(D, gain_acc, moved, marcs);
}

// Table slots (and arcs) a lane holds at once in the gather phases.
constexpr int kDecideSlots = 4;

// Rows up to the wave threshold: one wavefront, LDS table of TS slots.
template <int TS>
__device__ __forceinline__ void role_wave(const Dev& D, int64_t two_m, const int32_t* __restrict__ list, int64_t rb,
                                          int64_t nb, int32_t* s_keys, int32_t* s_vals, MoveAgg* agg) {
  const int64_t count = D.rc[rc_bin(BIN_WAVE)];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int32_t* keys = s_keys + wid * TS;
  int32_t* vals = s_vals + wid * TS;
  const int64_t wave = (rb * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = nb * blockDim.x / kWave;
  int64_t gain_acc = 0, moved = 0, marcs = 0;
  // the next row's id and metadata are loaded while this row is scanned
  int32_t n_i = 0, n_deg = 0, n_d = 0;
  int64_t n_start = 0;
  if (wave < count) {
    n_i = list[wave];
    n_start = D.row_start[n_i];
    n_deg = D.row_len[n_i];
    n_d = D.C[n_i];
  }
  for (int64_t idx = wave; idx < count; idx += nwaves) {
    const int32_t i = n_i;
    const int64_t start = n_start;
    const int32_t deg = n_deg;
    const int32_t d = n_d;
    const int64_t Ki = D.K[i];
    const int64_t Sd = D.Sigma[d];
    if (idx + nwaves < count) n_i = list[idx + nwaves];
    // table of the smallest power of two >= 2*deg slots (at least 64)
    const uint32_t ts = max(64u, 1u << (32 - __clz(static_cast<uint32_t>(2 * deg - 1))));
    for (uint32_t t = lane; t < ts; t += kWave) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // a lane's arcs (deg <= TS/2): all loads, then all gathers, then the
    // table, so the memory latencies overlap instead of adding up
    constexpr int U = TS / (2 * kWave);
    int32_t kid = 0;
    {
      int32_t js[U], xs[U], cs[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t k = lane + q * kWave;
        js[q] = k < deg ? D.col[start + k] : i;
        xs[q] = k < deg ? D.wt[start + k] : 0;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) cs[q] = js[q] != i ? D.C[js[q]] : d;
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (js[q] == i) continue;
        if (cs[q] == d) {
          kid += xs[q];
          continue;
        }
        uint32_t h = hash_slot(static_cast<uint32_t>(cs[q]), ts);
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, cs[q]);
          if (old == -1 || old == cs[q]) {
            atomicAdd(&vals[h], xs[q]);
            break;
          }
          h = (h + 1) & (ts - 1);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (idx + nwaves < count) {
      n_start = D.row_start[n_i];
      n_deg = D.row_len[n_i];
      n_d = D.C[n_i];
    }
    kid = wave_sum_i32(kid);
    const GainBar bar = gain_bar(two_m, kid, Ki, Sd);
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    // the table in chunks of kDecideSlots slots per lane (the gathers of a
    // chunk overlap; the chunk bounds the registers the phase holds)
    for (uint32_t t0 = 0; t0 < ts; t0 += kDecideSlots * kWave) {
      int32_t cc[kDecideSlots], vv[kDecideSlots];
      int64_t sg[kDecideSlots];
#pragma unroll
      for (int q = 0; q < kDecideSlots; ++q) {
        const uint32_t t = t0 + lane + q * kWave;
        cc[q] = t < ts ? keys[t] : -1;
        vv[q] = t < ts ? vals[t] : 0;
      }
#pragma unroll
      for (int q = 0; q < kDecideSlots; ++q) sg[q] = cc[q] >= 0 && bar.open(vv[q]) ? D.Sigma[cc[q]] : 0;
#pragma unroll
      for (int q = 0; q < kDecideSlots; ++q)
        if (cc[q] >= 0 && bar.open(vv[q])) {
          const int64_t g = gain_of(two_m, vv[q], kid, Ki, sg[q], Sd);
          if (better(g, cc[q], bg, bc)) {
            bg = g;
            bc = cc[q];
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
    if (decide_move(D, d, bc, bg)) {
      if (lane == 0) {
        commit_move(D, agg, i, d, bc, Ki);
        gain_acc += bg;
        moved += 1;
        marcs += deg;
      }
      if (D.push)
        for (int32_t b = lane; b < deg; b += kWave) {
          const int32_t j = D.col[start + b];
          front_mark(D.next, D.nl, j, j != i);
        }
    }
    // the next row's table clear must not overtake this row's reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  flush_totals(D, gain_acc, moved, marcs);
}

constexpr int kBlockTS = 2 * kBlockMaxDegree;

__device__ __forceinline__ void block_argmax(int64_t& bg, int32_t& bc, int64_t* r_g, int32_t* r_c) {
  for (int s = 1; s < kWave; s <<= 1) {
    const int64_t og = __shfl_xor(bg, s);
    const int32_t oc = __shfl_xor(bc, s);
    if (better(og, oc, bg, bc)) {
      bg = og;
      bc = oc;
    }
  }
  const int wid = threadIdx.x / kWave;
  if (lane_id() == 0) {
    r_g[wid] = bg;
    r_c[wid] = bc;
  }
  __syncthreads();
  for (int t = 0; t < kBlock / kWave; ++t)
    if (better(r_g[t], r_c[t], bg, bc)) {
      bg = r_g[t];
      bc = r_c[t];
    }
}

__device__ __forceinline__ int64_t block_total(int64_t v, int64_t* r) {
  v = wave_sum_i64(v);
  if (lane_id() == 0) r[threadIdx.x / kWave] = v;
  __syncthreads();
  int64_t s = 0;
  for (int t = 0; t < kBlock / kWave; ++t) s += r[t];
  return s;
}

// Exclusive prefix sums of a[0, n) in place (n <= kScanItems * kBlock),
// with the total in a[n]; called by the whole workgroup.  Thread t owns
// a[kScanItems t, kScanItems (t + 1)).  wsum: kBlock / kWave ints of LDS.
constexpr int kScanItems = 4;

__device__ __forceinline__ void block_exscan(int32_t* a, int n, int32_t* wsum) {
  const int t = threadIdx.x, lane = lane_id();
  int32_t own[kScanItems];
  int32_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int k = t * kScanItems + q;
    own[q] = k < n ? a[k] : 0;
    sum += own[q];
  }
  int32_t v = sum;
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) wsum[t / kWave] = v;
  __syncthreads();
  for (int w = 0; w < t / kWave; ++w) v += wsum[w];
  int32_t run = v - sum;  // sum of the elements before this thread's
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int k = t * kScanItems + q;
    if (k < n) a[k] = run;
    run += own[q];
    if (k == n - 1) a[n] = run;
  }
  if (n == 0 && t == 0) a[0] = 0;
  __syncthreads();
}

// Small per-workgroup scratch of the block and hub roles (with a small move
// aggregate: a workgroup of the block role commits a few moves at most).
struct Red {
  int64_t g[kBlock / kWave];
  int32_t c[kBlock / kWave];
  int64_t s[kBlock / kWave];
  int32_t w[kBlock / kWave];
  MoveAggSmall agg;
};

// Rows up to kBlockMaxDegree: one workgroup, LDS table of up to 4096 slots.
__device__ __forceinline__ void role_block(const Dev& D, int64_t two_m, const int32_t* __restrict__ list, int64_t rb,
                                           int64_t nb, int32_t* keys, int32_t* vals, Red* red) {
  const int64_t count = D.rc[rc_bin(BIN_BLOCK)];
  int64_t gain_acc = 0, moved = 0, marcs = 0;
  // the next row's id and metadata are loaded while this row is scanned
  // (no other workgroup changes C of a row this workgroup holds)
  int32_t n_i = 0, n_deg = 0, n_d = 0;
  int64_t n_start = 0;
  if (rb < count) {
    n_i = list[rb];
    n_start = D.row_start[n_i];
    n_deg = D.row_len[n_i];
    n_d = D.C[n_i];
  }
  for (int64_t idx = rb; idx < count; idx += nb) {
    const int32_t i = n_i;
    const int64_t start = n_start;
    const int32_t deg = n_deg;
    const int32_t d = n_d;
    const int64_t Ki = D.K[i];
    const int64_t Sd = D.Sigma[d];
    if (idx + nb < count) n_i = list[idx + nb];
    const uint32_t ts = max(256u, 1u << (32 - __clz(static_cast<uint32_t>(2 * deg - 1))));
    for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __syncthreads();
    // a thread's arcs and table slots are loaded, then gathered, in chunks
    constexpr int U = kDecideSlots;
    int64_t kid = 0;
    for (int32_t k0 = 0; k0 < deg; k0 += U * kBlock) {
      int32_t js[U], xs[U], cs[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t k = k0 + threadIdx.x + q * kBlock;
        js[q] = k < deg ? D.col[start + k] : i;
        xs[q] = k < deg ? D.wt[start + k] : 0;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) cs[q] = js[q] != i ? D.C[js[q]] : d;
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (js[q] == i) continue;
        if (cs[q] == d) {
          kid += xs[q];
          continue;
        }
        uint32_t h = hash_slot(static_cast<uint32_t>(cs[q]), ts);
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, cs[q]);
          if (old == -1 || old == cs[q]) {
            atomicAdd(&vals[h], xs[q]);
            break;
          }
          h = (h + 1) & (ts - 1);
        }
      }
    }
    if (idx + nb < count) {
      n_start = D.row_start[n_i];
      n_deg = D.row_len[n_i];
      n_d = D.C[n_i];
    }
    kid = block_total(kid, red->s);
    const GainBar bar = gain_bar(two_m, kid, Ki, Sd);
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    for (uint32_t t0 = 0; t0 < ts; t0 += kDecideSlots * kBlock) {
      int32_t cc[kDecideSlots], vv[kDecideSlots];
      int64_t sg[kDecideSlots];
#pragma unroll
      for (int q = 0; q < kDecideSlots; ++q) {
        const uint32_t t = t0 + threadIdx.x + q * kBlock;
        cc[q] = t < ts ? keys[t] : -1;
        vv[q] = t < ts ? vals[t] : 0;
      }
#pragma unroll
      for (int q = 0; q < kDecideSlots; ++q) sg[q] = cc[q] >= 0 && bar.open(vv[q]) ? D.Sigma[cc[q]] : 0;
#pragma unroll
      for (int q = 0; q < kDecideSlots; ++q)
        if (cc[q] >= 0 && bar.open(vv[q])) {
          const int64_t g = gain_of(two_m, vv[q], kid, Ki, sg[q], Sd);
          if (better(g, cc[q], bg, bc)) {
            bg = g;
            bc = cc[q];
          }
        }
    }
    block_argmax(bg, bc, red->g, red->c);
    if (decide_move(D, d, bc, bg)) {
      if (threadIdx.x == 0) {
        commit_move(D, &red->agg, i, d, bc, Ki);
        gain_acc += bg;
        moved += 1;
        marcs += deg;
      }
      if (D.push)
        for (int32_t k = threadIdx.x; k < deg; k += kBlock) {
          const int32_t j = D.col[start + k];
          front_mark(D.next, D.nl, j, j != i);
        }
    }
    __syncthreads();
  }
  flush_totals(D, gain_acc, moved, marcs);
}

// Hub rows, insert units: LDS pre-aggregation of 2048 arcs, flushed into
// the hub's global table.  A global slot packs key (high half) and value
// (low half) in 64 bits, so one compare-and-swap inserts a new key with
// its weight; a hit adds the weight to the low half (a sum of arc weights
// of one row stays below 2m < 2^31, so it never carries into the key).
constexpr int kHubTS = 4096;     // LDS pre-aggregation slots per unit
constexpr int kHubProbes = 8;
constexpr unsigned long long kEmptyPair = 0xFFFFFFFF00000000ull;  // key -1, value 0

__device__ __forceinline__ unsigned long long pack_pair(int32_t c, int32_t x) {
  return (static_cast<unsigned long long>(static_cast<uint32_t>(c)) << 32) | static_cast<uint32_t>(x);
}

__device__ __forceinline__ void gtable_add(unsigned long long* tab, uint32_t tsz, int32_t c, int32_t x) {
  uint32_t h = hash_slot(static_cast<uint32_t>(c), tsz);
  while (true) {
    const unsigned long long old = atomicCAS(&tab[h], kEmptyPair, pack_pair(c, x));
    if (old == kEmptyPair) return;
    if (static_cast<int32_t>(old >> 32) == c) {
      atomicAdd(&tab[h], static_cast<unsigned long long>(static_cast<uint32_t>(x)));
      return;
    }
    h = (h + 1 == tsz) ? 0 : h + 1;
  }
}

struct HubIn {
  const int32_t* list;
  const int64_t* off;
  const int32_t* u_b;
  const int64_t* u_a;
  unsigned long long* tab;
  int64_t* kid;
  int64_t pool_slots;
};

__device__ __forceinline__ void role_hub_insert(const Dev& D, const HubIn& H, int64_t rb, int64_t nb, int32_t* tk,
                                                int32_t* tv, int32_t* hist, Red* red) {
  const int64_t count = D.rc[RC_HUB_UNITS];
  for (int64_t u = rb; u < count; u += nb) {
    const int32_t h = H.u_b[u];
    const int32_t i = H.list[h];
    const int64_t start = D.row_start[i];
    const int32_t deg = D.row_len[i];
    const int32_t d = D.C[i];
    const uint32_t tsz = 2u * static_cast<uint32_t>(deg);
    const bool part = hub_part(deg);
    const int64_t off = H.off[h];
    if (off + hub_slots(deg) > H.pool_slots) {
      if (threadIdx.x == 0) set_error(D.ctr, LV_EWORKSPACE);
      continue;
    }
    unsigned long long* tab = H.tab + off;
    for (int s = threadIdx.x; s < kHubTS; s += kBlock) {
      tk[s] = -1;
      tv[s] = 0;
    }
    __syncthreads();
    const int64_t a0 = H.u_a[u];
    const int64_t a1 = min(static_cast<int64_t>(deg), a0 + kHubUnitArcs);
    int64_t kid = 0;
    // each thread's arcs: all loads first, then all gathers, then the table
    constexpr int kPer = kHubUnitArcs / kBlock;
    int32_t js[kPer], xs[kPer], cs[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int64_t a = a0 + threadIdx.x + static_cast<int64_t>(q) * kBlock;
      js[q] = a < a1 ? D.col[start + a] : i;
      xs[q] = a < a1 ? D.wt[start + a] : 0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) cs[q] = js[q] != i ? D.C[js[q]] : d;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (js[q] == i) continue;
      const int32_t c = cs[q], x = xs[q];
      if (c == d) {
        kid += x;
        continue;
      }
      // mix32, not hash_slot: an aggregated row lists its arcs in the order
      // of its community table's hash_slot, so a unit's keys share their
      // top hash bits and would pile into a few slots
      uint32_t p = mix32(static_cast<uint32_t>(c)) & (kHubTS - 1);
      bool done = false;
      // a partitioned row's unit has at most kHubUnitArcs keys, half the
      // table: probing always ends
      for (int t = 0; t < (part ? kHubTS : kHubProbes); ++t) {
        const int32_t old = atomicCAS(&tk[p], -1, c);
        if (old == -1 || old == c) {
          atomicAdd(&tv[p], x);
          done = true;
          break;
        }
        p = (p + 1) & (kHubTS - 1);
      }
      if (!done) gtable_add(tab, tsz, c, x);
    }
    kid = block_total(kid, red->s);
    if (threadIdx.x == 0 && kid) atomic_add_i64(&H.kid[h], kid);
    if (part) {
      // the unit's pairs grouped by segment: a histogram, its prefix sums
      // (stored as the unit's segment offsets), then the placement
      const uint32_t ns = static_cast<uint32_t>(hub_cunits(deg));
      const int64_t ui = a0 / kHubUnitArcs;
      unsigned long long* pairs = tab + ui * kHubUnitArcs;
      int32_t* segoff = reinterpret_cast<int32_t*>(tab + 2 * static_cast<int64_t>(deg)) + ui * (ns + 1);
      for (uint32_t q = threadIdx.x; q <= ns; q += kBlock) hist[q] = 0;
      __syncthreads();
      for (int sl = threadIdx.x; sl < kHubTS; sl += kBlock)
        if (tk[sl] >= 0) atomicAdd(&hist[hash_slot(static_cast<uint32_t>(tk[sl]), ns)], 1);
      __syncthreads();
      block_exscan(hist, static_cast<int>(ns), red->w);
      for (uint32_t q = threadIdx.x; q <= ns; q += kBlock) segoff[q] = hist[q];
      __syncthreads();
      for (int sl = threadIdx.x; sl < kHubTS; sl += kBlock)
        if (tk[sl] >= 0) {
          const int32_t pos = atomicAdd(&hist[hash_slot(static_cast<uint32_t>(tk[sl]), ns)], 1);
          pairs[pos] = pack_pair(tk[sl], tv[sl]);
        }
      __syncthreads();
      continue;
    }
    // Flush in rounds: every pending slot of the thread tries its current
    // table slot (the compare-and-swaps of a round are in flight
    // together); hits add their weight, collisions probe on.
    constexpr int F = 8;
    for (int s0 = 0; s0 < kHubTS; s0 += F * kBlock) {
      int32_t fk[F], fv[F];
      uint32_t fp[F];
      uint32_t pend = 0;
#pragma unroll
      for (int q = 0; q < F; ++q) {
        const int sl = s0 + threadIdx.x + q * kBlock;
        fk[q] = tk[sl];
        fv[q] = tv[sl];
        fp[q] = fk[q] >= 0 ? hash_slot(static_cast<uint32_t>(fk[q]), tsz) : 0;
        if (fk[q] >= 0) pend |= 1u << q;
      }
      while (pend) {
        unsigned long long old[F];
#pragma unroll
        for (int q = 0; q < F; ++q)
          old[q] = (pend >> q) & 1u ? atomicCAS(&tab[fp[q]], kEmptyPair, pack_pair(fk[q], fv[q])) : kEmptyPair;
#pragma unroll
        for (int q = 0; q < F; ++q) {
          if (!((pend >> q) & 1u)) continue;
          if (old[q] == kEmptyPair) {
            pend &= ~(1u << q);
          } else if (static_cast<int32_t>(old[q] >> 32) == fk[q]) {
            atomicAdd(&tab[fp[q]], static_cast<unsigned long long>(static_cast<uint32_t>(fv[q])));
            pend &= ~(1u << q);
          } else {
            fp[q] = fp[q] + 1 == tsz ? 0 : fp[q] + 1;
          }
        }
      }
    }
    __syncthreads();
  }
}

// Role block ranges of the fused kernel, laid end to end.
// The ranges run from the hub role down to the 4-lane role: workgroups are
// dispatched in index order, so the longest units start first instead of
// forming the launch's tail.
struct Roles {
  int64_t end[NBINS];  // exclusive end of range r, which holds role NBINS - 1 - r (hub = insert units)
};

// LDS of the roles (bytes): a small role uses the move aggregate only, the
// wavefront role its four tables and the aggregate, the workgroup and hub
// roles a 4096-slot table and the reduction scratch.
template <int TS>
constexpr size_t lds_wave() {
  return sizeof(MoveAgg) + 2 * sizeof(int32_t) * (kBlock / kWave) * TS;
}
constexpr size_t lds_table() {
  return sizeof(Red) + 2 * sizeof(int32_t) * kBlockTS + sizeof(int32_t) * (kHubMaxSegs + 1);
}

// ONLY == NBINS: the fused kernel, whose workgroups find their role from the
// block ranges laid end to end.  ONLY < NBINS: that role alone over the
// whole grid (its own register and LDS budget, so a higher occupancy).
template <int TS, int ONLY>
__global__ void __launch_bounds__(kBlock) k_move_all(Dev D, Bins bins, Roles R, HubIn H) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t two_m = load_two_m(D);
  if (two_m == 0) return;
  constexpr bool kAny = ONLY == NBINS;
  int role = ONLY;
  int64_t rb = blockIdx.x, nb = gridDim.x;
  if constexpr (kAny) {
    const int64_t b = blockIdx.x;
    int r = 0;
    while (r < NBINS - 1 && b >= R.end[r]) ++r;
    const int64_t lo = r == 0 ? 0 : R.end[r - 1];
    rb = b - lo;
    nb = R.end[r] - lo;
    role = NBINS - 1 - r;
  }
  if ((kAny || ONLY <= BIN_G32) && role <= BIN_G32) {
    MoveAgg* agg = reinterpret_cast<MoveAgg*>(smem);
    agg_begin(agg);
    switch (role) {
      case BIN_G4: role_lane4(D, two_m, bins.list[BIN_G4], rb, nb, agg); break;
      case BIN_G8: role_small<8>(D, two_m, bins.list[BIN_G8], BIN_G8, rb, nb, agg); break;
      case BIN_G16: role_small<16>(D, two_m, bins.list[BIN_G16], BIN_G16, rb, nb, agg); break;
      default: role_small<32>(D, two_m, bins.list[BIN_G32], BIN_G32, rb, nb, agg); break;
    }
    agg_end_moves(agg, D, two_m);
  } else if ((kAny || ONLY == BIN_WAVE) && role == BIN_WAVE) {
    MoveAgg* agg = reinterpret_cast<MoveAgg*>(smem);
    int32_t* keys = reinterpret_cast<int32_t*>(smem + sizeof(MoveAgg));
    int32_t* vals = keys + (kBlock / kWave) * TS;
    agg_begin(agg);
    role_wave<TS>(D, two_m, bins.list[BIN_WAVE], rb, nb, keys, vals, agg);
    agg_end_moves(agg, D, two_m);
  } else if ((kAny || ONLY == BIN_BLOCK) && role == BIN_BLOCK) {
    Red* red = reinterpret_cast<Red*>(smem);
    int32_t* keys = reinterpret_cast<int32_t*>(smem + sizeof(Red));
    agg_begin(&red->agg);
    role_block(D, two_m, bins.list[BIN_BLOCK], rb, nb, keys, keys + kBlockTS, red);
    agg_end_moves(&red->agg, D, two_m);
  } else if (kAny || ONLY == BIN_HUB) {
    Red* red = reinterpret_cast<Red*>(smem);
    int32_t* tk = reinterpret_cast<int32_t*>(smem + sizeof(Red));
    role_hub_insert(D, H, rb, nb, tk, tk + kHubTS, tk + 2 * kHubTS, red);
  }
}

// --------------------------------------------------------------------------
// Hub rows: table clear (before the fused kernel), then decisions.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_hub_clear(Dev D, const int32_t* __restrict__ list,
                                                     const int64_t* __restrict__ hub_off,
                                                     const int32_t* __restrict__ c_b, const int64_t* __restrict__ c_s,
                                                     unsigned long long* __restrict__ tab,
                                                     int64_t* __restrict__ hub_kid, int64_t pool_slots) {
  const int64_t count = D.rc[RC_HUB_CUNITS];
  for (int64_t u = blockIdx.x; u < count; u += gridDim.x) {
    const int32_t h = c_b[u];
    const int32_t deg = D.row_len[list[h]];
    const int64_t tsz = 2 * static_cast<int64_t>(deg);
    const int64_t off = hub_off[h];
    if (off + hub_slots(deg) > pool_slots) continue;  // reported by the insert role
    if (c_s[u] == 0 && threadIdx.x == 0) hub_kid[h] = 0;
    if (hub_part(deg)) continue;  // no global table
    const int64_t s1 = min(tsz, c_s[u] + kHubClearSlots);
    for (int64_t s = c_s[u] + threadIdx.x; s < s1; s += kBlock) tab[off + s] = kEmptyPair;
  }
}

// Keys one pass of a decide unit holds in its 4096-slot table; the rest of
// the table stays free for inserts in flight when the limit is reached.
constexpr int kDecideMaxKeys = kHubTS - 2 * kBlock;

// Best (gain, community) over table entries held by this thread.
__device__ __forceinline__ void best_of(const Dev& D, int64_t two_m, int64_t kid, int64_t Ki, int64_t Sd,
                                        const int32_t* cc, const int32_t* vv, int64_t& bg, int32_t& bc) {
  const GainBar bar = gain_bar(two_m, kid, Ki, Sd);
  int64_t sg[kDecideSlots];
#pragma unroll
  for (int q = 0; q < kDecideSlots; ++q) sg[q] = cc[q] >= 0 && bar.open(vv[q]) ? D.Sigma[cc[q]] : 0;
#pragma unroll
  for (int q = 0; q < kDecideSlots; ++q)
    if (cc[q] >= 0 && bar.open(vv[q])) {
      const int64_t g = gain_of(two_m, vv[q], kid, Ki, sg[q], Sd);
      if (better(g, cc[q], bg, bc)) {
        bg = g;
        bc = cc[q];
      }
    }
}

// One workgroup per decide unit publishes the unit's best (gain,
// community).  A unit of a partitioned row sums its segment's pairs from
// every insert unit in an LDS table (in several passes over disjoint key
// subsets if the segment holds more keys than one pass can); a unit of a
// long row reads its 4096 slots of the global table.  (A completion count
// with a device-scope fence would let the last unit decide, but on a
// multi-XCD part that fence writes back the L2 and costs more than a
// launch.)
__global__ void __launch_bounds__(kBlock) k_hub_decide(Dev D, const int32_t* __restrict__ list,
                                                      const int64_t* __restrict__ hub_off,
                                                      const int32_t* __restrict__ c_b,
                                                      const int64_t* __restrict__ c_s,
                                                      const unsigned long long* __restrict__ tab,
                                                      const int64_t* __restrict__ hub_kid,
                                                      int64_t* __restrict__ unit_g, int32_t* __restrict__ unit_c,
                                                      int64_t pool_slots) {
  __shared__ int64_t r_g[kBlock / kWave];
  __shared__ int32_t r_c[kBlock / kWave];
  __shared__ int32_t t_key[kHubTS];
  __shared__ int32_t t_val[kHubTS];
  __shared__ int32_t s_lo[kHubMaxUnits];
  __shared__ int32_t s_pre[kHubMaxUnits + 1];
  __shared__ int32_t s_nkeys;
  __shared__ int32_t s_ovf;
  __shared__ int32_t s_w[kBlock / kWave];
  const int64_t two_m = load_two_m(D);
  if (two_m == 0) return;
  const int64_t count = D.rc[RC_HUB_CUNITS];
  for (int64_t u = blockIdx.x; u < count; u += gridDim.x) {
    const int32_t h = c_b[u];
    const int32_t i = list[h];
    const int32_t d = D.C[i];
    const int32_t deg = D.row_len[i];
    const int64_t tsz = 2 * static_cast<int64_t>(deg);
    const int64_t off = hub_off[h];
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    if (off + hub_slots(deg) <= pool_slots) {
      const int64_t Ki = D.K[i];
      const int64_t kid = hub_kid[h];
      const int64_t Sd = D.Sigma[d];
      if (hub_part(deg)) {
        const uint32_t ns = static_cast<uint32_t>(hub_cunits(deg));
        const int32_t nu = static_cast<int32_t>(hub_units(deg));
        const int64_t seg = c_s[u] / kHubClearSlots;
        const unsigned long long* pairs = tab + off;
        const int32_t* segoff = reinterpret_cast<const int32_t*>(tab + off + tsz);
        for (int32_t q = threadIdx.x; q < nu; q += kBlock) {
          const int32_t lo = segoff[q * (ns + 1) + seg];
          s_lo[q] = lo;
          s_pre[q] = segoff[q * (ns + 1) + seg + 1] - lo;
        }
        __syncthreads();
        block_exscan(s_pre, nu, s_w);
        const int32_t total = s_pre[nu];
        for (uint32_t log2r = 0;; ++log2r) {
          bool redo = false;
          bg = LLONG_MIN;
          bc = INT_MAX;
          for (uint32_t r = 0; r < (1u << log2r) && !redo; ++r) {
            for (int t = threadIdx.x; t < kHubTS; t += kBlock) {
              t_key[t] = -1;
              t_val[t] = 0;
            }
            if (threadIdx.x == 0) {
              s_nkeys = 0;
              s_ovf = 0;
            }
            __syncthreads();
            for (int32_t j = threadIdx.x; j < total; j += kBlock) {
              int32_t lo = 0, hi = nu;  // the insert unit of flat index j: s_pre[lo] <= j < s_pre[hi]
              while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (s_pre[mid] <= j) lo = mid;
                else hi = mid;
              }
              const unsigned long long e = pairs[static_cast<int64_t>(lo) * kHubUnitArcs + s_lo[lo] + (j - s_pre[lo])];
              const int32_t c = static_cast<int32_t>(e >> 32);
              const int32_t x = static_cast<int32_t>(static_cast<uint32_t>(e));
              const uint32_t hk = mix32(static_cast<uint32_t>(c));
              if (log2r && (hk >> (32 - log2r)) != r) continue;
              if (__hip_atomic_load(&s_nkeys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= kDecideMaxKeys) {
                s_ovf = 1;
                continue;
              }
              uint32_t p = hk & (kHubTS - 1);
              while (true) {
                const int32_t old = atomicCAS(&t_key[p], -1, c);
                if (old == -1 || old == c) {
                  if (old == -1) atomicAdd(&s_nkeys, 1);
                  atomicAdd(&t_val[p], x);
                  break;
                }
                p = (p + 1) & (kHubTS - 1);
              }
            }
            __syncthreads();
            if (s_ovf) {
              redo = true;
            } else {
              for (int t0 = 0; t0 < kHubTS; t0 += kDecideSlots * kBlock) {
                int32_t cc[kDecideSlots], vv[kDecideSlots];
#pragma unroll
                for (int q = 0; q < kDecideSlots; ++q) {
                  cc[q] = t_key[t0 + threadIdx.x + q * kBlock];
                  vv[q] = t_val[t0 + threadIdx.x + q * kBlock];
                }
                best_of(D, two_m, kid, Ki, Sd, cc, vv, bg, bc);
              }
            }
            __syncthreads();
          }
          if (!redo) break;
        }
      } else {
        const int64_t s1 = min(tsz, c_s[u] + kHubClearSlots);
        for (int64_t t0 = c_s[u]; t0 < s1; t0 += kDecideSlots * kBlock) {
          int32_t cc[kDecideSlots], vv[kDecideSlots];
#pragma unroll
          for (int q = 0; q < kDecideSlots; ++q) {
            const int64_t t = t0 + threadIdx.x + q * kBlock;
            const unsigned long long e = t < s1 ? tab[off + t] : kEmptyPair;
            cc[q] = static_cast<int32_t>(e >> 32);
            vv[q] = static_cast<int32_t>(static_cast<uint32_t>(e));
          }
          best_of(D, two_m, kid, Ki, Sd, cc, vv, bg, bc);
        }
      }
    }
    block_argmax(bg, bc, r_g, r_c);
    if (threadIdx.x == 0) {
      unit_g[u] = bg;
      unit_c[u] = bc;
    }
    __syncthreads();
  }
}

// One wavefront per hub: best over its units, then the move decision.
__global__ void __launch_bounds__(kBlock) k_hub_final(Dev D, const int32_t* __restrict__ list,
                                                     const int64_t* __restrict__ hub_cbase,
                                                     const int32_t* __restrict__ hub_cnum,
                                                     const int64_t* __restrict__ unit_g,
                                                     const int32_t* __restrict__ unit_c,
                                                     int32_t* __restrict__ hub_moved) {
  if (load_two_m(D) == 0) return;
  const int64_t count = D.rc[rc_bin(BIN_HUB)];
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  int64_t gain_acc = 0, moved = 0, marcs = 0;
  for (int64_t h = wave; h < count; h += nwaves) {
    const int64_t b0 = hub_cbase[h];
    const int32_t nu = hub_cnum[h];
    int64_t bg = LLONG_MIN;
    int32_t bc = INT_MAX;
    for (int32_t t = lane; t < nu; t += kWave)
      if (better(unit_g[b0 + t], unit_c[b0 + t], bg, bc)) {
        bg = unit_g[b0 + t];
        bc = unit_c[b0 + t];
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
      const int32_t i = list[h];
      const int32_t d = D.C[i];
      const bool mv = decide_move(D, d, bc, bg);
      hub_moved[h] = mv ? 1 : 0;
      if (mv) {
        commit_move(D, static_cast<MoveAggSmall*>(nullptr), i, d, bc, D.K[i]);
        gain_acc += bg;
        moved += 1;
        marcs += D.row_len[i];
      }
    }
  }
  flush_totals(D, gain_acc, moved, marcs);
}

// Neighbours of moved hubs join the next frontier, one insert unit of arcs
// per workgroup (a hub row can hold over 10^5 arcs).
__global__ void __launch_bounds__(kBlock) k_hub_expand(Dev D, const int32_t* __restrict__ list,
                                                      const int32_t* __restrict__ u_b, const int64_t* __restrict__ u_a,
                                                      const int32_t* __restrict__ hub_moved) {
  const int64_t count = D.rc[RC_HUB_UNITS];
  for (int64_t u = blockIdx.x; u < count; u += gridDim.x) {
    const int32_t h = u_b[u];
    if (!hub_moved[h]) continue;
    const int32_t i = list[h];
    const int64_t start = D.row_start[i];
    const int64_t a1 = min(static_cast<int64_t>(D.row_len[i]), u_a[u] + kHubUnitArcs);
    for (int64_t a = u_a[u] + threadIdx.x; a < a1; a += kBlock) {
      const int32_t j = D.col[start + a];
      front_mark(D.next, D.nl, j, j != i);
    }
  }
}

// --------------------------------------------------------------------------
// SYNC: apply the recorded moves after every decision was taken; one thread
// per word of the movers bitmask.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_apply_moves(int32_t* __restrict__ C, const int64_t* __restrict__ K,
                                                       int64_t* __restrict__ Sigma, int32_t* __restrict__ size,
                                                       uint32_t* __restrict__ moved,
                                                       const int32_t* __restrict__ target, int32_t n,
                                                       int32_t clear) {
  __shared__ MoveAgg agg;
  agg_begin(&agg);
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < words;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t bits = moved[k];
    if (clear && bits) moved[k] = 0;  // nothing reads the movers after this kernel
    for (uint32_t r = bits; r; r &= r - 1) {
      const int32_t i = static_cast<int32_t>(k * 32 + (__ffs(r) - 1));
      const int32_t c = target[i];
      const int32_t d = C[i];
      const int64_t Ki = K[i];
      C[i] = c;
      agg_add(&agg, Sigma, size, d, -Ki, -1);
      agg_add(&agg, Sigma, size, c, Ki, 1);
    }
  }
  agg_end(&agg, Sigma, size);
}

// --------------------------------------------------------------------------
// Pull expansion: vertex j joins the next frontier iff a neighbour i != j
// moved.  The graph is symmetric, so this is the same set the movers would
// push, without one atomic per arc.  A wavefront owns one 32-vertex word
// (4 groups of 16 lanes, 8 rows each) and stores it whole; rows longer
// than kPullGroupMax are left to a workgroup each, which ORs its bit in.
// --------------------------------------------------------------------------
constexpr int kPullGroup = 16;
constexpr int kPullGroupMax = 2048;

// Pull or push: the expansion reads every row until it meets a mover
// (pull), or ORs in the neighbours of every mover (push).  Once the scan is
// done the iteration's statistics say which costs less: push when the
// movers' arcs are under an eighth of the arcs scanned.
constexpr int64_t kPushRatio = 8;

__device__ __forceinline__ int64_t stat_sum(const int64_t* sc, int st) {
  int64_t v = 0;
  for (int r = 0; r < kStatReplicas; ++r) v += sc[r * kStatStride + st];
  return v;
}

__device__ __forceinline__ bool expand_by_push(const int64_t* sc) {
  return stat_sum(sc, ST_EXPAND) * kPushRatio < stat_sum(sc, ST_ARCS);
}

__global__ void __launch_bounds__(kBlock) k_pull_words(const int64_t* __restrict__ row_start,
                                                      const int32_t* __restrict__ row_len,
                                                      const int32_t* __restrict__ col, int32_t n,
                                                      const uint32_t* __restrict__ moved, uint32_t* __restrict__ next,
                                                      int32_t* __restrict__ longlist, int64_t* __restrict__ ctr,
                                                      const int64_t* __restrict__ sc, int64_t* __restrict__ next_cnt) {
  // either way (pull here, or the push kernels) the next frontier is built
  // without its list
  if (blockIdx.x == 0 && threadIdx.x == 0) *next_cnt = kFlInvalid;
  if (expand_by_push(sc)) return;
  const int lane = lane_id();
  const int grp = lane / kPullGroup;
  const int sub = lane % kPullGroup;
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t w = wave; w < words; w += nwaves) {
    uint32_t word = 0;
    for (int r = 0; r < 8; ++r) {
      const int bit = grp * 8 + r;
      const int64_t j = w * 32 + bit;
      bool hit = false;
      if (j < n) {
        const int32_t len = row_len[j];
        if (len > kPullGroupMax) {
          if (sub == 0) {
            const int64_t pos = static_cast<int64_t>(
                atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_AUX1]), 1ull));
            longlist[pos] = static_cast<int32_t>(j);
          }
        } else {
          const int64_t s = row_start[j];
          for (int32_t k = sub; k < len && !hit; k += kPullGroup) {
            const int32_t i = col[s + k];
            hit = i != j && test_bit(moved, i);
          }
        }
      }
      // any lane of the group found a moved neighbour
      const uint64_t m = __ballot(hit);
      if ((m >> (grp * kPullGroup)) & 0xFFFFull) word |= 1u << bit;
    }
    // groups hold disjoint bits of the word
    word |= __shfl_xor(word, 16);
    word |= __shfl_xor(word, 32);
    if (lane == 0) next[w] = word;
  }
}

__global__ void __launch_bounds__(kBlock) k_pull_long(const int64_t* __restrict__ row_start,
                                                     const int32_t* __restrict__ row_len,
                                                     const int32_t* __restrict__ col,
                                                     const uint32_t* __restrict__ moved, uint32_t* __restrict__ next,
                                                     const int32_t* __restrict__ longlist, const int64_t* __restrict__ ctr,
                                                     const int64_t* __restrict__ sc) {
  __shared__ int s_hit;
  if (expand_by_push(sc)) return;
  const int64_t count = ctr[CTR_AUX1];
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t j = longlist[idx];
    if (threadIdx.x == 0) s_hit = 0;
    __syncthreads();
    const int64_t s = row_start[j];
    const int32_t len = row_len[j];
    for (int32_t k = threadIdx.x; k < len; k += kBlock) {
      if (s_hit) break;
      const int32_t i = col[s + k];
      if (i != j && test_bit(moved, i)) s_hit = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_hit) set_bit(next, j);
    __syncthreads();
  }
}

// Push: one wavefront per word of the movers bitmask flags the neighbours
// of its movers whose rows are short, a lane per arc; longer rows are
// queued for a workgroup each.  Flags are byte stores (idempotent, no
// read-modify-write at the memory side, unlike a bitmask atomicOr per arc);
// a last kernel packs them into the next frontier's words.
constexpr int32_t kPushShortMax = 256;

__global__ void __launch_bounds__(kBlock) k_push_words(const int64_t* __restrict__ row_start,
                                                      const int32_t* __restrict__ row_len,
                                                      const int32_t* __restrict__ col, int32_t n,
                                                      const uint32_t* __restrict__ moved, uint8_t* __restrict__ flags,
                                                      int32_t* __restrict__ longlist, int64_t* __restrict__ ctr,
                                                      const int64_t* __restrict__ sc) {
  if (!expand_by_push(sc)) return;
  const int lane = lane_id();
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t w = wave; w < words; w += nwaves) {
    const uint32_t bits = moved[w];
    if (!bits) continue;
    // each lane of the first 32 loads one mover's row; then the wavefront
    // walks the short rows together
    const int32_t i = static_cast<int32_t>(w * 32 + (lane & 31));
    const bool mine = lane < 32 && ((bits >> lane) & 1u);
    int32_t len = 0;
    int64_t s = 0;
    if (mine) {
      len = row_len[i];
      s = row_start[i];
      if (len > kPushShortMax) {
        const int64_t pos =
            static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_AUX1]), 1ull));
        longlist[pos] = i;
        len = 0;
      }
    }
    for (uint32_t r = bits; r; r &= r - 1) {
      const int b = __ffs(r) - 1;
      const int32_t v = static_cast<int32_t>(w * 32 + b);
      const int32_t vl = __shfl(len, b);
      const int64_t vs = __shfl(s, b);
      for (int32_t k = lane; k < vl; k += kWave) {
        const int32_t j = col[vs + k];
        if (j != v) flags[j] = 1;
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_push_long(const int64_t* __restrict__ row_start,
                                                     const int32_t* __restrict__ row_len,
                                                     const int32_t* __restrict__ col, uint8_t* __restrict__ flags,
                                                     const int32_t* __restrict__ longlist,
                                                     const int64_t* __restrict__ ctr, const int64_t* __restrict__ sc) {
  if (!expand_by_push(sc)) return;
  const int64_t count = ctr[CTR_AUX1];
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t i = longlist[idx];
    const int64_t s = row_start[i];
    const int32_t len = row_len[i];
    for (int32_t k = threadIdx.x; k < len; k += kBlock) {
      const int32_t j = col[s + k];
      if (j != i) flags[j] = 1;
    }
  }
}

// The pushed flags of 32 vertices become one word of the next frontier.
__global__ void __launch_bounds__(kBlock) k_push_pack(const uint8_t* __restrict__ flags, uint32_t* __restrict__ next,
                                                     int64_t words, const int64_t* __restrict__ sc) {
  if (!expand_by_push(sc)) return;
  for (int64_t w = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; w < words;
       w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint4* f = reinterpret_cast<const uint4*>(flags + w * 32);
    const uint4 lo = f[0], hi = f[1];
    const uint32_t part[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint32_t bits = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b) bits |= ((part[q] >> (8 * b)) & 0xFFu ? 1u : 0u) << (4 * q + b);
    next[w] = bits;
  }
}

int table_slots_for(int wave_max) {
  int ts = 64;
  while (ts < 2 * wave_max) ts <<= 1;
  return ts;
}

int grid_by_est(int64_t est, int64_t items_per_block, int max_blocks) {
  const int64_t b = (est + items_per_block - 1) / items_per_block;
  return static_cast<int>(b < 1 ? 1 : (b > max_blocks ? max_blocks : b));
}

template <int TS>
void launch_move_all(const Dev& D, const Bins& b, const Roles& R, const HubIn& H, size_t lds, TimerPair tp,
                     hipStream_t st) {
  hipExtLaunchKernelGGL((k_move_all<TS, NBINS>), dim3(static_cast<unsigned>(R.end[NBINS - 1])), dim3(kBlock),
                        static_cast<uint32_t>(lds), st, tp.start, tp.stop, 0, D, b, R, H);
}

// One role over its own grid, capped at the workgroups the device holds at
// once (a grid-stride loop on a larger grid leaves a tail of late
// workgroups behind the resident ones).
template <int TS, int ONLY>
void launch_role(const Dev& D, const Bins& b, const HubIn& H, size_t lds, int64_t grid, TimerPair tp,
                 hipStream_t st) {
  const auto fn = k_move_all<TS, ONLY>;
  grid = std::min<int64_t>(grid, resident_blocks(reinterpret_cast<const void*>(fn), kBlock, lds));
  Roles R{};
  hipExtLaunchKernelGGL(fn, dim3(static_cast<unsigned>(std::max<int64_t>(grid, 1))), dim3(kBlock),
                        static_cast<uint32_t>(lds), st, tp.start, tp.stop, 0, D, b, R, H);
}

// A grid-stride kernel's grid, capped at the workgroups resident at once.
template <class F>
unsigned cap_grid(F fn, int64_t grid) {
  grid = std::min<int64_t>(grid, resident_blocks(reinterpret_cast<const void*>(fn), kBlock, 0));
  return static_cast<unsigned>(std::max<int64_t>(grid, 1));
}

template <int TS>
void launch_one_role(int role, const Dev& D, const Bins& b, const HubIn& H, int64_t grid, TimerPair tp,
                     hipStream_t st) {
  switch (role) {
    case BIN_G4: launch_role<128, BIN_G4>(D, b, H, sizeof(MoveAgg), grid, tp, st); break;
    case BIN_G8: launch_role<128, BIN_G8>(D, b, H, sizeof(MoveAgg), grid, tp, st); break;
    case BIN_G16: launch_role<128, BIN_G16>(D, b, H, sizeof(MoveAgg), grid, tp, st); break;
    case BIN_G32: launch_role<128, BIN_G32>(D, b, H, sizeof(MoveAgg), grid, tp, st); break;
    case BIN_WAVE: launch_role<TS, BIN_WAVE>(D, b, H, lds_wave<TS>(), grid, tp, st); break;
    case BIN_BLOCK: launch_role<128, BIN_BLOCK>(D, b, H, lds_table(), grid, tp, st); break;
    default: launch_role<128, BIN_HUB>(D, b, H, lds_table(), grid, tp, st); break;
  }
}

}  // namespace

void launch_call_begin(Workspace& ws, const int64_t* two_m, bool dense_a, bool keep_err, hipStream_t st) {
  hipLaunchKernelGGL(k_call_begin, dim3(grid_for(std::max<int64_t>(ws.words, CTR_COUNT), kBlock, 2048)),
                     dim3(kBlock), 0, st, ws.ctr, ws.fr_a, ws.fr_b, ws.ever, ws.moved, ws.words, two_m,
                     dense_a ? 1 : 0, keep_err ? 1 : 0);
}

FrontList front_list(const Workspace& ws, int k) {
  return FrontList{ws.fl[k], ws.ctr + CTR_FL0 + k * kFlSet, ws.fl_capr};
}

__global__ void k_list_invalid(int64_t* cnt) { *cnt = kFlInvalid; }

void launch_list_invalid(const FrontList& f, hipStream_t st) {
  hipLaunchKernelGGL(k_list_invalid, dim3(1), dim3(1), 0, st, f.cnt);
}

// Bins whose degree range meets [lo, hi].
uint32_t bins_for_degrees(int32_t lo, int32_t hi, int32_t wave_max) {
  const int32_t blo[NBINS] = {1, 5, 9, 17, 33, wave_max + 1, kBlockMaxDegree + 1};
  const int32_t bhi[NBINS] = {4, 8, 16, 32, wave_max, kBlockMaxDegree, INT_MAX};
  uint32_t m = 0;
  for (int k = 0; k < NBINS; ++k)
    if (blo[k] <= hi && bhi[k] >= lo) m |= 1u << k;
  return m;
}

void launch_round(const MoveArgs& a, Workspace& ws, const lv_tuning& tu, const SubRound& r, uint32_t bin_mask,
                  hipStream_t st) {
  Dev D = make_dev(a, ws, tu);
  const int64_t words = (static_cast<int64_t>(a.g.n) + 31) / 32;
  // Large communities' changes are deferred only in a fused launch over a
  // frontier large enough for their atomics to queue (a smaller one does not
  // repay the extra launch); the launches per bin of a dense frontier run in
  // degree order so that each sees every change of the bins before it.
  const bool fuse = a.sparse && a.est <= tu.fuse_max_frontier;
  if (!fuse || a.est < kHotMinFrontier) D.hot = nullptr;
  Bins b;
  for (int k = 0; k < NBINS; ++k) b.list[k] = ws.bins[k];
  HubOut HO{ws.hub_off, ws.hub_cbase, ws.hub_cnum, ws.u_ins_b, ws.u_ins_a, ws.u_emit_b, ws.u_emit_s};
  const TimerPair tb = timer_pair(LV_TIME_BINNING);
  // (a listed frontier has at most a.est vertices; a bitmask walk is a
  // grid-stride loop, so a smaller grid only slows it)
  const int64_t bin_items = std::max<int64_t>(1, std::min<int64_t>(words, a.est));
  hipExtLaunchKernelGGL(k_bin_frontier, dim3(grid_for(bin_items, kBlock * kBinPer, 4096)), dim3(kBlock), 0, st, tb.start,
                        tb.stop, 0, const_cast<uint32_t*>(a.cur), a.cur_fl, a.sc_next ? a.next_fl.cnt : nullptr,
                        a.range, a.ever, a.g.row_len, a.g.n, a.wave_max,
                        r.hash_round, r.hash_shift, r.id_lo, r.id_hi, r.deg_lo, r.deg_hi, a.clear_cur, b, HO, a.rc,
                        a.sc, a.rc_next, a.sc_next);

  const int64_t est = a.est > 0 ? a.est : 1;
  const int bs = grid_by_est(est, 64, tu.blocks_small);  // sub-wavefront groups
  const int b4 = grid_by_est(est, 256, tu.blocks_small);  // one row per lane
  const int bw = grid_by_est(est, 4, tu.blocks_wave);    // one row per wavefront
  const int bh = grid_by_est(est, 1, tu.blocks_hub);     // one row / unit per workgroup
  const bool hubs = bin_mask & (1u << BIN_HUB);
  if (hubs) {
    const TimerPair tc = timer_pair(LV_TIME_HUB_CLEAR);
    hipExtLaunchKernelGGL(k_hub_clear, dim3(cap_grid(k_hub_clear, bh)), dim3(kBlock), 0, st, tc.start, tc.stop, 0, D,
                          ws.bins[BIN_HUB], ws.hub_off, ws.u_emit_b, ws.u_emit_s,
                          reinterpret_cast<unsigned long long*>(ws.pool_pairs), ws.hub_kid, ws.pool_slots);
  }

  // The scan: for a small, sparse frontier one launch whose role ranges lie
  // end to end; otherwise a launch per bin in increasing degree order, so
  // that (in ASYNC mode) each bin sees the moves of the bins before it (on
  // dense frontiers that ordering is worth modularity).
  const int per[NBINS] = {b4, bs, bs, bs, bw, bh, bh};
  const int ts = table_slots_for(a.wave_max);
  const size_t lw = ts <= 128 ? lds_wave<128>() : ts <= 256 ? lds_wave<256>() : ts <= 512 ? lds_wave<512>()
                                                                                        : lds_wave<1024>();
  const HubIn H{ws.bins[BIN_HUB], ws.hub_off, ws.u_ins_b, ws.u_ins_a,
                reinterpret_cast<unsigned long long*>(ws.pool_pairs), ws.hub_kid, ws.pool_slots};
  if (fuse) {
    Roles R;
    int64_t end = 0;
    for (int r = 0; r < NBINS; ++r) {
      const int k = NBINS - 1 - r;
      if (bin_mask & (1u << k)) end += per[k];
      R.end[r] = end;
    }
    size_t lds = sizeof(MoveAgg);
    if (bin_mask & (1u << BIN_WAVE)) lds = std::max(lds, lw);
    if (bin_mask & ((1u << BIN_BLOCK) | (1u << BIN_HUB))) lds = std::max(lds, lds_table());
    const TimerPair tp = timer_pair(LV_TIME_SCAN);
    if (ts <= 128)
      launch_move_all<128>(D, b, R, H, lds, tp, st);
    else if (ts <= 256)
      launch_move_all<256>(D, b, R, H, lds, tp, st);
    else if (ts <= 512)
      launch_move_all<512>(D, b, R, H, lds, tp, st);
    else
      launch_move_all<1024>(D, b, R, H, lds, tp, st);
  } else {
    for (int k = 0; k < NBINS; ++k) {
      if (!(bin_mask & (1u << k))) continue;
      const TimerPair tp = timer_pair(LV_TIME_SCAN);
      if (ts <= 128)
        launch_one_role<128>(k, D, b, H, per[k], tp, st);
      else if (ts <= 256)
        launch_one_role<256>(k, D, b, H, per[k], tp, st);
      else if (ts <= 512)
        launch_one_role<512>(k, D, b, H, per[k], tp, st);
      else
        launch_one_role<1024>(k, D, b, H, per[k], tp, st);
    }
  }
  if (D.hot)
    hipLaunchKernelGGL(k_hot_apply, dim3(kHotRegions), dim3(kBlock), 0, st, a.rc, D.hot, a.Sigma, a.size);
  if (hubs) {
    const TimerPair td = timer_pair(LV_TIME_HUB_DECIDE);
    hipExtLaunchKernelGGL(k_hub_decide, dim3(cap_grid(k_hub_decide, bh)), dim3(kBlock), 0, st, td.start, td.stop, 0,
                          D, ws.bins[BIN_HUB], ws.hub_off, ws.u_emit_b, ws.u_emit_s,
                          reinterpret_cast<const unsigned long long*>(ws.pool_pairs), ws.hub_kid, ws.unit_g,
                          ws.unit_c, ws.pool_slots);
    hipLaunchKernelGGL(k_hub_final, dim3(64), dim3(kBlock), 0, st, D, ws.bins[BIN_HUB], ws.hub_cbase, ws.hub_cnum,
                       ws.unit_g, ws.unit_c, ws.hub_moved);
    if (a.push)
      hipLaunchKernelGGL(k_hub_expand, dim3(cap_grid(k_hub_expand, bh)), dim3(kBlock), 0, st, D, ws.bins[BIN_HUB],
                         ws.u_ins_b, ws.u_ins_a, ws.hub_moved);
  }
}

void launch_pull_expand(const MoveArgs& a, Workspace& ws, hipStream_t st) {
  const int64_t words = (static_cast<int64_t>(a.g.n) + 31) / 32;
  (void)hipMemsetAsync(ws.ctr + CTR_AUX1, 0, sizeof(int64_t), st);
  hipLaunchKernelGGL(k_pull_words, dim3(grid_for(words * kWave, kBlock, 8192)), dim3(kBlock), 0, st, a.g.row_start,
                     a.g.row_len, a.g.col, a.g.n, a.moved, a.next, ws.bins[NBINS - 1] + 0, ws.ctr, a.sc,
                     a.next_fl.cnt);
  hipLaunchKernelGGL(k_pull_long, dim3(1024), dim3(kBlock), 0, st, a.g.row_start, a.g.row_len, a.g.col, a.moved,
                     a.next, ws.bins[NBINS - 1] + 0, ws.ctr, a.sc);
  // (only one of the pair above and the three below does any work)
  (void)hipMemsetAsync(ws.push_flags, 0, static_cast<size_t>(words) * 32, st);
  hipLaunchKernelGGL(k_push_words, dim3(grid_for(words * kWave, kBlock, 8192)), dim3(kBlock), 0, st, a.g.row_start,
                     a.g.row_len, a.g.col, a.g.n, a.moved, ws.push_flags, ws.bins[NBINS - 1] + 0, ws.ctr, a.sc);
  hipLaunchKernelGGL(k_push_long, dim3(1024), dim3(kBlock), 0, st, a.g.row_start, a.g.row_len, a.g.col,
                     ws.push_flags, ws.bins[NBINS - 1] + 0, ws.ctr, a.sc);
  hipLaunchKernelGGL(k_push_pack, dim3(grid_for(words, kBlock, 4096)), dim3(kBlock), 0, st, ws.push_flags, a.next,
                     words, a.sc);
}

void launch_apply_moves(const MoveArgs& a, Workspace& ws, bool clear_moved, hipStream_t st) {
  const int64_t words = (static_cast<int64_t>(a.g.n) + 31) / 32;
  hipLaunchKernelGGL(k_apply_moves, dim3(grid_for(words, kBlock, 2048)), dim3(kBlock), 0, st, a.C, a.K, a.Sigma,
                     a.size, a.moved, ws.mv_c, a.g.n, clear_moved ? 1 : 0);
}

}  // namespace lv
