// The paper's precision (Section 5.1.2): float32 edge weights with FP64
// hashtable values, weighted degrees K, community totals Sigma, 2m and
// modularity.  The steps are those of the integer path (batch edit, Alg. 7,
// Alg. 1, Alg. 4-6) with Eq. 2 evaluated as printed in FP64:
//     ΔQ(i: d -> c) = (K_{i->c} - K_{i->d}) / m - K_i (K_i + Σ_c - Σ_d) / (2 m^2)
// in ASYNC mode (a move's membership and totals are visible at once to
// later readers; the iteration runs the integer path's sub-rounds).
//
// Work mapping (wave64): rows up to 256 arcs take one wavefront with an LDS
// table of 512 (community, FP64 weight) slots; rows up to 2048 arcs one
// workgroup with a 4096-slot LDS table; longer rows one workgroup with a
// table of 2 x deg slots in the workspace pool.  The frontier is a bitmask;
// movers push their neighbours.  Aggregation gives each community one
// workgroup, whose table (LDS, or pool slots past 2048 arcs of member
// volume) sums the members' arcs by neighbouring community in FP64; the
// sums are stored as float32 weights of a slack CSR whose row capacities
// are the member volumes.
#include <cfloat>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int kFWaveMax = 256;
constexpr int kFWaveSlots = 2 * kFWaveMax;
constexpr int kFBlockMax = 2048;
constexpr int kFBlockSlots = 2 * kFBlockMax;
constexpr int kFNW = kBlock / kWave;
enum FBin { FB_WAVE = 0, FB_BLOCK, FB_HUB, FB_N };

// Counter block (int64 slots, one 128-byte line each where contended):
// errors, list counts, pool reservations, the batch edit's statistics, and
// kFReps replicas of the per-iteration statistics.
constexpr int kFReps = 32;
enum FCtr {
  F_ERR = 0,
  F_LIST0 = 1 * kCtrLine,   // three lines: items per bin
  F_POOL = 4 * kCtrLine,    // pool slots handed out in this round
  F_AUX = 5 * kCtrLine,     // scratch count (compaction rows)
  F_BSUM = 6 * kCtrLine,    // batch: FP64 Σ w_ins (slot 0), Σ w_del (slot 1) as doubles
  F_STATS = 8 * kCtrLine,   // kFReps replicas of a line: the statistics below
  F_COUNT = F_STATS + kFReps * kCtrLine
};
enum FStat { FS_MOVERS = 0, FS_ARCS, FS_PROCESSED, FS_EXPAND, FS_AFFECTED, FS_DQ /* double */, FS_SUM /* double */,
             FS_SUM2 /* double */ };

__device__ __forceinline__ int64_t* rep(int64_t* ctr) { return ctr + F_STATS + (blockIdx.x % kFReps) * kCtrLine; }
__device__ __forceinline__ void stat_i(int64_t* ctr, int k, int64_t v) {
  if (v) atomicAdd(reinterpret_cast<unsigned long long*>(rep(ctr) + k), static_cast<unsigned long long>(v));
}
__device__ __forceinline__ void stat_d(int64_t* ctr, int k, double v) {
  if (v != 0.0) atomicAdd(reinterpret_cast<double*>(rep(ctr) + k), v);
}
__device__ __forceinline__ void flag(int64_t* ctr, int64_t code) {
  atomicCAS(reinterpret_cast<unsigned long long*>(&ctr[F_ERR]), 0ull, static_cast<unsigned long long>(code));
}
template <class T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}
__device__ __forceinline__ bool better_f(double g1, int32_t c1, double g0, int32_t c0) {
  return g1 > g0 || (g1 == g0 && c1 < c0);
}
__device__ __forceinline__ void wave_arg(double& g, int32_t& c) {
  for (int s = 1; s < kWave; s <<= 1) {
    const double og = __shfl_xor(g, s);
    const int32_t oc = __shfl_xor(c, s);
    if (better_f(og, oc, g, c)) {
      g = og;
      c = oc;
    }
  }
}
__device__ __forceinline__ void block_arg(double& g, int32_t& c, double* sg, int32_t* sc) {
  wave_arg(g, c);
  __syncthreads();
  if (lane_id() == 0) {
    sg[threadIdx.x / kWave] = g;
    sc[threadIdx.x / kWave] = c;
  }
  __syncthreads();
  for (int k = 0; k < kFNW; ++k)
    if (better_f(sg[k], sc[k], g, c)) {
      g = sg[k];
      c = sc[k];
    }
  __syncthreads();
}
__device__ __forceinline__ double block_sum_d(double v, double* s) {
  v = wave_sum_d(v);
  __syncthreads();
  if (lane_id() == 0) s[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < kFNW; ++k) t += s[k];
  __syncthreads();
  return t;
}
__device__ __forceinline__ bool weight_ok(float w) { return isfinite(w) && w > 0.0f; }

struct FG {  // a level graph
  int32_t n;
  const int64_t* row_start;
  const int32_t* row_len;
  const int32_t* col;
  const float* w;
};

// ---------------------------------------------------------------------------
// Call start, row sums, totals
// ---------------------------------------------------------------------------
__global__ void k_f_begin(int64_t* __restrict__ ctr, uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                          uint32_t* __restrict__ ever, int64_t words, const double* __restrict__ two_m) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (int64_t k = t0; k < words; k += stride) {
    a[k] = 0;
    b[k] = 0;
    ever[k] = 0;
  }
  for (int64_t k = t0; k < F_COUNT; k += stride) {
    int64_t v = 0;
    if (k == F_ERR) v = (*two_m > 0.0 && isfinite(*two_m)) ? 0 : LV_EEMPTY;
    ctr[k] = v;
  }
}

// K_i = FP64 row sum (Sigma = K, C = identity, size = 1 when given); the
// total (2m) and, with C, the weight of arcs inside communities go to the
// statistics replicas.  One wavefront per row.
__global__ void __launch_bounds__(kBlock) k_f_rows(FG g, const int32_t* __restrict__ C, double* __restrict__ K,
                                                 double* __restrict__ Sigma, int32_t* __restrict__ Cinit,
                                                 int32_t* __restrict__ size, int64_t* __restrict__ ctr) {
  const int lane = lane_id();
  const int64_t nw = static_cast<int64_t>(gridDim.x) * kFNW;
  double tot = 0.0, intra = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kFNW) + threadIdx.x / kWave; i < g.n; i += nw) {
    const int64_t s = g.row_start[i];
    const int32_t len = g.row_len[i];
    const int32_t ci = C ? C[i] : 0;
    double acc = 0.0, in = 0.0;
    for (int32_t k = lane; k < len; k += kWave) {
      const double x = static_cast<double>(g.w[s + k]);
      acc += x;
      if (C && C[g.col[s + k]] == ci) in += x;
    }
    acc = wave_sum_d(acc);
    in = wave_sum_d(in);
    if (lane == 0) {
      if (K) K[i] = acc;
      if (Sigma) Sigma[i] = acc;
      if (Cinit) Cinit[i] = static_cast<int32_t>(i);
      if (size) size[i] = 1;
      tot += acc;
      intra += in;
    }
  }
  if (lane == 0) {
    stat_d(ctr, FS_SUM, tot);
    stat_d(ctr, FS_SUM2, intra);
  }
}

// tot[C_i] += K_i (community totals), FP64 atomics
__global__ void k_f_totals(const int32_t* __restrict__ C, const double* __restrict__ K, int32_t n,
                           double* __restrict__ tot, int64_t* __restrict__ ctr) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t c = C[i];
    if (c < 0 || c >= n)
      flag(ctr, LV_EINVAL);
    else if (K[i] != 0.0)
      atomicAdd(&tot[c], K[i]);
  }
}

// every membership lies in [0, n)
__global__ void k_f_check_c(const int32_t* __restrict__ C, int32_t n, int64_t* __restrict__ ctr) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (C[i] < 0 || C[i] >= n) flag(ctr, LV_EINVAL);
}

// Σ_c tot_c^2 into the statistics (slot FS_SUM)
__global__ void k_f_sumsq(const double* __restrict__ tot, int32_t n, int64_t* __restrict__ ctr) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s += tot[i] * tot[i];
  s = wave_sum_d(s);
  if (lane_id() == 0) stat_d(ctr, FS_SUM, s);
}

__global__ void k_f_zero_d(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Graph build
// ---------------------------------------------------------------------------
__global__ void k_f_count(const int32_t* __restrict__ u, const int32_t* __restrict__ v, const float* __restrict__ w,
                          int64_t m, int32_t n, int32_t* __restrict__ deg, int64_t* __restrict__ ctr) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < m;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t a = u[k], b = v[k];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b || !weight_ok(w[k])) {
      flag(ctr, LV_EINVAL);
      continue;
    }
    atomicAdd(&deg[a], 1);
    atomicAdd(&deg[b], 1);
  }
}

__global__ void k_f_scatter(const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                            const float* __restrict__ w, int64_t m, const int64_t* __restrict__ row_start,
                            int32_t* __restrict__ row_len, int32_t* __restrict__ col, float* __restrict__ wt) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < m;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t a = u[k], b = v[k];
    const int64_t pa = row_start[a] + atomicAdd(&row_len[a], 1);
    const int64_t pb = row_start[b] + atomicAdd(&row_len[b], 1);
    col[pa] = b;
    wt[pa] = w[k];
    col[pb] = a;
    wt[pb] = w[k];
  }
}

__global__ void k_f_set_two_m(double* __restrict__ two_m, const int64_t* __restrict__ ctr, int add) {
  double s = 0.0;
  for (int r = 0; r < kFReps; ++r) s += reinterpret_cast<const double*>(ctr + F_STATS + r * kCtrLine)[FS_SUM];
  if (add) {  // batch: 2 (Σ w_ins - Σ w_del)
    const double* b = reinterpret_cast<const double*>(ctr + F_BSUM);
    *two_m += 2.0 * (b[0] - b[1]);
  } else {
    *two_m = s;
  }
}

// ---------------------------------------------------------------------------
// Batch edit (Section 3.4), all-or-nothing.  A table of the batch's pairs
// (tagged deletion / insertion) finds repeats; a table of touched rows
// counts the arcs each row gains and loses, for the capacity check.
// ---------------------------------------------------------------------------
struct FBatch {
  const int32_t *du, *dv;
  const float* dw;
  int64_t nd;
  const int32_t *iu, *iv;
  const float* iw;
  int64_t ni;
};
struct FBTab {
  unsigned long long* pkey;  // pair tables: (canonical pair << 1 | is_insertion) + 1, 0 = empty
  int32_t* pzero;            // deletions: 1 when the arc's whole weight goes
  int64_t psize;             // power of two
  int32_t* rkey;             // row table: row + 1, 0 = empty
  int32_t* rapp;             // arcs appended to the row
  int32_t* rzero;            // arcs removed from the row
  int64_t rsize;
  int32_t* dpos;             // per deletion: arc offsets in row u and row v
  int32_t* imode;            // per insertion: 1 merge, 0 append
};

__device__ __forceinline__ unsigned long long pair_tag(int32_t a, int32_t b, int ins) {
  const unsigned long long lo = static_cast<uint32_t>(min(a, b)), hi = static_cast<uint32_t>(max(a, b));
  return (((lo << 32) | hi) << 1 | static_cast<unsigned long long>(ins)) + 1ull;
}
__device__ __forceinline__ uint32_t mixh(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return static_cast<uint32_t>(k);
}
// find-or-insert; returns (slot, inserted now)
__device__ __forceinline__ int64_t pair_slot(const FBTab& t, unsigned long long key, bool* fresh) {
  int64_t h = mixh(key) & (t.psize - 1);
  for (int64_t p = 0; p < t.psize; ++p) {
    const unsigned long long old = atomicCAS(&t.pkey[h], 0ull, key);
    if (old == 0ull || old == key) {
      *fresh = old == 0ull;
      return h;
    }
    h = (h + 1) & (t.psize - 1);
  }
  return -1;
}
__device__ __forceinline__ int64_t pair_find(const FBTab& t, unsigned long long key) {
  int64_t h = mixh(key) & (t.psize - 1);
  for (int64_t p = 0; p < t.psize; ++p) {
    const unsigned long long k = ld_agent(&t.pkey[h]);
    if (k == key) return h;
    if (k == 0ull) return -1;
    h = (h + 1) & (t.psize - 1);
  }
  return -1;
}
__device__ __forceinline__ int64_t row_slot(const FBTab& t, int32_t r) {
  int64_t h = mixh(static_cast<unsigned long long>(r) + 0x9E3779B97F4A7C15ull) & (t.rsize - 1);
  for (int64_t p = 0; p < t.rsize; ++p) {
    const int32_t old = atomicCAS(&t.rkey[h], 0, r + 1);
    if (old == 0 || old == r + 1) return h;
    h = (h + 1) & (t.rsize - 1);
  }
  return -1;
}
__device__ __forceinline__ int32_t find_arc(const int32_t* col, int64_t s, int32_t len, int32_t j) {
  for (int32_t k = 0; k < len; ++k)
    if (col[s + k] == j) return k;
  return -1;
}

// V1: deletions -- ids, weights, repeats, presence and weight; records the
// arc offsets and whether the whole weight goes (the row then loses it).
__global__ void k_f_val_del(FBatch b, lv_graph_f g, FBTab t, int64_t* __restrict__ ctr) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < b.nd;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t u = b.du[k], v = b.dv[k];
    const float x = b.dw[k];
    if (u < 0 || v < 0 || u >= g.n || v >= g.n || u == v || !weight_ok(x)) {
      flag(ctr, LV_EINVAL);
      continue;
    }
    bool fresh = false;
    const int64_t h = pair_slot(t, pair_tag(u, v, 0), &fresh);
    if (h < 0 || !fresh) {
      flag(ctr, h < 0 ? LV_EWORKSPACE : LV_EINVAL);
      continue;
    }
    const int32_t pu = find_arc(g.col, g.row_start[u], g.row_len[u], v);
    const int32_t pv = find_arc(g.col, g.row_start[v], g.row_len[v], u);
    if (pu < 0 || pv < 0 || g.w[g.row_start[u] + pu] < x) {
      flag(ctr, LV_ENOEDGE);
      continue;
    }
    t.dpos[2 * k] = pu;
    t.dpos[2 * k + 1] = pv;
    const bool whole = g.w[g.row_start[u] + pu] - x <= 0.0f;
    t.pzero[h] = whole ? 1 : 0;
    if (whole) {
      const int64_t ru = row_slot(t, u), rv = row_slot(t, v);
      if (ru < 0 || rv < 0) {
        flag(ctr, LV_EWORKSPACE);
        continue;
      }
      atomicAdd(&t.rzero[ru], 1);
      atomicAdd(&t.rzero[rv], 1);
    }
    atomicAdd(reinterpret_cast<double*>(ctr + F_BSUM) + 1, static_cast<double>(x));
  }
}

// V2: insertions -- ids, weights, repeats; merge into a present arc that
// the batch's deletions leave, else append (the rows gain an arc).
__global__ void k_f_val_ins(FBatch b, lv_graph_f g, FBTab t, int64_t* __restrict__ ctr) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < b.ni;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t u = b.iu[k], v = b.iv[k];
    const float x = b.iw[k];
    if (u < 0 || v < 0 || u >= g.n || v >= g.n || u == v || !weight_ok(x)) {
      flag(ctr, LV_EINVAL);
      continue;
    }
    bool fresh = false;
    const int64_t h = pair_slot(t, pair_tag(u, v, 1), &fresh);
    if (h < 0 || !fresh) {
      flag(ctr, h < 0 ? LV_EWORKSPACE : LV_EINVAL);
      continue;
    }
    bool merge = find_arc(g.col, g.row_start[u], g.row_len[u], v) >= 0;
    if (merge) {
      const int64_t hd = pair_find(t, pair_tag(u, v, 0));
      if (hd >= 0 && ld_agent(&t.pzero[hd])) merge = false;  // deleted whole first
    }
    t.imode[k] = merge ? 1 : 0;
    if (!merge) {
      const int64_t ru = row_slot(t, u), rv = row_slot(t, v);
      if (ru < 0 || rv < 0) {
        flag(ctr, LV_EWORKSPACE);
        continue;
      }
      atomicAdd(&t.rapp[ru], 1);
      atomicAdd(&t.rapp[rv], 1);
    }
    atomicAdd(reinterpret_cast<double*>(ctr + F_BSUM), static_cast<double>(x));
  }
}

// V3: every touched row fits its capacity after the batch
__global__ void k_f_val_cap(lv_graph_f g, FBTab t, int64_t* __restrict__ ctr) {
  for (int64_t h = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; h < t.rsize;
       h += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t key = t.rkey[h];
    if (!key) continue;
    const int32_t r = key - 1;
    const int64_t cap = g.row_start[r + 1] - g.row_start[r];
    if (static_cast<int64_t>(g.row_len[r]) - t.rzero[h] + t.rapp[h] > cap) flag(ctr, LV_ENOSLACK);
  }
}

// A1: deletions subtract their weight from both arcs
__global__ void k_f_del(FBatch b, lv_graph_f g, FBTab t, const int64_t* __restrict__ ctr) {
  if (ctr[F_ERR]) return;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < b.nd;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    g.w[g.row_start[b.du[k]] + t.dpos[2 * k]] -= b.dw[k];
    g.w[g.row_start[b.dv[k]] + t.dpos[2 * k + 1]] -= b.dw[k];
  }
}

// A2: rows that lost arcs drop the ones of weight 0 (one lane per row)
__global__ void k_f_compact(lv_graph_f g, FBTab t, const int64_t* __restrict__ ctr) {
  if (ctr[F_ERR]) return;
  for (int64_t h = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; h < t.rsize;
       h += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t key = t.rkey[h];
    if (!key || t.rzero[h] == 0) continue;
    const int32_t r = key - 1;
    const int64_t s = g.row_start[r];
    const int32_t len = g.row_len[r];
    int32_t o = 0;
    for (int32_t q = 0; q < len; ++q) {
      const float x = g.w[s + q];
      if (x > 0.0f) {
        g.col[s + o] = g.col[s + q];
        g.w[s + o] = x;
        ++o;
      }
    }
    g.row_len[r] = o;
  }
}

// A3: insertions merge or append, in both directions
__global__ void k_f_ins(FBatch b, lv_graph_f g, FBTab t, const int64_t* __restrict__ ctr) {
  if (ctr[F_ERR]) return;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < b.ni;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t e[2][2] = {{b.iu[k], b.iv[k]}, {b.iv[k], b.iu[k]}};
    for (int q = 0; q < 2; ++q) {
      const int32_t a = e[q][0], c = e[q][1];
      const int64_t s = g.row_start[a];
      if (t.imode[k]) {
        const int32_t p = find_arc(g.col, s, g.row_len[a], c);
        if (p >= 0) atomicAdd(&g.w[s + p], b.iw[k]);
      } else {
        const int64_t p = s + atomicAdd(&g.row_len[a], 1);
        g.col[p] = c;
        g.w[p] = b.iw[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// updateWeights (Alg. 7) in FP64 and DF marking (Alg. 1)
// ---------------------------------------------------------------------------
__global__ void k_f_update(FBatch b, int32_t n, const int32_t* __restrict__ C, double* __restrict__ K,
                           double* __restrict__ Sigma, uint32_t* __restrict__ fr, int64_t* __restrict__ ctr) {
  if (ctr[F_ERR]) return;
  const int64_t total = b.nd + b.ni;
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < total;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const bool del = k < b.nd;
    const int32_t u = del ? b.du[k] : b.iu[k - b.nd];
    const int32_t v = del ? b.dv[k] : b.iv[k - b.nd];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) {  // not the batch apply_batch_f took
      flag(ctr, LV_EINVAL);
      continue;
    }
    const double x = del ? -static_cast<double>(b.dw[k]) : static_cast<double>(b.iw[k - b.nd]);
    const int32_t cu = C[u], cv = C[v];
    atomicAdd(&K[u], x);
    atomicAdd(&K[v], x);
    atomicAdd(&Sigma[cu], x);
    atomicAdd(&Sigma[cv], x);
    if (fr && (cu == cv) == del) {
      set_bit(fr, u);
      set_bit(fr, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Local moving (Alg. 5), ASYNC
// ---------------------------------------------------------------------------
struct FMove {
  FG g;
  int32_t* C;
  const double* K;
  double* Sigma;
  int32_t* size;
  uint32_t* next;
  int32_t* list[FB_N];
  double m;  // 2m / 2
  int32_t guard;
  int64_t* ctr;
  int64_t pool_slots;
  int32_t* pkeys;
  double* pvals;
};

__device__ __forceinline__ double dq_of(double m, double kic, double kid, double Ki, double Sc, double Sd) {
  return (kic - kid) / m - Ki * (Ki + Sc - Sd) / (2.0 * m * m);
}

// the move of vertex i (one thread): returns whether it moved
__device__ __forceinline__ bool commit(const FMove& M, int32_t i, int32_t d, int32_t c, double dq, double Ki) {
  if (c == INT_MAX || !(dq > 0.0)) return false;
  if (M.guard && M.size[d] == 1 && M.size[c] == 1 && c > d) return false;
  M.C[i] = c;
  atomicAdd(&M.Sigma[d], -Ki);
  atomicAdd(&M.Sigma[c], Ki);
  atomicSub(&M.size[d], 1);
  atomicAdd(&M.size[c], 1);
  return true;
}

// LDS table insert: (c, x) into keys/vals of `size` slots (power of two)
__device__ __forceinline__ void tab_add(int32_t* keys, double* vals, uint32_t size, int32_t c, double x) {
  uint32_t h = hash_slot(static_cast<uint32_t>(c), size);
  while (true) {
    const int32_t old = atomicCAS(&keys[h], -1, c);
    if (old == -1 || old == c) {
      atomicAdd(&vals[h], x);
      return;
    }
    h = (h + 1) & (size - 1);
  }
}

__global__ void __launch_bounds__(kBlock) k_f_scan_wave(FMove M) {
  __shared__ int32_t s_keys[kFNW][kFWaveSlots];
  __shared__ double s_vals[kFNW][kFWaveSlots];
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  int32_t* keys = s_keys[wv];
  double* vals = s_vals[wv];
  const int64_t count = M.ctr[F_LIST0 + FB_WAVE * kCtrLine];
  const int64_t nw = static_cast<int64_t>(gridDim.x) * kFNW;
  int64_t movers = 0, expand = 0;
  double dq_sum = 0.0;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(kFNW) + wv; idx < count; idx += nw) {
    const int32_t i = M.list[FB_WAVE][idx];
    const int64_t s = M.g.row_start[i];
    const int32_t deg = M.g.row_len[i];
    const int32_t d = M.C[i];
    const double Ki = M.K[i];
    const uint32_t ts = max(64u, 1u << (32 - __clz(static_cast<uint32_t>(2 * max(deg, 1) - 1))));
    for (uint32_t t = lane; t < ts; t += kWave) {
      keys[t] = -1;
      vals[t] = 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double kid = 0.0;
    for (int32_t k = lane; k < deg; k += kWave) {
      const int32_t j = M.g.col[s + k];
      if (j == i) continue;
      const double x = static_cast<double>(M.g.w[s + k]);
      const int32_t c = M.C[j];
      if (c == d)
        kid += x;
      else
        tab_add(keys, vals, ts, c, x);
    }
    kid = wave_sum_d(kid);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double Sd = M.Sigma[d];
    double bg = -DBL_MAX;
    int32_t bc = INT_MAX;
    for (uint32_t t = lane; t < ts; t += kWave) {
      const int32_t c = keys[t];
      if (c < 0) continue;
      const double g = dq_of(M.m, vals[t], kid, Ki, M.Sigma[c], Sd);
      if (better_f(g, c, bg, bc)) {
        bg = g;
        bc = c;
      }
    }
    wave_arg(bg, bc);
    bool mv = false;
    if (lane == 0) mv = commit(M, i, d, bc, bg, Ki);
    mv = __shfl(mv ? 1 : 0, 0) != 0;
    if (mv) {
      if (lane == 0) {
        movers += 1;
        expand += deg;
        dq_sum += bg;
      }
      for (int32_t k = lane; k < deg; k += kWave) {
        const int32_t j = M.g.col[s + k];
        if (j != i) set_bit(M.next, j);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (lane == 0) {
    stat_i(M.ctr, FS_MOVERS, movers);
    stat_i(M.ctr, FS_EXPAND, expand);
    stat_d(M.ctr, FS_DQ, dq_sum);
  }
}

// rows past the wavefront bin: one workgroup each; the table lies in LDS
// (up to 2048 arcs) or in pool slots (2 x deg, reserved per row)
template <bool HUB>
__global__ void __launch_bounds__(kBlock) k_f_scan_group(FMove M) {
  __shared__ int32_t s_keys[HUB ? 1 : kFBlockSlots];
  __shared__ double s_vals[HUB ? 1 : kFBlockSlots];
  __shared__ double s_g[kFNW];
  __shared__ int32_t s_c[kFNW];
  __shared__ int64_t s_off;
  __shared__ int32_t s_mv;
  const int b = HUB ? FB_HUB : FB_BLOCK;
  const int64_t count = M.ctr[F_LIST0 + b * kCtrLine];
  int64_t movers = 0, expand = 0;
  double dq_sum = 0.0;
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t i = M.list[b][idx];
    const int64_t s = M.g.row_start[i];
    const int32_t deg = M.g.row_len[i];
    const int32_t d = M.C[i];
    const double Ki = M.K[i];
    int32_t* keys;
    double* vals;
    uint32_t ts;
    if (HUB) {
      ts = 1u << (32 - __clz(static_cast<uint32_t>(2 * deg - 1)));
      if (threadIdx.x == 0) {
        const int64_t off = static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long*>(&M.ctr[F_POOL]),
                                                           static_cast<unsigned long long>(ts)));
        s_off = off + ts <= M.pool_slots ? off : -1;
        if (s_off < 0) flag(M.ctr, LV_EWORKSPACE);
      }
      __syncthreads();
      if (s_off < 0) break;  // (uniform) the error is flagged
      keys = M.pkeys + s_off;
      vals = M.pvals + s_off;
    } else {
      ts = kFBlockSlots;
      keys = s_keys;
      vals = s_vals;
    }
    for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
      keys[t] = -1;
      vals[t] = 0.0;
    }
    __syncthreads();
    double kid = 0.0;
    for (int32_t k = threadIdx.x; k < deg; k += kBlock) {
      const int32_t j = M.g.col[s + k];
      if (j == i) continue;
      const double x = static_cast<double>(M.g.w[s + k]);
      const int32_t c = M.C[j];
      if (c == d)
        kid += x;
      else
        tab_add(keys, vals, ts, c, x);
    }
    kid = block_sum_d(kid, s_g);
    const double Sd = M.Sigma[d];
    double bg = -DBL_MAX;
    int32_t bc = INT_MAX;
    for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
      const int32_t c = HUB ? ld_agent(&keys[t]) : keys[t];
      if (c < 0) continue;
      const double x = HUB ? ld_agent(&vals[t]) : vals[t];
      const double g = dq_of(M.m, x, kid, Ki, M.Sigma[c], Sd);
      if (better_f(g, c, bg, bc)) {
        bg = g;
        bc = c;
      }
    }
    block_arg(bg, bc, s_g, s_c);
    if (threadIdx.x == 0) s_mv = commit(M, i, d, bc, bg, Ki) ? 1 : 0;
    __syncthreads();
    if (s_mv) {
      if (threadIdx.x == 0) {
        movers += 1;
        expand += deg;
        dq_sum += bg;
      }
      for (int32_t k = threadIdx.x; k < deg; k += kBlock) {
        const int32_t j = M.g.col[s + k];
        if (j != i) set_bit(M.next, j);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stat_i(M.ctr, FS_MOVERS, movers);
    stat_i(M.ctr, FS_EXPAND, expand);
    stat_d(M.ctr, FS_DQ, dq_sum);
  }
}

// Frontier -> three bins (one thread per bitmask word), with the sub-round
// filters of the integer path (hash round, degree class); the last round
// clears the words it reads.  Workgroup counts per bin, one reservation.
__global__ void __launch_bounds__(kBlock) k_f_bin(uint32_t* __restrict__ cur, uint32_t* __restrict__ ever,
                                                const int32_t* __restrict__ row_len, int32_t n, uint32_t round,
                                                uint32_t shift, int32_t id_lo, int32_t id_hi, int32_t deg_lo,
                                                int32_t deg_hi, int32_t clear,
                                                int32_t* l0, int32_t* l1, int32_t* l2, int64_t* __restrict__ ctr) {
  __shared__ int32_t s_cnt[FB_N];
  __shared__ int64_t s_base[FB_N];
  int32_t* lists[FB_N] = {l0, l1, l2};
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  int64_t arcs = 0, processed = 0, affected = 0;
  for (int64_t w0 = blockIdx.x * static_cast<int64_t>(blockDim.x); w0 < words;
       w0 += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (threadIdx.x < FB_N) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t k = w0 + threadIdx.x;
    uint32_t bits = 0;
    if (k < words) {
      bits = cur[k];
      if (clear && bits) cur[k] = 0;
      if (shift < 32 && bits) {
        uint32_t keep = 0;
        for (uint32_t r = bits; r; r &= r - 1) {
          const uint32_t i = static_cast<uint32_t>(k * 32 + (__ffs(r) - 1));
          if (((i * 0x9E3779B1u) >> shift) == round) keep |= 1u << (__ffs(r) - 1);
        }
        bits = keep;
      }
      if (bits && (id_lo > k * 32 || id_hi < (k + 1) * 32)) {
        uint32_t keep = 0;
        for (uint32_t r = bits; r; r &= r - 1) {
          const int64_t i = k * 32 + (__ffs(r) - 1);
          if (i >= id_lo && i < id_hi) keep |= 1u << (__ffs(r) - 1);
        }
        bits = keep;
      }
      if (bits && (deg_lo > 0 || deg_hi < INT_MAX)) {
        uint32_t keep = 0;
        for (uint32_t r = bits; r; r &= r - 1) {
          const int32_t dg = row_len[k * 32 + (__ffs(r) - 1)];
          if (dg >= deg_lo && dg <= deg_hi) keep |= 1u << (__ffs(r) - 1);
        }
        bits = keep;
      }
      if (ever && bits) {
        const uint32_t old = ever[k];
        affected += __popc(bits & ~old);
        ever[k] = old | bits;
      }
    }
    int32_t cnt[FB_N] = {0, 0, 0};
    for (uint32_t r = bits; r; r &= r - 1) {
      const int32_t dg = row_len[k * 32 + (__ffs(r) - 1)];
      processed += 1;
      arcs += dg;
      cnt[dg <= kFWaveMax ? FB_WAVE : dg <= kFBlockMax ? FB_BLOCK : FB_HUB] += 1;
    }
    for (int q = 0; q < FB_N; ++q)
      if (cnt[q]) atomicAdd(&s_cnt[q], cnt[q]);
    __syncthreads();
    if (threadIdx.x < FB_N) {
      const int32_t c = s_cnt[threadIdx.x];
      s_base[threadIdx.x] = c ? static_cast<int64_t>(atomicAdd(
                                    reinterpret_cast<unsigned long long*>(&ctr[F_LIST0 + threadIdx.x * kCtrLine]),
                                    static_cast<unsigned long long>(c)))
                              : 0;
      s_cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    for (uint32_t r = bits; r; r &= r - 1) {
      const int32_t i = static_cast<int32_t>(k * 32 + (__ffs(r) - 1));
      const int32_t dg = row_len[i];
      const int q = dg <= kFWaveMax ? FB_WAVE : dg <= kFBlockMax ? FB_BLOCK : FB_HUB;
      lists[q][s_base[q] + atomicAdd(&s_cnt[q], 1)] = i;
    }
    __syncthreads();
  }
  arcs = wave_sum_i64(arcs);
  processed = wave_sum_i64(processed);
  affected = wave_sum_i64(affected);
  if (lane_id() == 0) {
    stat_i(ctr, FS_ARCS, arcs);
    stat_i(ctr, FS_PROCESSED, processed);
    stat_i(ctr, FS_AFFECTED, affected);
  }
}

// bits [0, n) set, the rest of the `words` words cleared
__global__ void k_f_set_all(uint32_t* __restrict__ bm, int32_t n, int64_t words) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < words;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    bm[k] = (k + 1) * 32 <= n ? 0xFFFFFFFFu : k * 32 >= n ? 0u : ((1u << (n - k * 32)) - 1u);
}

// ---------------------------------------------------------------------------
// Aggregation (Alg. 6)
// ---------------------------------------------------------------------------
// One workgroup per community c: its members' arcs summed by neighbouring
// community (self-loops included) in FP64, written as the float32 row of
// super-vertex c at vstart[c] (capacity: the members' volume).
__global__ void __launch_bounds__(kBlock) k_f_aggregate(FG g, const int32_t* __restrict__ C,
                                                      const int32_t* __restrict__ coff,
                                                      const int32_t* __restrict__ cmem,
                                                      const int64_t* __restrict__ vstart, int32_t nc,
                                                      int32_t* __restrict__ out_len, int32_t* __restrict__ out_col,
                                                      float* __restrict__ out_w, double* __restrict__ K2,
                                                      double* __restrict__ S2, int32_t* __restrict__ pkeys,
                                                      double* __restrict__ pvals) {
  __shared__ int32_t s_keys[kFBlockSlots];
  __shared__ double s_vals[kFBlockSlots];
  __shared__ double s_r[kFNW];
  __shared__ int32_t s_n;
  for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const int64_t v0 = vstart[c], vol = vstart[c + 1] - v0;
    const bool big = vol > kFBlockMax;
    const uint32_t ts = big ? static_cast<uint32_t>(1) << (32 - __clz(static_cast<uint32_t>(2 * vol - 1)))
                            : static_cast<uint32_t>(kFBlockSlots);
    int32_t* keys = big ? pkeys + 4 * v0 : s_keys;  // ts <= 4 vol
    double* vals = big ? pvals + 4 * v0 : s_vals;
    for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
      keys[t] = -1;
      vals[t] = 0.0;
    }
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int32_t q = coff[c]; q < coff[c + 1]; ++q) {
      const int32_t i = cmem[q];
      const int64_t s = g.row_start[i];
      const int32_t len = g.row_len[i];
      for (int32_t k = threadIdx.x; k < len; k += kBlock)
        tab_add(keys, vals, ts, C[g.col[s + k]], static_cast<double>(g.w[s + k]));
    }
    __syncthreads();
    double k2 = 0.0;
    for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
      const int32_t d = big ? ld_agent(&keys[t]) : keys[t];
      if (d < 0) continue;
      const float x = static_cast<float>(big ? ld_agent(&vals[t]) : vals[t]);
      const int32_t p = atomicAdd(&s_n, 1);
      out_col[v0 + p] = d;
      out_w[v0 + p] = x;
      k2 += static_cast<double>(x);
    }
    k2 = block_sum_d(k2, s_r);
    if (threadIdx.x == 0) {
      out_len[c] = s_n;
      K2[c] = k2;
      S2[c] = k2;
    }
    __syncthreads();
  }
}

__global__ void k_f_sigma(const int32_t* __restrict__ C, const double* __restrict__ K, int32_t n,
                          double* __restrict__ Sigma) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (K[i] != 0.0) atomicAdd(&Sigma[C[i]], K[i]);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct FWs {
  int64_t words = 0;
  uint32_t *fa = nullptr, *fb = nullptr, *ever = nullptr;
  int32_t* list[FB_N] = {};
  int32_t* size = nullptr;
  int32_t* lC = nullptr;
  double *lK = nullptr, *lS = nullptr, *tot = nullptr;
  int32_t *flags = nullptr, *newid = nullptr, *ccount = nullptr, *coff = nullptr, *cmem = nullptr;
  int64_t *vol = nullptr, *vstart = nullptr;
  int64_t* lrs[2] = {};
  int32_t* llen[2] = {};
  int32_t* lcol[2] = {};
  float* lw[2] = {};
  int32_t* pkeys = nullptr;
  double* pvals = nullptr;
  int64_t pool_slots = 0;
  // batch edit tables
  unsigned long long* pkey = nullptr;
  int32_t* pzero = nullptr;
  int64_t psize = 0;
  int32_t *rkey = nullptr, *rapp = nullptr, *rzero = nullptr;
  int64_t rsize = 0;
  int32_t *dpos = nullptr, *imode = nullptr;
  Workspace scan;  // scan partials only
  int64_t* ctr = nullptr;
  size_t bytes = 0;
};

size_t carve_f(FWs& w, void* base, int32_t n, int64_t cap) {
  char* cur = static_cast<char*>(base);
  size_t total = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? cur : nullptr;
    const size_t b = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    cur += b;
    total += b;
    return p;
  };
  const size_t un = static_cast<size_t>(n > 0 ? n : 1), ucap = static_cast<size_t>(cap > 0 ? cap : 1);
  w.words = (static_cast<int64_t>(un) + 31) / 32 + 1;
  w.fa = static_cast<uint32_t*>(take(4 * w.words));
  w.fb = static_cast<uint32_t*>(take(4 * w.words));
  w.ever = static_cast<uint32_t*>(take(4 * w.words));
  for (int b = 0; b < FB_N; ++b) w.list[b] = static_cast<int32_t*>(take(4 * un));
  w.size = static_cast<int32_t*>(take(4 * un));
  w.lC = static_cast<int32_t*>(take(4 * un));
  w.lK = static_cast<double*>(take(8 * un));
  w.lS = static_cast<double*>(take(8 * un));
  w.tot = static_cast<double*>(take(8 * un));
  w.flags = static_cast<int32_t*>(take(4 * (un + 1)));
  w.newid = static_cast<int32_t*>(take(4 * (un + 1)));
  w.ccount = static_cast<int32_t*>(take(4 * (un + 1)));
  w.coff = static_cast<int32_t*>(take(4 * (un + 1)));
  w.cmem = static_cast<int32_t*>(take(4 * un));
  w.vol = static_cast<int64_t*>(take(8 * (un + 1)));
  w.vstart = static_cast<int64_t*>(take(8 * (un + 1)));
  for (int k = 0; k < 2; ++k) {
    w.lrs[k] = static_cast<int64_t*>(take(8 * (un + 1)));
    w.llen[k] = static_cast<int32_t*>(take(4 * un));
    w.lcol[k] = static_cast<int32_t*>(take(4 * ucap));
    w.lw[k] = static_cast<float*>(take(4 * ucap));
  }
  w.pool_slots = 4 * static_cast<int64_t>(ucap) + 8192;
  w.pkeys = static_cast<int32_t*>(take(4 * static_cast<size_t>(w.pool_slots)));
  w.pvals = static_cast<double*>(take(8 * static_cast<size_t>(w.pool_slots)));
  w.scan.scan_part_len = scan_parts_needed(static_cast<int64_t>(un) + 2) + 8;
  w.scan.scan_part = static_cast<int64_t*>(take(8 * static_cast<size_t>(w.scan.scan_part_len)));
  w.ctr = static_cast<int64_t*>(take(8 * F_COUNT));
  w.bytes = total;
  return total;
}

// Carves the batch tables out of the pool for a batch of `updates`.
bool carve_batch(FWs& w, int64_t updates) {
  int64_t ps = 64;
  while (ps < 4 * updates) ps <<= 1;
  int64_t rs = 64;
  while (rs < 4 * updates) rs <<= 1;
  const size_t need = 8 * ps + 4 * ps + 12 * rs + 4 * 2 * updates + 4 * updates + 8 * 256;
  // the pool (keys, then values: 12 bytes a slot) is free during a batch edit
  if (need > static_cast<size_t>(w.pool_slots) * 12) return false;
  char* p = reinterpret_cast<char*>(w.pkeys);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~size_t(255);
    return q;
  };
  w.psize = ps;
  w.rsize = rs;
  w.pkey = reinterpret_cast<unsigned long long*>(take(8 * ps));
  w.pzero = reinterpret_cast<int32_t*>(take(4 * ps));
  w.rkey = reinterpret_cast<int32_t*>(take(4 * rs));
  w.rapp = reinterpret_cast<int32_t*>(take(4 * rs));
  w.rzero = reinterpret_cast<int32_t*>(take(4 * rs));
  w.dpos = reinterpret_cast<int32_t*>(take(8 * std::max<int64_t>(updates, 1)));
  w.imode = reinterpret_cast<int32_t*>(take(4 * std::max<int64_t>(updates, 1)));
  return true;
}

#define F_HIP(expr)                                                          \
  do {                                                                       \
    hipError_t e__ = (expr);                                                 \
    if (e__ != hipSuccess) return lv_fail(LV_EHIP, hipGetErrorString(e__));  \
  } while (0)

int blocks(int64_t items, int cap = 8192) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, cap)));
}

lv_status setup(FWs& w, const lv_graph_f* g, void* ws, size_t ws_bytes) {
  if (!g || g->n <= 0 || !g->row_start || !g->row_len || !g->col || !g->w || !g->two_m || g->cap < 0)
    return lv_fail(LV_EINVAL, "invalid graph");
  if (g->cap >= (int64_t(1) << 30)) return lv_fail(LV_EINVAL, "capacity of 2^30 arcs or more");
  if (!ws) return lv_fail(LV_EINVAL, "workspace pointer is null");
  if (ws_bytes < carve_f(w, nullptr, g->n, g->cap)) return lv_fail(LV_EWORKSPACE, "workspace too small");
  carve_f(w, ws, g->n, g->cap);
  return LV_OK;
}

// Counters back on the host (the error slot and the statistics replicas).
struct FRead {
  int64_t err = 0, movers = 0, arcs = 0, processed = 0, expand = 0, affected = 0;
  double dq = 0.0, sum = 0.0, sum2 = 0.0;
};
lv_status read(const FWs& w, FRead& r, hipStream_t st) {
  std::vector<int64_t> h(F_COUNT);
  F_HIP(hipMemcpyAsync(h.data(), w.ctr, sizeof(int64_t) * F_COUNT, hipMemcpyDeviceToHost, st));
  F_HIP(hipStreamSynchronize(st));
  r = FRead{};
  r.err = h[F_ERR];
  for (int k = 0; k < kFReps; ++k) {
    const int64_t* x = h.data() + F_STATS + k * kCtrLine;
    r.movers += x[FS_MOVERS];
    r.arcs += x[FS_ARCS];
    r.processed += x[FS_PROCESSED];
    r.expand += x[FS_EXPAND];
    r.affected += x[FS_AFFECTED];
    double d;
    std::memcpy(&d, x + FS_DQ, 8);
    r.dq += d;
    std::memcpy(&d, x + FS_SUM, 8);
    r.sum += d;
    std::memcpy(&d, x + FS_SUM2, 8);
    r.sum2 += d;
  }
  return LV_OK;
}

lv_status zero_stats(const FWs& w, hipStream_t st) {
  F_HIP(hipMemsetAsync(w.ctr + F_LIST0, 0, sizeof(int64_t) * (F_COUNT - F_LIST0), st));
  return LV_OK;
}

lv_status dev_error(int64_t code) {
  if (code == LV_EEMPTY) return lv_fail(LV_EEMPTY, "graph has no edges (2m = 0)");
  if (code == LV_EINVAL) return lv_fail(LV_EINVAL, "the batch names a vertex outside [0, n), a self-loop or a "
                                                   "weight that is not finite and positive");
  if (code == LV_ENOEDGE) return lv_fail(LV_ENOEDGE, "a deletion names a missing edge or more weight than present");
  if (code == LV_ENOSLACK) return lv_fail(LV_ENOSLACK, "a row lacks free capacity; nothing was changed");
  if (code == LV_EWORKSPACE) return lv_fail(LV_EWORKSPACE, "workspace pool too small");
  return lv_fail(static_cast<lv_status>(code), "device error");
}

bool params_ok_f(const lv_params* p) {
  return p && p->mode == LV_ASYNC && p->max_iterations >= 1 && p->max_iterations <= LV_MAX_ITERS &&
         p->max_passes >= 1 && p->max_passes <= LV_MAX_PASSES && p->tolerance >= 0.0 && p->tolerance_drop > 0.0 &&
         p->aggregation_tolerance >= 0.0 && p->recompute_weights == 0 && p->reserved == 0;
}

FBatch fbatch(const lv_edges_f* del, const lv_edges_f* ins) {
  FBatch b{};
  if (del && del->count > 0) {
    b.du = del->u;
    b.dv = del->v;
    b.dw = del->w;
    b.nd = del->count;
  }
  if (ins && ins->count > 0) {
    b.iu = ins->u;
    b.iv = ins->v;
    b.iw = ins->w;
    b.ni = ins->count;
  }
  return b;
}

bool edges_ok_f(const lv_edges_f* e) { return !e || e->count == 0 || (e->count > 0 && e->u && e->v && e->w); }

// Alg. 4 in the paper's precision, ASYNC; DF marking and updateWeights first
// for the dynamic call.
lv_status run_f(bool df, const lv_graph_f* g, const lv_edges_f* del, const lv_edges_f* ins, const lv_params* p,
                lv_state_f* state, void* wsp, size_t ws_bytes, lv_stats* stats, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!params_ok_f(p)) return lv_fail(LV_EINVAL, "invalid parameters (the paper-precision path runs LV_ASYNC)");
  if (!state || !state->C || !state->K || !state->Sigma) return lv_fail(LV_EINVAL, "invalid state");
  if (df && (!edges_ok_f(del) || !edges_ok_f(ins))) return lv_fail(LV_EINVAL, "invalid batch");
  FWs w;
  lv_status s = setup(w, g, wsp, ws_bytes);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  lv_stats local;
  lv_stats& S = stats ? *stats : local;
  std::memset(&S, 0, sizeof(lv_stats));
  const int32_t N = g->n;
  const lv_tuning tu = lv_effective_tuning();
  hipLaunchKernelGGL(k_f_begin, dim3(blocks(std::max<int64_t>(w.words, F_COUNT), 2048)), dim3(kBlock), 0, st, w.ctr,
                     w.fa, w.fb, w.ever, w.words, g->two_m);
  FG L0{N, g->row_start, g->row_len, g->col, g->w};
  int32_t* size0 = state->size ? state->size : w.size;
  if (!df) {
    hipLaunchKernelGGL(k_f_rows, dim3(blocks(static_cast<int64_t>(N) * kWave, 16384)), dim3(kBlock), 0,
                       st, L0, nullptr, state->K, state->Sigma, state->C, size0, w.ctr);
    hipLaunchKernelGGL(k_f_set_all, dim3(blocks(w.words)), dim3(kBlock), 0, st, w.fa, N, w.words);
  } else {
    const FBatch b = fbatch(del, ins);
    hipLaunchKernelGGL(k_f_check_c, dim3(blocks(N)), dim3(kBlock), 0, st, state->C, N, w.ctr);
    FRead rc;
    if ((s = read(w, rc, st))) return s;  // (the member counts below index by C)
    if (rc.err) return rc.err == LV_EINVAL ? lv_fail(LV_EINVAL, "a membership lies outside [0, n)")
                                           : dev_error(rc.err);
    if (b.nd + b.ni > 0)
      hipLaunchKernelGGL(k_f_update, dim3(blocks(b.nd + b.ni)), dim3(kBlock), 0, st, b, N, state->C, state->K,
                         state->Sigma, w.fa, w.ctr);
    if (!state->size) launch_community_sizes(state->C, N, w.size, st);
  }
  F_HIP(hipGetLastError());
  double two_m = 0.0;
  F_HIP(hipMemcpyAsync(&two_m, g->two_m, sizeof(double), hipMemcpyDeviceToHost, st));
  FRead rd;
  if ((s = read(w, rd, st))) return s;
  if (rd.err) return dev_error(rd.err);
  const double m = two_m / 2.0;

  FG L = L0;
  int32_t* Cl = state->C;
  const double* Kl = state->K;
  double* Sl = state->Sigma;
  int32_t* size = size0;
  uint32_t* cur = w.fa;
  uint32_t* next = w.fb;
  double tau = p->tolerance;
  bool aggregated = false;
  for (int32_t pass = 0; pass < p->max_passes; ++pass) {
    int32_t li = p->max_iterations;
    int64_t est = L.n;
    if (pass == 0 && df) est = 2 * (fbatch(del, ins).nd + fbatch(del, ins).ni);
    for (int32_t it = 0; it < p->max_iterations; ++it) {
      if ((s = zero_stats(w, st))) return s;
      const std::vector<SubRound> plan = lv_sub_rounds(LV_ASYNC, pass, est, L.n, tu);
      for (size_t r = 0; r < plan.size(); ++r) {
        F_HIP(hipMemsetAsync(w.ctr + F_LIST0, 0, sizeof(int64_t) * 4 * kCtrLine, st));  // lists and pool
        hipLaunchKernelGGL(k_f_bin, dim3(blocks(w.words, 4096)), dim3(kBlock), 0, st, cur,
                           pass == 0 ? w.ever : nullptr, L.row_len, L.n, plan[r].hash_round, plan[r].hash_shift,
                           plan[r].id_lo, plan[r].id_hi, plan[r].deg_lo, plan[r].deg_hi, r + 1 == plan.size() ? 1 : 0, w.list[FB_WAVE],
                           w.list[FB_BLOCK], w.list[FB_HUB], w.ctr);
        FMove M{L, Cl, Kl, Sl, size, next, {w.list[FB_WAVE], w.list[FB_BLOCK], w.list[FB_HUB]}, m,
                p->swap_guard, w.ctr, w.pool_slots, w.pkeys, w.pvals};
        const int64_t e = std::max<int64_t>(64, est);
        hipLaunchKernelGGL(k_f_scan_group<true>, dim3(static_cast<int>(std::min<int64_t>(e, 1024))), dim3(kBlock), 0,
                           st, M);
        hipLaunchKernelGGL(k_f_scan_group<false>, dim3(static_cast<int>(std::min<int64_t>(e, 2048))), dim3(kBlock),
                           0, st, M);
        hipLaunchKernelGGL(k_f_scan_wave, dim3(blocks(e * kWave / kFNW, 4096)), dim3(kBlock), 0, st, M);
      }
      F_HIP(hipGetLastError());
      std::swap(cur, next);
      if ((s = read(w, rd, st))) return s;
      if (rd.err) return dev_error(rd.err);
      est = rd.expand;
      S.moves += rd.movers;
      S.arcs_scanned += rd.arcs;
      if (pass == 0) S.vertices_affected += rd.affected;
      if (pass < LV_MAX_PASSES && it < LV_MAX_ITERS) S.iter_moves[pass][it] = rd.movers;
      if (rd.dq <= tau) {
        li = it + 1;
        break;
      }
    }
    S.passes = pass + 1;
    S.iterations[pass] = li;
    if (li <= 1) break;
    // renumber (ascending old id), then the aggregation stop
    F_HIP(hipMemsetAsync(w.flags, 0, sizeof(int32_t) * (static_cast<size_t>(L.n) + 1), st));
    launch_mark_exists(Cl, L.n, w.flags, st);
    exclusive_scan_i32(w.flags, w.newid, L.n, w.scan, st);
    int32_t nc = 0;
    F_HIP(hipMemcpyAsync(&nc, w.newid + L.n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    F_HIP(hipStreamSynchronize(st));
    S.communities[pass] = nc;
    if (static_cast<double>(nc) / static_cast<double>(L.n) > p->aggregation_tolerance) break;
    launch_relabel(Cl, L.n, w.newid, st);
    if (pass > 0) launch_lookup(state->C, N, Cl, st);
    // members and volumes of the communities
    F_HIP(hipMemsetAsync(w.ccount, 0, sizeof(int32_t) * (static_cast<size_t>(nc) + 1), st));
    F_HIP(hipMemsetAsync(w.vol, 0, sizeof(int64_t) * (static_cast<size_t>(nc) + 1), st));
    launch_accumulate(Cl, L.n, L.row_len, nullptr, w.ccount, w.vol, st);  // member counts, volumes
    exclusive_scan_i32(w.ccount, w.coff, nc, w.scan, st);
    F_HIP(hipMemsetAsync(w.flags, 0, sizeof(int32_t) * (static_cast<size_t>(nc) + 1), st));
    launch_fill_members(Cl, L.n, w.coff, w.flags, w.cmem, st);
    const int k = pass & 1;
    exclusive_scan_i64(w.vol, w.lrs[k], nc, w.scan, st);
    hipLaunchKernelGGL(k_f_aggregate, dim3(static_cast<int>(std::min<int32_t>(nc, 8192))), dim3(kBlock), 0, st, L,
                       Cl, w.coff, w.cmem, w.lrs[k], nc, w.llen[k], w.lcol[k], w.lw[k], w.lK, w.lS, w.pkeys,
                       w.pvals);
    // the aggregate read the level's memberships (w.lC past the first pass)
    launch_iota_i32(w.lC, nc, st);
    launch_fill_i32(w.size, 1, nc, st);
    hipLaunchKernelGGL(k_f_set_all, dim3(blocks(w.words)), dim3(kBlock), 0, st, cur, nc, w.words);
    F_HIP(hipGetLastError());
    L = FG{nc, w.lrs[k], w.llen[k], w.lcol[k], w.lw[k]};
    Cl = w.lC;
    Kl = w.lK;
    Sl = w.lS;
    size = w.size;
    tau /= p->tolerance_drop;
    aggregated = true;
  }
  if (aggregated) {
    launch_lookup(state->C, N, Cl, st);
    hipLaunchKernelGGL(k_f_zero_d, dim3(blocks(N)), dim3(kBlock), 0, st, state->Sigma, static_cast<int64_t>(N));
    hipLaunchKernelGGL(k_f_sigma, dim3(blocks(N)), dim3(kBlock), 0, st, state->C, state->K, N, state->Sigma);
    if (state->size) launch_community_sizes(state->C, N, state->size, st);
    F_HIP(hipGetLastError());
  }
  F_HIP(hipStreamSynchronize(st));
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return LV_OK;
}

}  // namespace
}  // namespace lv

using namespace lv;

extern "C" {

size_t lv_workspace_bytes_f(int32_t n, int64_t cap) {
  FWs w;
  return carve_f(w, nullptr, n, cap);
}

lv_status lv_graph_build_f(lv_graph_f* g, const lv_edges_f* e, float slack_frac, int32_t slack_min, void* wsp,
                           size_t ws_bytes, void* stream) {
  if (!e || !edges_ok_f(e) || slack_frac < 0.f || slack_min < 0) return lv_fail(LV_EINVAL, "invalid arguments");
  FWs w;
  lv_status s = setup(w, g, wsp, ws_bytes);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t n = g->n;
  F_HIP(hipMemsetAsync(w.ctr, 0, sizeof(int64_t) * F_COUNT, st));
  F_HIP(hipMemsetAsync(g->row_len, 0, sizeof(int32_t) * static_cast<size_t>(n), st));
  if (e->count > 0)
    hipLaunchKernelGGL(k_f_count, dim3(blocks(e->count)), dim3(kBlock), 0, st, e->u, e->v, e->w, e->count, n,
                       g->row_len, w.ctr);
  // capacities: deg + max(slack_min, ceil(frac * deg)), then their scan
  launch_row_capacity(g->row_len, w.vol, n, slack_frac, slack_min, st);
  exclusive_scan_i64(w.vol, g->row_start, n, w.scan, st);
  FRead rd;
  if ((s = read(w, rd, st))) return s;
  if (rd.err) return dev_error(rd.err);
  int64_t need = 0;
  F_HIP(hipMemcpyAsync(&need, g->row_start + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  F_HIP(hipStreamSynchronize(st));
  if (need > g->cap) return lv_fail(LV_ENOSLACK, "graph capacity too small (see lv_graph_capacity_bound)");
  F_HIP(hipMemsetAsync(g->row_len, 0, sizeof(int32_t) * static_cast<size_t>(n), st));
  if (e->count > 0)
    hipLaunchKernelGGL(k_f_scatter, dim3(blocks(e->count)), dim3(kBlock), 0, st, e->u, e->v, e->w, e->count,
                       g->row_start, g->row_len, g->col, g->w);
  FG G{n, g->row_start, g->row_len, g->col, g->w};
  hipLaunchKernelGGL(k_f_rows, dim3(blocks(static_cast<int64_t>(n) * kWave, 16384)), dim3(kBlock), 0, st,
                     G, nullptr, nullptr, nullptr, nullptr, nullptr, w.ctr);
  hipLaunchKernelGGL(k_f_set_two_m, dim3(1), dim3(1), 0, st, g->two_m, w.ctr, 0);
  F_HIP(hipGetLastError());
  F_HIP(hipStreamSynchronize(st));
  return LV_OK;
}

lv_status apply_batch_f(lv_graph_f* g, const lv_edges_f* del, const lv_edges_f* ins, void* wsp, size_t ws_bytes,
                        void* stream) {
  if (!edges_ok_f(del) || !edges_ok_f(ins)) return lv_fail(LV_EINVAL, "invalid batch");
  FWs w;
  lv_status s = setup(w, g, wsp, ws_bytes);
  if (s) return s;
  const FBatch b = fbatch(del, ins);
  if (b.nd + b.ni == 0) return LV_OK;
  if (!carve_batch(w, b.nd + b.ni)) return lv_fail(LV_EWORKSPACE, "batch too large for the workspace pool");
  hipStream_t st = static_cast<hipStream_t>(stream);
  F_HIP(hipMemsetAsync(w.ctr, 0, sizeof(int64_t) * F_COUNT, st));
  F_HIP(hipMemsetAsync(w.pkey, 0, 8 * static_cast<size_t>(w.psize), st));
  F_HIP(hipMemsetAsync(w.pzero, 0, 4 * static_cast<size_t>(w.psize), st));
  F_HIP(hipMemsetAsync(w.rkey, 0, 4 * static_cast<size_t>(w.rsize), st));
  F_HIP(hipMemsetAsync(w.rapp, 0, 4 * static_cast<size_t>(w.rsize), st));
  F_HIP(hipMemsetAsync(w.rzero, 0, 4 * static_cast<size_t>(w.rsize), st));
  FBTab t{w.pkey, w.pzero, w.psize, w.rkey, w.rapp, w.rzero, w.rsize, w.dpos, w.imode};
  lv_graph_f G = *g;
  if (b.nd) hipLaunchKernelGGL(k_f_val_del, dim3(blocks(b.nd)), dim3(kBlock), 0, st, b, G, t, w.ctr);
  if (b.ni) hipLaunchKernelGGL(k_f_val_ins, dim3(blocks(b.ni)), dim3(kBlock), 0, st, b, G, t, w.ctr);
  hipLaunchKernelGGL(k_f_val_cap, dim3(blocks(w.rsize)), dim3(kBlock), 0, st, G, t, w.ctr);
  F_HIP(hipGetLastError());
  FRead rd;
  if ((s = read(w, rd, st))) return s;
  if (rd.err) return dev_error(rd.err);
  if (b.nd) hipLaunchKernelGGL(k_f_del, dim3(blocks(b.nd)), dim3(kBlock), 0, st, b, G, t, w.ctr);
  hipLaunchKernelGGL(k_f_compact, dim3(blocks(w.rsize)), dim3(kBlock), 0, st, G, t, w.ctr);
  if (b.ni) hipLaunchKernelGGL(k_f_ins, dim3(blocks(b.ni)), dim3(kBlock), 0, st, b, G, t, w.ctr);
  hipLaunchKernelGGL(k_f_set_two_m, dim3(1), dim3(1), 0, st, g->two_m, w.ctr, 1);
  F_HIP(hipGetLastError());
  F_HIP(hipStreamSynchronize(st));
  return LV_OK;
}

lv_status louvain_static_f(const lv_graph_f* g, const lv_params* p, lv_state_f* out, void* ws, size_t ws_bytes,
                           lv_stats* stats, void* stream) {
  return run_f(false, g, nullptr, nullptr, p, out, ws, ws_bytes, stats, stream);
}

lv_status louvain_df_f(const lv_graph_f* g, const lv_edges_f* del, const lv_edges_f* ins, const lv_params* p,
                       lv_state_f* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream) {
  return run_f(true, g, del, ins, p, state, ws, ws_bytes, stats, stream);
}

lv_status modularity_f(const lv_graph_f* g, const int32_t* C, double* q_host, void* wsp, size_t ws_bytes,
                       void* stream) {
  if (!C || !q_host) return lv_fail(LV_EINVAL, "invalid arguments");
  FWs w;
  lv_status s = setup(w, g, wsp, ws_bytes);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t n = g->n;
  F_HIP(hipMemsetAsync(w.ctr, 0, sizeof(int64_t) * F_COUNT, st));
  FG G{n, g->row_start, g->row_len, g->col, g->w};
  hipLaunchKernelGGL(k_f_rows, dim3(blocks(static_cast<int64_t>(n) * kWave, 16384)), dim3(kBlock), 0, st,
                     G, C, w.lK, nullptr, nullptr, nullptr, w.ctr);
  FRead rd;
  if ((s = read(w, rd, st))) return s;
  const double intra = rd.sum2;
  F_HIP(hipMemsetAsync(w.ctr, 0, sizeof(int64_t) * F_COUNT, st));
  hipLaunchKernelGGL(k_f_zero_d, dim3(blocks(n)), dim3(kBlock), 0, st, w.tot, static_cast<int64_t>(n));
  hipLaunchKernelGGL(k_f_totals, dim3(blocks(n)), dim3(kBlock), 0, st, C, w.lK, n, w.tot, w.ctr);
  hipLaunchKernelGGL(k_f_sumsq, dim3(blocks(n, 4096)), dim3(kBlock), 0, st, w.tot, n, w.ctr);
  F_HIP(hipGetLastError());
  double two_m = 0.0;
  F_HIP(hipMemcpyAsync(&two_m, g->two_m, sizeof(double), hipMemcpyDeviceToHost, st));
  if ((s = read(w, rd, st))) return s;
  if (rd.err) return lv_fail(LV_EINVAL, "a membership lies outside [0, n)");
  if (!(two_m > 0.0)) return lv_fail(LV_EEMPTY, "graph has no edges (2m = 0)");
  *q_host = intra / two_m - rd.sum / (two_m * two_m);
  return LV_OK;
}

}  // extern "C"
