// Community renumbering and dendrogram lookup (Alg. 4) and the aggregation
// phase (Alg. 6): the community-vertex CSR by count / scan / fill, super-
// vertex row capacities from community volumes (the paper's over-estimated,
// "holey" offsets), and per community a hashtable over its members' arcs,
// self-loops included, whose entries become the super-vertex's row.
//
// Three tiers by community volume (arcs of all members):
//   <= 256   one wavefront, LDS table of 512 slots;
//   <= 2048  one workgroup, LDS table of 4096 slots;
//   larger   many workgroups: the community's arc range is cut into units of
//            2048 arcs; each unit sums its arcs per neighbour community in an
//            LDS table (at most 2048 keys in 4096 slots) and flushes the sums
//            into the community's global table (2 x min(volume, communities)
//            slots of packed key:weight pairs), then emit units compact the
//            table into the row.
// Arcs into the community itself (its self-loop weight, usually the most
// frequent key) are summed in registers in every tier.  K''_c = Σ''_c is
// the row sum.
#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int kAggWaveVol = 256;
constexpr int kAggWaveTS = 512;
constexpr int kAggBlockVol = 2048;
constexpr int kAggBlockTS = 4096;
constexpr int kUnitArcs = 2048;       // arcs per insert unit of a big community
constexpr int kArcsPerThread = kUnitArcs / kBlock;
constexpr int kEmitSlots = 4096;      // table slots per emit unit
constexpr int kUnitTS = 4096;         // LDS slots for a unit's pre-aggregation
// A global table slot packs a key (high half) and a weight (low half): one
// compare-and-swap inserts a new key with its weight; a hit adds to the low
// half, which never carries (a sum of arc weights stays below 2m < 2^31).
constexpr unsigned long long kEmptyPair = 0xFFFFFFFF00000000ull;

__device__ __forceinline__ unsigned long long pack_pair(int32_t d, int32_t x) {
  return (static_cast<unsigned long long>(static_cast<uint32_t>(d)) << 32) | static_cast<uint32_t>(x);
}

// Global table slots of a big community: distinct neighbour communities are
// at most min(volume, communities), load factor <= 1/2.
__device__ __forceinline__ int64_t big_slots(int64_t vol, int32_t nc) { return 2 * min(vol, static_cast<int64_t>(nc)); }

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

// arcs of the k-th member in community-vertex order (for the arc prefix)
__global__ void k_member_degrees(const int32_t* __restrict__ cmem, const int32_t* __restrict__ row_len, int32_t n,
                                 int64_t* __restrict__ out) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[k] = row_len[cmem[k]];
}

// Split communities by volume; big ones get a global table (their insert /
// emit units are written by k_big_units).  Each thread takes kBinItems
// consecutive communities and each workgroup reserves its list entries with
// one atomic per list.
constexpr int kBinItems = 16;
__global__ void __launch_bounds__(kBlock) k_bin_communities(const int64_t* __restrict__ out_start, int32_t nc,
                                  int32_t* __restrict__ small, int32_t* __restrict__ medium,
                                  int32_t* __restrict__ big, int64_t* __restrict__ big_off,
                                  int32_t* __restrict__ out_len, int64_t* __restrict__ Kout,
                                  int64_t* __restrict__ Sout, int64_t* __restrict__ ctr) {
  __shared__ int64_t lds[kBlock / kWave + 1];
  const int64_t span = static_cast<int64_t>(kBlock) * kBinItems;
  for (int64_t c0 = blockIdx.x * span; c0 < nc; c0 += static_cast<int64_t>(gridDim.x) * span) {
    const int64_t first = c0 + static_cast<int64_t>(threadIdx.x) * kBinItems;
    int64_t ns = 0, nm = 0, nb = 0, pool = 0;
    for (int q = 0; q < kBinItems && first + q < nc; ++q) {
      const int64_t c = first + q;
      const int64_t vol = out_start[c + 1] - out_start[c];
      if (vol == 0 || vol > kAggBlockVol) {  // empty rows and big rows start from zero
        out_len[c] = 0;
        Kout[c] = 0;
        Sout[c] = 0;
      }
      ns += (vol > 0 && vol <= kAggWaveVol) ? 1 : 0;
      nm += (vol > kAggWaveVol && vol <= kAggBlockVol) ? 1 : 0;
      if (vol > kAggBlockVol) {
        nb += 1;
        pool += big_slots(vol, nc);
      }
    }
    int64_t ps = block_reserve(ns, &ctr[CTR_AGG_SMALL], lds);
    int64_t pm = block_reserve(nm, &ctr[CTR_AGG_MEDIUM], lds);
    int64_t pb = block_reserve(nb, &ctr[CTR_AGG_BIG], lds);
    int64_t pp = block_reserve(pool, &ctr[CTR_AGG_POOL], lds);
    for (int q = 0; q < kBinItems && first + q < nc; ++q) {
      const int64_t c = first + q;
      const int64_t vol = out_start[c + 1] - out_start[c];
      if (vol > 0 && vol <= kAggWaveVol) {
        small[ps++] = static_cast<int32_t>(c);
      } else if (vol > kAggWaveVol && vol <= kAggBlockVol) {
        medium[pm++] = static_cast<int32_t>(c);
      } else if (vol > kAggBlockVol) {
        big[pb] = static_cast<int32_t>(c);
        big_off[pb++] = pp;
        pp += big_slots(vol, nc);
      }
    }
  }
}

// One thread per big community writes its unit descriptors.
__global__ void k_big_units(const int32_t* __restrict__ big, const int64_t* __restrict__ out_start, int32_t nc,
                            int32_t* __restrict__ ins_b, int64_t* __restrict__ ins_a, int32_t* __restrict__ emit_b,
                            int64_t* __restrict__ emit_s, int64_t* __restrict__ ctr) {
  const int64_t count = ctr[CTR_AGG_BIG];
  for (int64_t b = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; b < count;
       b += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t c = big[b];
    const int64_t vol = out_start[c + 1] - out_start[c];
    const int64_t nu = (vol + kUnitArcs - 1) / kUnitArcs;
    const int64_t ne = (big_slots(vol, nc) + kEmitSlots - 1) / kEmitSlots;
    const int64_t bu = static_cast<int64_t>(
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_UNITS_INS]), static_cast<unsigned long long>(nu)));
    const int64_t be = static_cast<int64_t>(
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[CTR_UNITS_EMIT]), static_cast<unsigned long long>(ne)));
    for (int64_t u = 0; u < nu; ++u) {
      ins_b[bu + u] = static_cast<int32_t>(b);
      ins_a[bu + u] = u * kUnitArcs;
    }
    for (int64_t u = 0; u < ne; ++u) {
      emit_b[be + u] = static_cast<int32_t>(b);
      emit_s[be + u] = u * kEmitSlots;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_big_clear(const int32_t* __restrict__ emit_b,
                                                     const int64_t* __restrict__ emit_s,
                                                     const int32_t* __restrict__ big, const int64_t* __restrict__ big_off,
                                                     const int64_t* __restrict__ out_start,
                                                     const int64_t* __restrict__ ctr, int32_t nc,
                                                     unsigned long long* __restrict__ tab, int64_t pool_slots) {
  const int64_t count = ctr[CTR_UNITS_EMIT];
  for (int64_t u = blockIdx.x; u < count; u += gridDim.x) {
    const int32_t b = emit_b[u];
    const int32_t c = big[b];
    const int64_t tsz = big_slots(out_start[c + 1] - out_start[c], nc);
    const int64_t off = big_off[b];
    if (off + tsz > pool_slots) continue;  // reported by the insert kernel
    const int64_t s1 = min(tsz, emit_s[u] + kEmitSlots);
    for (int64_t s = emit_s[u] + threadIdx.x; s < s1; s += kBlock) tab[off + s] = kEmptyPair;
  }
}

__device__ __forceinline__ void table_add(unsigned long long* tab, uint32_t tsz, int32_t d, int32_t x) {
  uint32_t h = hash_slot(static_cast<uint32_t>(d), tsz);
  while (true) {
    const unsigned long long old = atomicCAS(&tab[h], kEmptyPair, pack_pair(d, x));
    if (old == kEmptyPair) return;
    if (static_cast<int32_t>(old >> 32) == d) {
      atomicAdd(&tab[h], static_cast<unsigned long long>(static_cast<uint32_t>(x)));
      return;
    }
    h = (h + 1 == tsz) ? 0 : h + 1;
  }
}

// One workgroup per insert unit.  The unit's members' first-arc offsets are
// staged in LDS; each thread then takes kArcsPerThread consecutive arcs and
// issues their loads in batches (member rows, arcs, neighbour communities)
// so the latencies overlap; sums go to the LDS table, and the table is
// flushed in rounds of compare-and-swaps that are in flight together.
__global__ void __launch_bounds__(kBlock) k_big_insert(
    const int64_t* __restrict__ row_start, const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
    const int32_t* __restrict__ C, const int32_t* __restrict__ coff, const int32_t* __restrict__ cmem,
    const int64_t* __restrict__ mpre, const int32_t* __restrict__ ins_b, const int64_t* __restrict__ ins_a,
    const int32_t* __restrict__ big, const int64_t* __restrict__ big_off, const int64_t* __restrict__ out_start,
    int64_t* __restrict__ ctr, int32_t nc, unsigned long long* __restrict__ tab_all, int64_t pool_slots) {
  constexpr int A = kArcsPerThread;
  __shared__ int32_t tk[kUnitTS];
  __shared__ int32_t tv[kUnitTS];
  __shared__ int32_t s_moff[kUnitArcs + 2];  // member first-arc offsets from the unit start
  __shared__ int32_t s_mlo, s_mcnt;
  __shared__ int64_t r_self[kBlock / kWave];
  const int64_t count = ctr[CTR_UNITS_INS];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  for (int64_t u = blockIdx.x; u < count; u += gridDim.x) {
    const int32_t b = ins_b[u];
    const int32_t c = big[b];
    const int64_t vol = out_start[c + 1] - out_start[c];
    const uint32_t tsz = static_cast<uint32_t>(big_slots(vol, nc));
    const int64_t off = big_off[b];
    if (off + static_cast<int64_t>(tsz) > pool_slots) {
      if (threadIdx.x == 0) set_error(ctr, LV_EWORKSPACE);
      continue;
    }
    unsigned long long* tab = tab_all + off;
    for (int sl = threadIdx.x; sl < kUnitTS; sl += kBlock) {
      tk[sl] = -1;
      tv[sl] = 0;
    }
    const int32_t m0 = coff[c], m1 = coff[c + 1];
    const int64_t base = mpre[m0];
    const int64_t a_u = ins_a[u];
    if (threadIdx.x == 0) {  // last member whose first arc is <= the unit's first arc
      int32_t lo = m0, hi = m1 - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (mpre[mid] - base <= a_u) lo = mid;
        else hi = mid - 1;
      }
      s_mlo = lo;
      // members starting inside the unit number at most kUnitArcs; one more
      // entry bounds the last one
      s_mcnt = static_cast<int32_t>(min(static_cast<int64_t>(m1 - lo), static_cast<int64_t>(kUnitArcs + 1)));
    }
    __syncthreads();
    const int32_t mlo = s_mlo, mcnt = s_mcnt;
    for (int t = threadIdx.x; t <= mcnt; t += kBlock)
      s_moff[t] = static_cast<int32_t>(min(mpre[mlo + t] - base - a_u, static_cast<int64_t>(kUnitArcs)));
    __syncthreads();
    // this thread's arcs: unit offsets [o0, o0 + A)
    const int32_t o0 = threadIdx.x * A;
    const int32_t olim = static_cast<int32_t>(min(static_cast<int64_t>(kUnitArcs), vol - a_u));
    int32_t mt[A];
#pragma unroll
    for (int q = 0; q < A; ++q) {
      const int32_t o = o0 + q;
      int32_t lo = 0, hi = mcnt - 1;  // last staged member with s_moff <= o
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_moff[mid] <= o) lo = mid;
        else hi = mid - 1;
      }
      mt[q] = lo;
    }
    // an arc is taken when its member's range holds it (members start at
    // most kUnitArcs times inside a unit unless some have no arcs, which a
    // community of more than one vertex never has)
    bool ok[A];
#pragma unroll
    for (int q = 0; q < A; ++q) {
      ok[q] = o0 + q < olim && o0 + q < s_moff[mt[q] + 1];
      if (o0 + q < olim && !ok[q]) set_error(ctr, LV_EINVAL);
    }
    int32_t cm[A];
#pragma unroll
    for (int q = 0; q < A; ++q) cm[q] = ok[q] ? cmem[mlo + mt[q]] : 0;
    int64_t pp[A];
#pragma unroll
    for (int q = 0; q < A; ++q) pp[q] = ok[q] ? row_start[cm[q]] + (o0 + q - s_moff[mt[q]]) : 0;
    int32_t js[A], xs[A];
#pragma unroll
    for (int q = 0; q < A; ++q) {
      js[q] = ok[q] ? col[pp[q]] : 0;
      xs[q] = ok[q] ? wt[pp[q]] : 0;
    }
    int32_t ds[A];
#pragma unroll
    for (int q = 0; q < A; ++q) ds[q] = ok[q] ? C[js[q]] : c;
    int64_t self = 0;
#pragma unroll
    for (int q = 0; q < A; ++q) {
      if (!ok[q]) continue;
      const int32_t d = ds[q], x = xs[q];
      if (d == c) {
        self += x;
        continue;
      }
      uint32_t h = mix32(static_cast<uint32_t>(d)) & (kUnitTS - 1);
      while (true) {  // at most kUnitArcs keys in kUnitTS = 2 kUnitArcs slots: ends
        const int32_t old = atomicCAS(&tk[h], -1, d);
        if (old == -1 || old == d) {
          atomicAdd(&tv[h], x);
          break;
        }
        h = (h + 1) & (kUnitTS - 1);
      }
    }
    self = wave_sum_i64(self);
    if (lane == 0) r_self[wid] = self;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t sum = 0;
      for (int q = 0; q < kBlock / kWave; ++q) sum += r_self[q];
      if (sum) table_add(tab, tsz, c, static_cast<int32_t>(sum));
    }
    // flush: the thread's table slots in rounds of compare-and-swaps
    constexpr int F = 8;
    for (int s0 = 0; s0 < kUnitTS; s0 += F * kBlock) {
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

// Compacts one unit of a big community's table into its row: one global
// atomic per unit reserves the row positions.
__global__ void __launch_bounds__(kBlock) k_big_emit(const int32_t* __restrict__ emit_b,
                                                    const int64_t* __restrict__ emit_s,
                                                    const int32_t* __restrict__ big, const int64_t* __restrict__ big_off,
                                                    const int64_t* __restrict__ out_start, const int64_t* __restrict__ ctr,
                                                    int32_t nc, const unsigned long long* __restrict__ tab,
                                                    int64_t pool_slots,
                                                    int32_t* __restrict__ out_len, int32_t* __restrict__ out_col,
                                                    int32_t* __restrict__ out_w, int64_t* __restrict__ Kout,
                                                    int64_t* __restrict__ Sout) {
  constexpr int kPer = kEmitSlots / kBlock;
  __shared__ int32_t s_cnt[kBlock / kWave];
  __shared__ int32_t s_base;
  __shared__ int64_t s_sum[kBlock / kWave];
  const int64_t count = ctr[CTR_UNITS_EMIT];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  for (int64_t u = blockIdx.x; u < count; u += gridDim.x) {
    const int32_t b = emit_b[u];
    const int32_t c = big[b];
    const int64_t tsz = big_slots(out_start[c + 1] - out_start[c], nc);
    const int64_t off = big_off[b];
    if (off + tsz > pool_slots) continue;
    // this thread's slots: emit_s[u] + threadIdx.x * kPer + [0, kPer)
    const int64_t s0 = emit_s[u] + static_cast<int64_t>(threadIdx.x) * kPer;
    int32_t d[kPer], x[kPer];
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t s = s0 + j;
      const unsigned long long e = s < tsz ? tab[off + s] : kEmptyPair;
      d[j] = static_cast<int32_t>(e >> 32);
      x[j] = static_cast<int32_t>(static_cast<uint32_t>(e));
      mine += d[j] >= 0 ? 1 : 0;
    }
    // exclusive scan of `mine` over the workgroup
    int32_t incl = mine;
    for (int q = 1; q < kWave; q <<= 1) {
      const int32_t o = __shfl_up(incl, q);
      if (lane >= q) incl += o;
    }
    if (lane == kWave - 1) s_cnt[wid] = incl;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int q = 0; q < kBlock / kWave; ++q) {
      if (q < wid) before += s_cnt[q];
      total += s_cnt[q];
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(&out_len[c], total) : 0;
    __syncthreads();
    int64_t p = out_start[c] + s_base + before + incl - mine;
    int64_t ksum = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
      if (d[j] >= 0) {
        out_col[p] = d[j];
        out_w[p] = x[j];
        ksum += x[j];
        ++p;
      }
    ksum = wave_sum_i64(ksum);
    if (lane == 0) s_sum[wid] = ksum;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int q = 0; q < kBlock / kWave; ++q) t += s_sum[q];
      if (t) {
        atomic_add_i64(&Kout[c], t);
        atomic_add_i64(&Sout[c], t);
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_merge_wave(
    const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len, const int32_t* __restrict__ col,
    const int32_t* __restrict__ wt, const int32_t* __restrict__ C, const int32_t* __restrict__ coff,
    const int32_t* __restrict__ cmem, const int32_t* __restrict__ list, const int64_t* __restrict__ ctr,
    const int64_t* __restrict__ out_start, int32_t* __restrict__ out_len, int32_t* __restrict__ out_col,
    int32_t* __restrict__ out_w, int64_t* __restrict__ Kout, int64_t* __restrict__ Sout) {
  __shared__ int32_t s_keys[kBlock / kWave][kAggWaveTS];
  __shared__ int32_t s_vals[kBlock / kWave][kAggWaveTS];
  const int64_t count = ctr[CTR_AGG_SMALL];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int32_t* keys = s_keys[wid];
  int32_t* vals = s_vals[wid];
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t idx = wave; idx < count; idx += nwaves) {
    const int32_t c = list[idx];
    const int32_t vol = static_cast<int32_t>(out_start[c + 1] - out_start[c]);
    const uint32_t ts = max(64u, 1u << (32 - __clz(static_cast<uint32_t>(2 * vol - 1))));
    for (uint32_t t = lane; t < ts; t += kWave) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t m0 = coff[c], m1 = coff[c + 1];
    int32_t self = 0;
    for (int32_t m = m0; m < m1; ++m) {
      const int32_t i = cmem[m];
      const int64_t s = row_start[i];
      const int32_t l = row_len[i];
      for (int32_t k = lane; k < l; k += kWave) {
        const int32_t d = C[col[s + k]];
        const int32_t x = wt[s + k];
        if (d == c) {
          self += x;
          continue;
        }
        uint32_t h = hash_slot(static_cast<uint32_t>(d), ts);
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, d);
          if (old == -1 || old == d) {
            atomicAdd(&vals[h], x);
            break;
          }
          h = (h + 1) & (ts - 1);
        }
      }
    }
    self = wave_sum_i32(self);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t base = out_start[c];
    int32_t written = 0;
    int64_t ksum = 0;
    if (self > 0) {  // the self-loop arc (c, c) first
      if (lane == 0) {
        out_col[base] = c;
        out_w[base] = self;
      }
      written = 1;
      ksum = lane == 0 ? self : 0;
    }
    for (uint32_t t0 = 0; t0 < ts; t0 += kWave) {
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

__global__ void __launch_bounds__(kBlock) k_merge_block(
    const int64_t* __restrict__ row_start, const int32_t* __restrict__ row_len, const int32_t* __restrict__ col,
    const int32_t* __restrict__ wt, const int32_t* __restrict__ C, const int32_t* __restrict__ coff,
    const int32_t* __restrict__ cmem, const int32_t* __restrict__ list, const int64_t* __restrict__ ctr,
    const int64_t* __restrict__ out_start, int32_t* __restrict__ out_len, int32_t* __restrict__ out_col,
    int32_t* __restrict__ out_w, int64_t* __restrict__ Kout, int64_t* __restrict__ Sout) {
  __shared__ int32_t keys[kAggBlockTS];
  __shared__ int32_t vals[kAggBlockTS];
  __shared__ int32_t s_cnt[kBlock / kWave];
  __shared__ int64_t s_sum[kBlock / kWave];
  const int64_t count = ctr[CTR_AGG_MEDIUM];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t c = list[idx];
    const int32_t vol = static_cast<int32_t>(out_start[c + 1] - out_start[c]);
    const uint32_t ts = max(static_cast<uint32_t>(kBlock), 1u << (32 - __clz(static_cast<uint32_t>(2 * vol - 1))));
    for (uint32_t t = threadIdx.x; t < ts; t += kBlock) {
      keys[t] = -1;
      vals[t] = 0;
    }
    __syncthreads();
    const int32_t m0 = coff[c], m1 = coff[c + 1];
    int32_t self = 0;
    for (int32_t m = m0; m < m1; ++m) {
      const int32_t i = cmem[m];
      const int64_t s = row_start[i];
      const int32_t l = row_len[i];
      for (int32_t k = threadIdx.x; k < l; k += kBlock) {
        const int32_t d = C[col[s + k]];
        const int32_t x = wt[s + k];
        if (d == c) {
          self += x;
          continue;
        }
        uint32_t h = hash_slot(static_cast<uint32_t>(d), ts);
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, d);
          if (old == -1 || old == d) {
            atomicAdd(&vals[h], x);
            break;
          }
          h = (h + 1) & (ts - 1);
        }
      }
    }
    self = wave_sum_i32(self);
    if (lane == 0) s_cnt[wid] = self;
    __syncthreads();
    int32_t selfsum = 0;
    for (int q = 0; q < kBlock / kWave; ++q) selfsum += s_cnt[q];
    __syncthreads();
    const int64_t base = out_start[c];
    int32_t written = selfsum > 0 ? 1 : 0;
    int64_t ksum = (threadIdx.x == 0) ? selfsum : 0;
    if (selfsum > 0 && threadIdx.x == 0) {
      out_col[base] = c;
      out_w[base] = selfsum;
    }
    for (uint32_t t0 = 0; t0 < ts; t0 += kBlock) {
      const uint32_t t = t0 + threadIdx.x;
      const int32_t d = keys[t];
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
        const int32_t x = vals[t];
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
  launch_accumulate(C, g.n, g.row_len, nullptr, ws.ccount, ws.vol, st);
  exclusive_scan_i32(ws.ccount, ws.coff, nc, ws, st);
  (void)hipMemsetAsync(ws.flags, 0, sizeof(int32_t) * (static_cast<size_t>(nc) + 1), st);
  launch_fill_members(C, g.n, ws.coff, ws.flags, ws.cmem, st);
}

void launch_aggregate(const LevelGraph& g, const int32_t* C, int32_t nc, LevelGraph& out, int64_t* Kout,
                      int64_t* Sout, int32_t* Cout, int32_t* sizeout, Workspace& ws, const lv_tuning& tu,
                      hipStream_t st) {
  launch_community_members(C, g, nc, ws, st);
  // super-vertex row offsets = exclusive scan of community volumes
  exclusive_scan_i64(ws.vol, out.row_start, nc, ws, st);
  // arc prefix over the members in community order (for big communities)
  hipLaunchKernelGGL(k_member_degrees, dim3(grid_for(g.n, kBlock, 8192)), dim3(kBlock), 0, st, ws.cmem, g.row_len,
                     g.n, ws.i64tmp);
  exclusive_scan_i64(ws.i64tmp, ws.vol, g.n, ws, st);
  out.n = nc;
  (void)hipMemsetAsync(ws.ctr + CTR_AGG_SMALL, 0, sizeof(int64_t) * 5 * kCtrLine, st);
  (void)hipMemsetAsync(ws.ctr + CTR_AGG_POOL, 0, sizeof(int64_t), st);
  hipLaunchKernelGGL(k_bin_communities, dim3(grid_for(nc, kBlock * kBinItems, 4096)), dim3(kBlock), 0, st,
                     out.row_start, nc,
                     ws.bins[0], ws.bins[1], ws.bins[2], ws.hub_off, out.row_len, Kout, Sout, ws.ctr);
  hipLaunchKernelGGL(k_merge_wave, dim3(tu.blocks_wave), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col,
                     g.w, C, ws.coff, ws.cmem, ws.bins[0], ws.ctr, out.row_start, out.row_len, out.col, out.w,
                     Kout, Sout);
  hipLaunchKernelGGL(k_merge_block, dim3(tu.blocks_hub), dim3(kBlock), 0, st, g.row_start, g.row_len, g.col,
                     g.w, C, ws.coff, ws.cmem, ws.bins[1], ws.ctr, out.row_start, out.row_len, out.col, out.w,
                     Kout, Sout);
  hipLaunchKernelGGL(k_big_units, dim3(64), dim3(kBlock), 0, st, ws.bins[2], out.row_start, nc, ws.u_ins_b,
                     ws.u_ins_a, ws.u_emit_b, ws.u_emit_s, ws.ctr);
  const int gb = 4 * tu.blocks_hub;
  hipLaunchKernelGGL(k_big_clear, dim3(gb), dim3(kBlock), 0, st, ws.u_emit_b, ws.u_emit_s, ws.bins[2], ws.hub_off,
                     out.row_start, ws.ctr, nc, reinterpret_cast<unsigned long long*>(ws.pool_pairs), ws.pool_slots);
  hipLaunchKernelGGL(k_big_insert, dim3(gb), dim3(kBlock), 0, st, g.row_start, g.col, g.w, C, ws.coff, ws.cmem,
                     ws.vol, ws.u_ins_b, ws.u_ins_a, ws.bins[2], ws.hub_off, out.row_start, ws.ctr, nc,
                     reinterpret_cast<unsigned long long*>(ws.pool_pairs), ws.pool_slots);
  hipLaunchKernelGGL(k_big_emit, dim3(gb), dim3(kBlock), 0, st, ws.u_emit_b, ws.u_emit_s, ws.bins[2], ws.hub_off,
                     out.row_start, ws.ctr, nc, reinterpret_cast<const unsigned long long*>(ws.pool_pairs),
                     ws.pool_slots, out.row_len, out.col, out.w, Kout, Sout);
  // the next level starts from singletons; written only after the merges,
  // which still read the current membership (the same array from pass 1 on)
  launch_iota_i32(Cout, nc, st);
  if (sizeout) launch_fill_i32(sizeout, 1, nc, st);
}

void launch_sigma_from_members(const int32_t* C, const int64_t* K, int32_t n, int64_t* Sigma, hipStream_t st) {
  (void)hipMemsetAsync(Sigma, 0, sizeof(int64_t) * static_cast<size_t>(n), st);
  launch_accumulate(C, n, nullptr, K, nullptr, Sigma, st);
}

}  // namespace lv
