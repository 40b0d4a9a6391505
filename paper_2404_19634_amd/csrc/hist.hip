// Per-community accumulation over all vertices (community sizes, member
// counts and volumes, community totals Σ_c = Σ_{i in c} K_i, member lists).
// A community can hold a large share of the vertices, so plain per-vertex
// global atomics pile onto one address.  Each workgroup first accumulates
// its 4096 vertices in an LDS open-addressing table and then issues one
// global atomic per distinct community; keys that do not find a slot
// within a few probes go straight to global memory.
#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int kItems = 16;
constexpr int kPerBlock = kBlock * kItems;  // vertices per workgroup
constexpr int kTS = 2048;                   // LDS slots
constexpr int kProbes = 8;

// Returns the LDS slot holding `key` (inserting it) or -1 when the probe
// limit is hit.
__device__ __forceinline__ int lds_slot(int32_t* tk, int32_t key) {
  uint32_t h = hash_slot(static_cast<uint32_t>(key), kTS);
  for (int p = 0; p < kProbes; ++p) {
    const int32_t old = atomicCAS(&tk[h], -1, key);
    if (old == -1 || old == key) return static_cast<int>(h);
    h = (h + 1) & (kTS - 1);
  }
  return -1;
}

__device__ __forceinline__ int lds_find(const int32_t* tk, int32_t key) {
  uint32_t h = hash_slot(static_cast<uint32_t>(key), kTS);
  for (int p = 0; p < kProbes; ++p) {
    const int32_t k = tk[h];
    if (k == key) return static_cast<int>(h);
    if (k == -1) return -1;
    h = (h + 1) & (kTS - 1);
  }
  return -1;
}

// out_count[C[i]] += 1 (if out_count), out_val[C[i]] += val_i where val_i is
// v32[i] or v64[i] (if out_val)
__global__ void __launch_bounds__(kBlock) k_accumulate(const int32_t* __restrict__ C, int32_t n,
                                                      const int32_t* __restrict__ v32,
                                                      const int64_t* __restrict__ v64,
                                                      int32_t* __restrict__ out_count,
                                                      int64_t* __restrict__ out_val) {
  __shared__ int32_t tk[kTS];
  __shared__ int32_t tc[kTS];
  __shared__ int64_t tv[kTS];
  for (int s = threadIdx.x; s < kTS; s += kBlock) {
    tk[s] = -1;
    tc[s] = 0;
    tv[s] = 0;
  }
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kPerBlock;
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * kBlock + threadIdx.x;
    if (i >= n) break;
    const int32_t key = C[i];
    int64_t v = 0;
    if (out_val) v = v32 ? static_cast<int64_t>(v32[i]) : v64[i];
    const int h = lds_slot(tk, key);
    if (h >= 0) {
      if (out_count) atomicAdd(&tc[h], 1);
      if (out_val && v) atomicAdd(reinterpret_cast<unsigned long long*>(&tv[h]), static_cast<unsigned long long>(v));
    } else {
      if (out_count) atomicAdd(&out_count[key], 1);
      if (out_val && v) atomic_add_i64(&out_val[key], v);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kTS; s += kBlock) {
    const int32_t key = tk[s];
    if (key < 0) continue;
    if (out_count && tc[s]) atomicAdd(&out_count[key], tc[s]);
    if (out_val && tv[s]) atomic_add_i64(&out_val[key], tv[s]);
  }
}

// cmem[coff[C[i]] + slot] = i with slots handed out per community; the
// workgroup reserves one range per distinct community with a single
// global atomic on cursor[c] (zero on entry)
__global__ void __launch_bounds__(kBlock) k_fill(const int32_t* __restrict__ C, int32_t n,
                                                const int32_t* __restrict__ coff, int32_t* __restrict__ cursor,
                                                int32_t* __restrict__ cmem) {
  __shared__ int32_t tk[kTS];
  __shared__ int32_t tc[kTS];
  __shared__ int32_t tb[kTS];
  for (int s = threadIdx.x; s < kTS; s += kBlock) {
    tk[s] = -1;
    tc[s] = 0;
  }
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kPerBlock;
  uint32_t direct = 0;  // bit k: item k was placed with a global atomic
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * kBlock + threadIdx.x;
    if (i >= n) break;
    const int32_t key = C[i];
    const int h = lds_slot(tk, key);
    if (h >= 0) {
      atomicAdd(&tc[h], 1);
    } else {
      const int32_t pos = atomicAdd(&cursor[key], 1);
      cmem[coff[key] + pos] = static_cast<int32_t>(i);
      direct |= 1u << k;
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kTS; s += kBlock) {
    const int32_t key = tk[s];
    if (key >= 0 && tc[s]) tb[s] = atomicAdd(&cursor[key], tc[s]);
    tc[s] = 0;
  }
  __syncthreads();
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * kBlock + threadIdx.x;
    if (i >= n) break;
    if (direct & (1u << k)) continue;
    const int32_t key = C[i];
    const int h = lds_find(tk, key);  // present: inserted above
    const int32_t pos = tb[h] + atomicAdd(&tc[h], 1);
    cmem[coff[key] + pos] = static_cast<int32_t>(i);
  }
}

unsigned blocks_for(int32_t n) { return static_cast<unsigned>((static_cast<int64_t>(n) + kPerBlock - 1) / kPerBlock); }

}  // namespace

void launch_accumulate(const int32_t* C, int32_t n, const int32_t* v32, const int64_t* v64, int32_t* out_count,
                       int64_t* out_val, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_accumulate, dim3(blocks_for(n)), dim3(kBlock), 0, st, C, n, v32, v64, out_count, out_val);
}

void launch_fill_members(const int32_t* C, int32_t n, const int32_t* coff, int32_t* cursor, int32_t* cmem,
                         hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, st, C, n, coff, cursor, cmem);
}

}  // namespace lv
