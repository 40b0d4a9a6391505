// Device-wide exclusive prefix sum (three phases: tile sums, scan of the
// tile sums in one workgroup, tile scans with offsets).  Used for the CSR
// row offsets, community renumbering (Alg. 4) and the community-vertex and
// super-vertex offsets of aggregation (Alg. 6).  out[n] receives the total.
#include "lv_internal.hpp"

namespace lv {
namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;  // 2048 elements per workgroup

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* total, int64_t* lds) {
  // lds: kBlock / kWave entries
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  int64_t incl = v;
  for (int s = 1; s < kWave; s <<= 1) {
    int64_t o = __shfl_up(incl, s);
    if (lane >= s) incl += o;
  }
  if (lane == kWave - 1) lds[wid] = incl;
  __syncthreads();
  int64_t wbase = 0, tot = 0;
  for (int k = 0; k < kBlock / kWave; ++k) {
    const int64_t x = lds[k];
    if (k < wid) wbase += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return wbase + incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_tile_sums(const T* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ part) {
  __shared__ int64_t lds[kBlock / kWave];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  int64_t s = 0;
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * kBlock + threadIdx.x;
    if (i < n) s += static_cast<int64_t>(in[i]);
  }
  int64_t tot;
  block_exclusive_scan(s, &tot, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_parts(int64_t* __restrict__ part, int64_t nb) {
  __shared__ int64_t lds[kBlock / kWave];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nb ? part[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, &tot, lds);
    if (i < nb) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_tile_scan(const T* in, T* out,
                                                     int64_t n, const int64_t* __restrict__ part,
                                                     int64_t nb) {
  __shared__ int64_t lds[kBlock / kWave];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile + static_cast<int64_t>(threadIdx.x) * kItems;
  T vals[kItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    vals[k] = i < n ? in[i] : T(0);
    s += static_cast<int64_t>(vals[k]);
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(s, &tot, lds) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = static_cast<T>(run);
    run += static_cast<int64_t>(vals[k]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = static_cast<T>(part[nb]);
}

template <typename T>
void scan_impl(const T* in, T* out, int64_t n, Workspace& ws, hipStream_t st) {
  const int64_t nb = (n + kTile - 1) / kTile;
  if (nb == 0) {
    (void)hipMemsetAsync(out, 0, sizeof(T), st);
    return;
  }
  // nb + 1 <= ws.scan_part_len is guaranteed by the workspace layout
  hipLaunchKernelGGL(k_tile_sums<T>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, st, in, n,
                     ws.scan_part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, st, ws.scan_part, nb);
  hipLaunchKernelGGL(k_tile_scan<T>, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, st, in, out, n,
                     ws.scan_part, nb);
}

}  // namespace

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, Workspace& ws, hipStream_t st) {
  scan_impl<int32_t>(in, out, n, ws, st);
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, Workspace& ws, hipStream_t st) {
  scan_impl<int64_t>(in, out, n, ws, st);
}

int64_t scan_parts_needed(int64_t n) { return (n + kTile - 1) / kTile + 1; }

}  // namespace lv
