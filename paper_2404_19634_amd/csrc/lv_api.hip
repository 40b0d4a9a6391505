// C interface and host controller.  The pass / iteration loop of the
// Louvain driver (Alg. 4) runs here: each local-moving iteration (Alg. 5) is
// a few kernels followed by one small readback of the iteration's counters
// (moves, gain sum, arcs scanned), from which the convergence test of the
// paper is taken exactly:
//   ΔQ_iteration = 2 * Σ gains / (2m)^2 <= τ   (FP64 on the host)
// Between passes the communities are renumbered, the dendrogram looked up
// and the level graph aggregated (Alg. 6); τ drops by the given factor.
#include <atomic>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "lv_internal.hpp"

namespace lv {
namespace {

thread_local std::string g_last_error;
lv_tuning g_tuning = {256, 2048, 2560, 1280, 7, 256, 2, 1 << 20, 1, 128};

lv_status fail(lv_status code, const char* msg) {
  g_last_error = msg;
  return code;
}

#define LV_HIP(expr)                                                         \
  do {                                                                       \
    hipError_t e__ = (expr);                                                 \
    if (e__ != hipSuccess) {                                                 \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(e__);     \
      return LV_EHIP;                                                        \
    }                                                                        \
  } while (0)

#define LV_CHECK_LAUNCH()                                                    \
  do {                                                                       \
    hipError_t e__ = hipGetLastError();                                      \
    if (e__ != hipSuccess) {                                                 \
      g_last_error = std::string("kernel launch: ") + hipGetErrorString(e__); \
      return LV_EHIP;                                                        \
    }                                                                        \
  } while (0)

// Set while a call of louvain_df_noalloc runs on this thread: counters are
// read back into plain host memory, and no HIP events are created or
// recorded (no timing), so the call allocates nothing.
thread_local bool g_no_alloc = false;
thread_local int64_t g_plain_host[CTR_COUNT + kCtrLine];

// Small pinned buffer for counter readback, one per host thread.
struct Pinned {
  int64_t* p = nullptr;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local Pinned g_pinned;

lv_status pinned(int64_t** out) {
  if (g_no_alloc) {
    *out = g_plain_host;
    return LV_OK;
  }
  if (!g_pinned.p) {
    void* q = nullptr;
    LV_HIP(hipHostMalloc(&q, sizeof(int64_t) * (CTR_COUNT + kCtrLine), hipHostMallocDefault));
    g_pinned.p = static_cast<int64_t*>(q);
  }
  *out = g_pinned.p;
  return LV_OK;
}

// ---- measurement hook (lv_set_timing) ------------------------------------
std::atomic<uint32_t> g_timed_mask{0};
constexpr int kTimerPairs = 4096;
struct Timer {
  std::vector<hipEvent_t> ev;   // 2 per launch, created on first use
  std::vector<int> kernel;      // kernel of each recorded pair
  int used = 0;                 // pairs handed out since the last collect
  ~Timer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};
thread_local Timer g_timer;

}  // namespace

TimerPair timer_pair(int kernel) {
  TimerPair p;
  if (g_no_alloc || !((g_timed_mask.load(std::memory_order_relaxed) >> kernel) & 1u)) return p;
  Timer& t = g_timer;
  if (t.used >= kTimerPairs) return p;
  while (static_cast<int>(t.ev.size()) < 2 * (t.used + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return p;
    t.ev.push_back(e);
  }
  if (static_cast<int>(t.kernel.size()) < t.used + 1) t.kernel.resize(t.used + 1);
  p.start = t.ev[2 * t.used];
  p.stop = t.ev[2 * t.used + 1];
  t.kernel[t.used++] = kernel;
  return p;
}

void timer_collect(int32_t* launches, double* ms) {
  Timer& t = g_timer;
  for (int k = 0; k < t.used; ++k) {
    float x = 0.f;
    if (hipEventElapsedTime(&x, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess) {
      launches[t.kernel[k]] += 1;
      ms[t.kernel[k]] += x;
    }
  }
  t.used = 0;
}

namespace {

// Timing events, one set per host thread.
struct Events {
  hipEvent_t e[8] = {};
  bool made = false;
  ~Events() {
    if (made)
      for (auto& x : e) (void)hipEventDestroy(x);
  }
};
thread_local Events g_events;

lv_status events(hipEvent_t** out) {
  if (g_no_alloc) {
    *out = nullptr;
    return LV_OK;
  }
  if (!g_events.made) {
    for (auto& x : g_events.e) LV_HIP(hipEventCreate(&x));
    g_events.made = true;
  }
  *out = g_events.e;
  return LV_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

template <class T>
T* take(char*& cur, size_t& total, void* base, size_t count) {
  T* p = base ? reinterpret_cast<T*>(cur) : nullptr;
  const size_t b = align_up(sizeof(T) * (count ? count : 1));
  cur += b;
  total += b;
  return p;
}

lv_status read_counters(int64_t* host, const Workspace& ws, int count, hipStream_t st) {
  LV_HIP(hipMemcpyAsync(host, ws.ctr, sizeof(int64_t) * count, hipMemcpyDeviceToHost, st));
  LV_HIP(hipStreamSynchronize(st));
  return LV_OK;
}

// A per-iteration statistic of one set, summed over its replicas.
int64_t stat(const int64_t* set, int st) {
  int64_t v = 0;
  for (int r = 0; r < kStatReplicas; ++r) v += set[r * kStatStride + st];
  return v;
}

lv_status device_error(int64_t code, const char* phase) {
  if (code == LV_EEMPTY) return fail(LV_EEMPTY, "graph has no edges (2m = 0)");
  if (code == LV_EOVERFLOW) return fail(LV_EOVERFLOW, "total arc weight 2m >= 2^31");
  if (code == LV_EINVAL)
    return fail(LV_EINVAL, "the batch names a vertex outside [0, n) or a self-loop (not the batch apply_batch "
                           "took); such updates were skipped and the state is unspecified");
  static thread_local char msg[96];
  std::snprintf(msg, sizeof(msg), "device error in %s", phase);
  return fail(static_cast<lv_status>(code), msg);
}

// Errors of a batch edit (Section 3.4's update refused as a whole), or of
// the first kernel of the call that follows it.
lv_status batch_error(int64_t code) {
  switch (code) {
    case LV_ENOEDGE: return fail(LV_ENOEDGE, "a deletion names a missing edge or too much weight");
    case LV_ENOSLACK: return fail(LV_ENOSLACK, "a row lacks free capacity (relayout with more slack)");
    case LV_EOVERFLOW: return fail(LV_EOVERFLOW, "total arc weight would reach 2^31");
    case LV_EINVAL: return fail(LV_EINVAL, "bad id, self-loop, non-positive weight or repeated pair");
    default: return device_error(code, "batch edit");
  }
}

lv_status read_i64(int64_t* host, const int64_t* dev, hipStream_t st) {
  LV_HIP(hipMemcpyAsync(host, dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LV_HIP(hipStreamSynchronize(st));
  return LV_OK;
}

bool params_ok(const lv_params* p) {
  return p && p->max_iterations >= 1 && p->max_iterations <= LV_MAX_ITERS && p->max_passes >= 1 &&
         p->max_passes <= LV_MAX_PASSES && (p->mode == LV_SYNC || p->mode == LV_ASYNC) &&
         p->tolerance >= 0.0 && p->tolerance_drop > 0.0 && p->aggregation_tolerance >= 0.0 &&
         (p->recompute_weights == 0 || p->recompute_weights == 1) && p->reserved == 0;
}

bool graph_ok(const lv_graph* g) {
  return g && g->n > 0 && g->row_start && g->row_len && g->col && g->w && g->two_m && g->cap >= 0;
}

bool edges_ok(const lv_edges* e) { return e && e->count >= 0 && (e->count == 0 || (e->u && e->v && e->w)); }

lv_status setup_ws(Workspace& ws, const lv_graph* g, void* base, size_t bytes) {
  if (!base) return fail(LV_EINVAL, "workspace pointer is null");
  const size_t need = carve_workspace(ws, nullptr, g->n, g->cap);
  if (bytes < need) return fail(LV_EWORKSPACE, "workspace smaller than lv_workspace_bytes()");
  carve_workspace(ws, base, g->n, g->cap);
  return LV_OK;
}

}  // namespace

lv_status lv_fail(lv_status code, const char* msg) { return fail(code, msg); }

namespace {

lv_tuning effective_tuning() {
  lv_tuning t = g_tuning;
  if (t.wave_max_degree <= 0) t.wave_max_degree = 256;
  if (t.wave_max_degree < 32) t.wave_max_degree = 32;
  if (t.wave_max_degree > kWaveTableMaxDegree) t.wave_max_degree = kWaveTableMaxDegree;
  if (t.blocks_small <= 0) t.blocks_small = 2048;
  if (t.blocks_wave <= 0) t.blocks_wave = 2560;
  if (t.blocks_hub <= 0) t.blocks_hub = 1280;
  if (t.async_rounds_log2 < 0) t.async_rounds_log2 = 0;
  if (t.async_rounds_log2 > 7) t.async_rounds_log2 = 7;
  if (t.async_round_order < 0 || t.async_round_order > 2) t.async_round_order = 0;
  if (t.async_rounds_min_frontier < 0) t.async_rounds_min_frontier = 0;
  if (t.fuse_max_frontier < -1) t.fuse_max_frontier = -1;
  t.defer_totals = t.defer_totals ? 1 : 0;
  if (t.revisit_min_degree < 0) t.revisit_min_degree = 0;
  return t;
}

}  // namespace

lv_tuning lv_effective_tuning() { return effective_tuning(); }

namespace {

enum Approach { A_STATIC, A_ND, A_DS, A_DF };

// The sub-rounds of one ASYNC iteration.  Splitting the frontier lets a
// vertex see most of its neighbours' moves (the paper's loop is nearly
// sequential per thread); SYNC and small frontiers run one round.
//  - level 0 (the input graph), order 2: four degree classes, highest
//    first, each hashed into 2^(k-2) rounds, so hubs settle before the many
//    low-degree vertices that hang off them;
//  - order 0 / 1: 2^k rounds by id hash / by contiguous id ranges;
//  - super-vertex levels (dense): 2^min(k, 4) rounds by id hash.
// Aggregated levels up to this many vertices take the full 2^k ASYNC rounds,
// each in one fused launch.
constexpr int32_t kSmallLevel = 4096;

std::vector<SubRound> sub_rounds(int32_t mode, int32_t pass, int64_t est_frontier, int32_t n, const lv_tuning& tu) {
  std::vector<SubRound> out;
  SubRound all;
  all.id_hi = n;
  const bool split = mode == LV_ASYNC && (pass > 0 || est_frontier > tu.async_rounds_min_frontier);
  if (!split || tu.async_rounds_log2 <= 0) {
    out.push_back(all);
    return out;
  }
  // conflicts scale with the frontier's density: a sparse frontier (small
  // DF batches) has few adjacent members, so it gets proportionally fewer
  // rounds (2^k for a full sweep)
  int k = tu.async_rounds_log2;
  const double density = n > 0 ? static_cast<double>(std::min<int64_t>(est_frontier, n)) / n : 1.0;
  while (k > 0 && static_cast<double>(int64_t(1) << tu.async_rounds_log2) * density < static_cast<double>(int64_t(1) << k))
    --k;
  if (k <= 0) {
    out.push_back(all);
    return out;
  }
  if (pass > 0 || tu.async_round_order == 0 || (tu.async_round_order == 2 && k < 2)) {
    // aggregated levels: 16 rounds, or 2^k when the level is small (its
    // super-vertices are densely linked, and few per round keep a move from
    // acting on totals that a neighbour's move in the same round changed)
    const int kk = pass > 0 ? (n <= kSmallLevel ? k : std::min(k, 4)) : k;
    for (int r = 0; r < (1 << kk); ++r) {
      SubRound s = all;
      s.hash_round = static_cast<uint32_t>(r);
      s.hash_shift = 32u - static_cast<uint32_t>(kk);
      out.push_back(s);
    }
  } else if (tu.async_round_order == 1) {
    const int64_t R = int64_t(1) << k;
    for (int64_t r = 0; r < R; ++r) {
      SubRound s = all;
      s.id_lo = static_cast<int32_t>(n * r / R);
      s.id_hi = static_cast<int32_t>(n * (r + 1) / R);
      out.push_back(s);
    }
  } else {
    static const int32_t cls_lo[4] = {1025, 129, 17, 0};
    static const int32_t cls_hi[4] = {0x7fffffff, 1024, 128, 16};
    const int kh = k - 2;
    for (int c = 0; c < 4; ++c) {
      // classes of long rows are visited twice: hubs that chose on the same
      // snapshot often picked communities their neighbours were leaving,
      // and the second visit lets them follow
      const int visits = (tu.revisit_min_degree > 0 && cls_lo[c] > tu.revisit_min_degree) ? 2 : 1;
      for (int v = 0; v < visits; ++v)
        for (int r = 0; r < (1 << kh); ++r) {
          SubRound s = all;
          s.deg_lo = cls_lo[c];
          s.deg_hi = cls_hi[c];
          if (kh > 0) {
            s.hash_round = static_cast<uint32_t>(r);
            s.hash_shift = 32u - static_cast<uint32_t>(kh);
          }
          out.push_back(s);
        }
    }
  }
  return out;
}

}  // namespace

std::vector<SubRound> lv_sub_rounds(int32_t mode, int32_t pass, int64_t est_frontier, int32_t n,
                                    const lv_tuning& tu) {
  return sub_rounds(mode, pass, est_frontier, n, tu);
}

namespace {

struct DsTables {
  uint64_t* keys;
  int64_t* vals;
  uint32_t size;
  uint64_t* skeys;
  int64_t* sbest;
  int32_t* sbestc;
  uint32_t ssize;
};

uint32_t pow2_at_least(int64_t x) {
  uint32_t s = 16;
  while (static_cast<int64_t>(s) < x) s <<= 1;
  return s;
}

// Carves the DS tables out of the global-table pool.
bool carve_ds(const Workspace& ws, int64_t ni, DsTables& t) {
  t.size = pow2_at_least(4 * ni);
  t.ssize = pow2_at_least(4 * ni);
  const size_t need = align_up(8ull * t.size) * 2 + align_up(8ull * t.ssize) * 2 + align_up(4ull * t.ssize);
  if (need > static_cast<size_t>(ws.pool_slots) * 4) return false;
  char* p = reinterpret_cast<char*>(ws.pool_keys);
  t.keys = reinterpret_cast<uint64_t*>(p);
  p += align_up(8ull * t.size);
  t.vals = reinterpret_cast<int64_t*>(p);
  p += align_up(8ull * t.size);
  t.skeys = reinterpret_cast<uint64_t*>(p);
  p += align_up(8ull * t.ssize);
  t.sbest = reinterpret_cast<int64_t*>(p);
  p += align_up(8ull * t.ssize);
  t.sbestc = reinterpret_cast<int32_t*>(p);
  return true;
}

__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Records event k of `ev` (none when ev is null: no timing).
hipError_t record(hipEvent_t* ev, int k, hipStream_t st) { return ev ? hipEventRecord(ev[k], st) : hipSuccess; }

float ms_between(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

float ms_between(hipEvent_t* ev, int a, int b) {
  if (!ev) return 0.f;
  return ms_between(ev[a], ev[b]);
}

// resume_li > 0: the local-moving iterations of pass 0 already ran (the
// batched kernel did them, with that l_i); the call goes on from the end of
// pass 0 with the state as it is (Alg. 4: renumber, aggregate, passes >= 1).
// after_batch: a batch edit of the same batch was enqueued just before on
// the stream, unread; its error (if any) is reported by this call.
lv_status run_louvain(Approach ap, const lv_graph* g, const lv_edges* del, const lv_edges* ins,
                      const lv_params* p, lv_state* state, void* wsp, size_t ws_bytes, lv_stats* stats,
                      void* stream, int32_t resume_li = 0, bool after_batch = false) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!graph_ok(g)) return fail(LV_EINVAL, "invalid graph");
  if (!params_ok(p)) return fail(LV_EINVAL, "invalid parameters");
  if (!state || !state->C || !state->K || !state->Sigma) return fail(LV_EINVAL, "invalid state");
  if (ap != A_STATIC && (!edges_ok(del) || !edges_ok(ins))) return fail(LV_EINVAL, "invalid batch");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace ws;
  lv_status s = setup_ws(ws, g, wsp, ws_bytes);
  if (s) return s;
  const lv_tuning tu = effective_tuning();
  int64_t* host = nullptr;
  if ((s = pinned(&host))) return s;
  hipEvent_t* ev = nullptr;
  if ((s = events(&ev))) return s;

  lv_stats local;
  lv_stats& S = stats ? *stats : local;
  std::memset(&S, 0, sizeof(lv_stats));

  const int32_t N = g->n;
  const lv_edges no_edges = {nullptr, nullptr, nullptr, 0};
  const lv_edges& D = del ? *del : no_edges;
  const lv_edges& I = ins ? *ins : no_edges;

  // The first kernel zeroes counters and frontier bitmasks and checks
  // 0 < 2m < 2^31 on the device; with 2m out of range every later kernel
  // leaves the state alone and the first readback reports the error.
  LV_HIP(record(ev, 0, st));
  // fr_a's list is kept for DF's marking (and a resumed pass); the other
  // approaches fill the bitmask whole
  const bool dense_start = resume_li == 0 && ap != A_DF;
  launch_call_begin(ws, g->two_m, dense_start, after_batch, st);
  LevelGraph L0;
  L0.n = N;
  L0.row_start = g->row_start;
  L0.row_len = g->row_len;
  L0.col = g->col;
  L0.w = g->w;
  bool use_range = false;
  // member counts of level-0 communities: the caller's carried array when
  // given (kept exact by the moves), else counted here for the swap guard
  int32_t* size0 = state->size ? state->size : (p->swap_guard ? ws.size : nullptr);
  if (resume_li > 0) {
    // nothing to mark: pass 0's moves are done
  } else if (ap == A_STATIC) {
    launch_row_sums(L0, nullptr, state->K, state->Sigma, state->C, size0 ? size0 : ws.size, ws,
                    st);
    launch_set_all_bits(ws.fr_a, N, st);
  } else {
    uint32_t* df_frontier = nullptr;
    switch (ap) {
      case A_DF:
        df_frontier = ws.fr_a;  // marked by the updateWeights pass
        break;
      case A_ND:
        launch_set_all_bits(ws.fr_a, N, st);
        break;
      case A_DS: {
        DsTables t;
        if (!carve_ds(ws, I.count, t)) return fail(LV_EWORKSPACE, "batch too large for the workspace pool");
        LV_HIP(hipMemsetAsync(ws.range, 0, sizeof(uint32_t) * ws.words, st));
        LV_HIP(hipMemsetAsync(ws.dE, 0, sizeof(uint32_t) * ws.words, st));
        LV_HIP(hipMemsetAsync(ws.dC, 0, sizeof(uint32_t) * ws.words, st));
        LV_HIP(hipMemsetAsync(t.keys, 0xFF, 8ull * t.size, st));
        LV_HIP(hipMemsetAsync(t.vals, 0, 8ull * t.size, st));
        LV_HIP(hipMemsetAsync(t.skeys, 0xFF, 8ull * t.ssize, st));
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(t.ssize, kBlock, 1024)), dim3(kBlock), 0, st, t.sbest,
                           static_cast<int64_t>(INT64_MIN), static_cast<int64_t>(t.ssize));
        launch_fill_i32(t.sbestc, 0x7fffffff, t.ssize, st);
        launch_batch_weight_sums(D, I, ws.ctr, st);
        launch_ds_deletions(D, N, state->C, ws.range, ws.dE, ws.dC, ws.ctr, st);
        launch_ds_insert_pairs(I, N, state->C, t.keys, t.vals, t.size, ws.ctr, st);
        launch_ds_best(t.keys, t.vals, t.size, state->K, state->Sigma, g->two_m, ws.ctr, t.skeys, t.sbest,
                       t.sbestc, t.ssize, 0, st);
        launch_ds_best(t.keys, t.vals, t.size, state->K, state->Sigma, g->two_m, ws.ctr, t.skeys, t.sbest,
                       t.sbestc, t.ssize, 1, st);
        launch_ds_mark_sources(t.skeys, t.sbestc, t.ssize, ws.range, ws.dE, ws.dC, st);
        launch_ds_expand(L0, D, I, state->C, ws.dE, ws.dC, ws.range, st);
        launch_copy_bits(ws.range, ws.fr_a, ws.words, st);
        use_range = true;
        break;
      }
      default:
        break;
    }
    launch_update_weights(D, I, N, state->C, state->K, state->Sigma, df_frontier, front_list(ws, 0), ws.ctr, st);
    if (p->recompute_weights) {
      // without auxiliary information (Section 4.2): K^t from the rows of
      // G^t and Sigma^t from C^{t-1}, replacing the incremental values
      launch_row_sums(L0, nullptr, state->K, nullptr, nullptr, nullptr, ws, st);
      launch_sigma_from_members(state->C, state->K, N, state->Sigma, st);
    }
    if (p->swap_guard && !state->size) launch_community_sizes(state->C, N, ws.size, st);
  }
  LV_CHECK_LAUNCH();
  LV_HIP(record(ev, 1, st));

  // ---- Alg. 4: passes of local-moving and aggregation --------------------
  LevelGraph L = L0;
  int32_t* Cl = state->C;
  int64_t* Kl = state->K;
  int64_t* Sl = state->Sigma;
  int32_t* size = size0;
  uint32_t* cur = ws.fr_a;
  uint32_t* next = ws.fr_b;
  FrontList cur_fl = front_list(ws, 0), next_fl = front_list(ws, 1);
  double tau = p->tolerance;
  bool aggregated = false;
  bool moved_dirty = false;  // cleared by the first kernel, then by the SYNC apply unless pulled
  int64_t iter_seq = 0, round_seq = 0;  // select the alternating counter sets
  int64_t two_m = 0;
  float ms_move = 0.f, ms_agg = 0.f;
  int64_t arcs_agg = 0;
  for (int32_t pass = 0; pass < p->max_passes; ++pass) {
    LV_HIP(record(ev, 2, st));
    int32_t li = p->max_iterations;
    MoveArgs a;
    a.g = L;
    a.C = Cl;
    a.K = Kl;
    a.Sigma = Sl;
    a.size = size;
    a.range = (pass == 0 && use_range) ? ws.range : nullptr;
    a.ever = pass == 0 ? ws.ever : nullptr;
    a.two_m = g->two_m;
    a.mode = p->mode;
    a.guard = p->swap_guard;
    a.wave_max = tu.wave_max_degree;
    const int64_t words_l = (static_cast<int64_t>(L.n) + 31) / 32;
    // upper bound of the frontier size, for the choice of sub-rounds
    int64_t est_frontier = L.n;
    if (pass == 0 && ap == A_DF) est_frontier = 2 * (D.count + I.count);
    if (pass == 0 && resume_li > 0) {
      li = resume_li;
      LV_HIP(record(ev, 3, st));
    }
    for (int32_t it = 0; it < p->max_iterations && !(pass == 0 && resume_li > 0); ++it, ++iter_seq) {
      a.cur = cur;
      a.next = next;
      a.cur_fl = cur_fl;
      a.next_fl = next_fl;
      // large frontiers pull the next frontier (reads) instead of pushing it
      // (one atomic per arc of every mover)
      const bool pull = est_frontier > L.n / 4;
      a.push = pull ? 0 : 1;
      a.moved = (pull || p->mode == LV_SYNC) ? ws.moved : nullptr;
      if (a.moved && moved_dirty) {
        LV_HIP(hipMemsetAsync(ws.moved, 0, sizeof(uint32_t) * words_l, st));
        moved_dirty = false;
      }
      int64_t* sc = ws.ctr + CTR_STATS0 + (iter_seq & 1) * kStatSet;
      int64_t* sc_next = ws.ctr + CTR_STATS0 + ((iter_seq + 1) & 1) * kStatSet;
      const std::vector<SubRound> plan = sub_rounds(p->mode, pass, est_frontier, L.n, tu);
      // a sub-round holds at most about 4 / rounds of the frontier (four
      // degree classes); grids are sized for that
      a.est = std::max<int64_t>(64, est_frontier * 4 / static_cast<int64_t>(plan.size()));
      a.sparse = (est_frontier * 8 <= L.n || (pass > 0 && L.n <= kSmallLevel)) ? 1 : 0;
      for (size_t r = 0; r < plan.size(); ++r, ++round_seq) {
        a.rc = ws.ctr + CTR_ROUND0 + (round_seq & 1) * kRoundSet;
        a.rc_next = ws.ctr + CTR_ROUND0 + ((round_seq + 1) & 1) * kRoundSet;
        a.sc = sc;
        a.sc_next = r == 0 ? sc_next : nullptr;
        a.clear_cur = r + 1 == plan.size() ? 1 : 0;
        const uint32_t mask = bins_for_degrees(plan[r].deg_lo, plan[r].deg_hi, a.wave_max);
        launch_round(a, ws, tu, plan[r], mask, st);
        for (int b = 0; b < NBINS; ++b) S.bin_launches[b] += (mask >> b) & 1u;
      }
      if (p->mode == LV_SYNC) launch_apply_moves(a, ws, !pull, st);
      if (pull) {
        launch_pull_expand(a, ws, st);
        moved_dirty = true;
      }
      LV_CHECK_LAUNCH();
      std::swap(cur, next);
      std::swap(cur_fl, next_fl);
      LV_HIP(record(ev, 3, st));
      if ((s = read_counters(host, ws, CTR_ROUND0, st))) return s;
      if (host[CTR_ERR])
        return after_batch ? batch_error(host[CTR_ERR]) : device_error(host[CTR_ERR], "local-moving");
      two_m = host[CTR_TWO_M];
      const int64_t* hs = host + CTR_STATS0 + (iter_seq & 1) * kStatSet;
      const int64_t movers = stat(hs, ST_MOVERS), gain = stat(hs, ST_GAIN);
      est_frontier = stat(hs, ST_EXPAND);
      S.moves += movers;
      S.arcs_scanned += stat(hs, ST_ARCS);
      S.vertices_affected += stat(hs, ST_AFFECTED);
      for (int b = 0; b < NBINS; ++b) {
        S.bin_vertices[b] += stat(hs, ST_BIN_V0 + b);
        S.bin_arcs[b] += stat(hs, ST_BIN_A0 + b);
      }
      if (pass < LV_MAX_PASSES && it < LV_MAX_ITERS) {
        S.iter_moves[pass][it] = movers;
        S.iter_gain[pass][it] = gain;
      }
      const double two_m_d = static_cast<double>(two_m);
      const double dq = (2.0 * static_cast<double>(gain)) / (two_m_d * two_m_d);
      if (dq <= tau) {
        li = it + 1;
        ++iter_seq;
        break;
      }
    }
    ms_move += ms_between(ev, 2, 3);
    S.passes = pass + 1;
    S.iterations[pass] = li;
    if (li <= 1) break;
    // renumber communities of this level (ascending old id)
    LV_HIP(hipMemsetAsync(ws.flags, 0, sizeof(int32_t) * (static_cast<size_t>(L.n) + 1), st));
    launch_mark_exists(Cl, L.n, ws.flags, st);
    exclusive_scan_i32(ws.flags, ws.newid, L.n, ws, st);
    LV_CHECK_LAUNCH();
    int32_t nc32 = 0;
    LV_HIP(hipMemcpyAsync(&host[CTR_TOTAL], ws.newid + L.n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LV_HIP(hipStreamSynchronize(st));
    std::memcpy(&nc32, &host[CTR_TOTAL], sizeof(int32_t));
    const int32_t nc = nc32;
    S.communities[pass] = nc;
    if (static_cast<double>(nc) / static_cast<double>(L.n) > p->aggregation_tolerance) break;
    LV_HIP(record(ev, 4, st));
    launch_relabel(Cl, L.n, ws.newid, st);
    if (pass > 0) launch_lookup(state->C, N, Cl, st);
    LevelGraph out = ws.lg[pass & 1];
    launch_aggregate(L, Cl, nc, out, ws.lK, ws.lS, ws.lC, ws.size, ws, tu, st);
    LV_CHECK_LAUNCH();
    LV_HIP(hipMemsetAsync(cur, 0, sizeof(uint32_t) * ws.words, st));
    launch_set_all_bits(cur, nc, st);
    launch_list_invalid(cur_fl, st);
    LV_HIP(record(ev, 5, st));
    LV_HIP(hipMemcpyAsync(&host[CTR_COUNT], out.row_start + nc, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if ((s = read_counters(host, ws, CTR_STATS0, st))) return s;
    if (host[CTR_ERR]) return device_error(host[CTR_ERR], "aggregation");
    ms_agg += ms_between(ev, 4, 5);
    arcs_agg += host[CTR_COUNT];
    L = out;
    Cl = ws.lC;
    Kl = ws.lK;
    Sl = ws.lS;
    size = p->swap_guard ? ws.size : nullptr;
    tau = tau / p->tolerance_drop;
    aggregated = true;
  }
  if (aggregated) {
    LV_HIP(record(ev, 6, st));
    launch_lookup(state->C, N, Cl, st);
    launch_sigma_from_members(state->C, state->K, N, state->Sigma, st);
    if (state->size) launch_community_sizes(state->C, N, state->size, st);
    LV_CHECK_LAUNCH();
    LV_HIP(record(ev, 7, st));
    LV_HIP(hipStreamSynchronize(st));
    S.ms_other = ms_between(ev, 6, 7);
  }
  timer_collect(S.timed_launches, S.timed_ms);
  S.ms_mark = ms_between(ev, 0, 1);
  S.ms_move = ms_move;
  S.ms_aggregate = ms_agg;
  S.arcs_aggregated = arcs_agg;
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return LV_OK;
}

}  // namespace

size_t carve_workspace(Workspace& ws, void* base, int32_t n, int64_t cap) {
  char* cur = static_cast<char*>(base);
  size_t total = 0;
  const size_t un = static_cast<size_t>(n > 0 ? n : 1);
  const size_t ucap = static_cast<size_t>(cap > 0 ? cap : 1);
  ws.n = n;
  ws.cap = cap;
  ws.words = (static_cast<int64_t>(un) + 31) / 32 + 1;
  ws.fr_a = take<uint32_t>(cur, total, base, ws.words);
  ws.fr_b = take<uint32_t>(cur, total, base, ws.words);
  ws.ever = take<uint32_t>(cur, total, base, ws.words);
  ws.range = take<uint32_t>(cur, total, base, ws.words);
  ws.dE = take<uint32_t>(cur, total, base, ws.words);
  ws.dC = take<uint32_t>(cur, total, base, ws.words);
  ws.moved = take<uint32_t>(cur, total, base, ws.words);
  ws.push_flags = take<uint8_t>(cur, total, base, static_cast<size_t>(ws.words) * 32);
  // frontier lists: regions of n/16 (twice an even share), so a region
  // overflows only when its writers append far more than their share
  ws.fl_capr = static_cast<int64_t>(un) / 16 + 64;
  for (int k = 0; k < 2; ++k)
    ws.fl[k] = take<int32_t>(cur, total, base, static_cast<size_t>(ws.fl_capr) * kFlRegions);
  for (int b = 0; b < NBINS; ++b) ws.bins[b] = take<int32_t>(cur, total, base, un + kRowListPad);
  ws.hub_off = take<int64_t>(cur, total, base, un);
  ws.hub_kid = take<int64_t>(cur, total, base, un);
  ws.hub_moved = take<int32_t>(cur, total, base, un);
  ws.hub_cbase = take<int64_t>(cur, total, base, un);
  ws.hub_cnum = take<int32_t>(cur, total, base, un);
  ws.mv_c = take<int32_t>(cur, total, base, un);
  ws.size = take<int32_t>(cur, total, base, un);
  ws.lC = take<int32_t>(cur, total, base, un);
  ws.lK = take<int64_t>(cur, total, base, un);
  ws.lS = take<int64_t>(cur, total, base, un);
  ws.flags = take<int32_t>(cur, total, base, un + 1);
  ws.newid = take<int32_t>(cur, total, base, un + 1);
  ws.ccount = take<int32_t>(cur, total, base, un + 1);
  ws.coff = take<int32_t>(cur, total, base, un + 1);
  ws.cmem = take<int32_t>(cur, total, base, un);
  ws.vol = take<int64_t>(cur, total, base, un + 1);
  ws.i64tmp = take<int64_t>(cur, total, base, un + 1);
  for (int k = 0; k < 2; ++k) {
    ws.lg[k].n = 0;
    ws.lg[k].row_start = take<int64_t>(cur, total, base, un + 1);
    ws.lg[k].row_len = take<int32_t>(cur, total, base, un);
    ws.lg[k].col = take<int32_t>(cur, total, base, ucap);
    ws.lg[k].w = take<int32_t>(cur, total, base, ucap);
  }
  ws.units_max = static_cast<int64_t>(un) + static_cast<int64_t>(ucap) / 2048 + 64;
  ws.u_ins_b = take<int32_t>(cur, total, base, static_cast<size_t>(ws.units_max));
  ws.u_ins_a = take<int64_t>(cur, total, base, static_cast<size_t>(ws.units_max));
  ws.u_emit_b = take<int32_t>(cur, total, base, static_cast<size_t>(ws.units_max));
  ws.u_emit_s = take<int64_t>(cur, total, base, static_cast<size_t>(ws.units_max));
  ws.unit_g = take<int64_t>(cur, total, base, static_cast<size_t>(ws.units_max));
  ws.unit_c = take<int32_t>(cur, total, base, static_cast<size_t>(ws.units_max));
  // hub tables take 2 slots per arc; rows that aggregate by segment add
  // their segment offsets: at most d/8 + d/1365 + 2 slots for a row of d
  // arcs (d <= 2^20 > 2048), so under cap/8 + cap/512 in all
  ws.pool_slots = 2 * static_cast<int64_t>(ucap) + static_cast<int64_t>(ucap) / 8 +
                  static_cast<int64_t>(ucap) / 512 + 4096;
  ws.pool_pairs = take<uint64_t>(cur, total, base, static_cast<size_t>(ws.pool_slots));
  ws.pool_keys = reinterpret_cast<int32_t*>(ws.pool_pairs);
  ws.pool_vals = base ? ws.pool_keys + ws.pool_slots : nullptr;
  ws.hot = take<HotRec>(cur, total, base, static_cast<size_t>(kHotRegions * kHotCap));
  ws.scan_part_len = scan_parts_needed(static_cast<int64_t>(un) + 2) + 8;
  ws.scan_part = take<int64_t>(cur, total, base, static_cast<size_t>(ws.scan_part_len));
  ws.ctr = take<int64_t>(cur, total, base, CTR_COUNT);
  ws.bytes = total;
  return total;
}

// Batched launches are replayed from captured graphs: copy of the
// descriptors in, the persistent kernel, copy of the results out.  The
// kernel reads the item count from the descriptor header, so one graph
// serves every count up to its size bucket (a power of two); graphs are
// kept per host thread, keyed by descriptor buffer, bucket and parameters,
// and copy through one pinned host buffer of that thread.
struct ManyGraph {
  void* desc = nullptr;
  int32_t bucket = 0;
  lv_params p{};
  lv_many_tuning t{};
  char* host = nullptr;  // the thread's pinned staging buffer
  hipGraphExec_t exec = nullptr;
};

struct ManyGraphs {
  std::vector<ManyGraph> g;
  char* host = nullptr;
  size_t host_bytes = 0;
  hipStream_t cap = nullptr;
  void drop() {
    for (auto& x : g) (void)hipGraphExecDestroy(x.exec);
    g.clear();
  }
  ~ManyGraphs() {
    drop();
    if (host) (void)hipHostFree(host);
    if (cap) (void)hipStreamDestroy(cap);
  }
};
thread_local ManyGraphs g_many;
constexpr size_t kManyGraphsMax = 64;

bool same_params(const lv_params& a, const lv_params& b) {
  return a.tolerance == b.tolerance && a.max_iterations == b.max_iterations && a.mode == b.mode &&
         a.swap_guard == b.swap_guard;
}

// Batched-launch tuning per size class (lv_many_tuning).
lv_many_tuning g_many_tuning[LV_MANY_CLASSES] = {
    {256, 65535}, {256, 65535}, {256, 65535}, {256, 65535}, {256, 65535}, {256, 65535},
    {256, 65535}, {256, 65535}, {256, 65535}, {256, 65535}, {256, 65535}, {256, 65535}};

lv_many_tuning clamp_many(lv_many_tuning t) {
  t.wave_max_degree = std::max(1, std::min(t.wave_max_degree, kManyWaveDeg));
  t.grid = std::max(1, std::min(t.grid, 65535));
  return t;
}

lv_status many_graph(void* desc, size_t desc_bytes, int32_t count, const lv_params& p, const lv_many_tuning& tu,
                     ManyGraph** out) {
  // the next power of two, within the descriptor buffer (>= count: checked by the caller)
  const int64_t fit = static_cast<int64_t>((desc_bytes - kManyHeader) / sizeof(ManyItem));
  int64_t b = 1;
  while (b < count) b <<= 1;
  const int32_t bucket = static_cast<int32_t>(std::min<int64_t>(b, fit));
  const size_t bytes = kManyHeader + sizeof(ManyItem) * static_cast<size_t>(bucket);
  ManyGraphs& G = g_many;
  if (bytes > G.host_bytes) {  // a larger staging buffer: graphs that copy through the old one go
    G.drop();
    if (G.host) LV_HIP(hipHostFree(G.host));
    G.host = nullptr;
    G.host_bytes = 0;
    void* q = nullptr;
    LV_HIP(hipHostMalloc(&q, bytes, hipHostMallocDefault));
    G.host = static_cast<char*>(q);
    G.host_bytes = bytes;
  }
  for (auto& x : G.g)
    if (x.desc == desc && x.bucket == bucket && same_params(x.p, p) && x.t.wave_max_degree == tu.wave_max_degree &&
        x.t.grid == tu.grid) {
      *out = &x;
      return LV_OK;
    }
  if (G.g.size() >= kManyGraphsMax) G.drop();
  if (!G.cap) LV_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  char* d = static_cast<char*>(desc);
  hipGraph_t graph = nullptr;
  LV_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
  (void)hipMemcpyAsync(d, G.host, bytes, hipMemcpyHostToDevice, G.cap);
  launch_many_df(reinterpret_cast<const int32_t*>(d), reinterpret_cast<ManyItem*>(d + kManyHeader),
                 std::min(bucket, tu.grid), p, tu.wave_max_degree, G.cap);
  (void)hipMemcpyAsync(G.host, d, bytes, hipMemcpyDeviceToHost, G.cap);
  LV_HIP(hipStreamEndCapture(G.cap, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  LV_HIP(e);
  ManyGraph x;
  x.desc = desc;
  x.bucket = bucket;
  x.p = p;
  x.t = tu;
  x.host = G.host;
  x.exec = exec;
  G.g.push_back(x);
  *out = &G.g.back();
  return LV_OK;
}

}  // namespace lv

// ---- scratch of the entry point for callers that cannot allocate ---------
// A file-scope device array: each GPU the library runs on holds its own copy
// (64 MiB) from the time the code object is loaded until the process ends.
// Host code never passes its name to a kernel (the name is a host-side
// stand-in); it takes the device address once per device with
// hipGetSymbolAddress and uses that.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace lv {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the
// first call on that device.
lv_status scratch_address(void** out) {
  int dev = -1;
  LV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LV_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LV_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LV_OK;
}

struct NoAllocScope {
  NoAllocScope() { g_no_alloc = true; }
  ~NoAllocScope() { g_no_alloc = false; }
};

}  // namespace
}  // namespace lv

using namespace lv;

extern "C" {

size_t lv_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

lv_status louvain_df_noalloc(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                             lv_state* state, lv_stats* stats, void* stream) {
  if (!graph_ok(g)) return fail(LV_EINVAL, "invalid graph");
  const size_t need = lv_workspace_bytes(g->n, g->cap);
  if (need > kNoAllocScratchBytes) {
    static thread_local char msg[160];
    std::snprintf(msg, sizeof(msg),
                  "louvain_df_noalloc: the graph needs %zu bytes of scratch, above the %zu bytes it holds "
                  "(use louvain_df with a workspace)",
                  need, kNoAllocScratchBytes);
    return fail(LV_EWORKSPACE, msg);
  }
  void* ws = nullptr;
  lv_status s = scratch_address(&ws);
  if (s) return s;
  NoAllocScope scope;
  return run_louvain(A_DF, g, del, ins, p, state, ws, kNoAllocScratchBytes, stats, stream);
}

void lv_default_params(lv_params* p) {
  if (!p) return;
  p->tolerance = 1e-2;
  p->tolerance_drop = 10.0;
  p->aggregation_tolerance = 0.8;
  p->max_iterations = 20;
  p->max_passes = 10;
  p->mode = LV_ASYNC;
  p->swap_guard = 1;
  p->recompute_weights = 0;
  p->reserved = 0;
}

size_t lv_workspace_bytes(int32_t n, int64_t cap) {
  Workspace ws;
  return carve_workspace(ws, nullptr, n, cap);
}

int64_t lv_graph_capacity_bound(int32_t n, int64_t m, float slack_frac, int32_t slack_min) {
  if (n < 0 || m < 0) return -1;
  const double arcs = 2.0 * static_cast<double>(m);
  const double frac = slack_frac > 0.f ? slack_frac : 0.0;
  const int64_t smin = slack_min > 0 ? slack_min : 0;
  return static_cast<int64_t>(std::ceil(arcs * (1.0 + frac))) + static_cast<int64_t>(n) * (smin + 1) + 1;
}

lv_status lv_graph_build(lv_graph* g, const lv_edges* e, float slack_frac, int32_t slack_min, void* wsp,
                         size_t ws_bytes, void* stream) {
  if (!graph_ok(g) || !edges_ok(e)) return fail(LV_EINVAL, "invalid graph or edge list");
  if (slack_frac < 0.f || slack_min < 0) return fail(LV_EINVAL, "negative slack");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace ws;
  lv_status s = setup_ws(ws, g, wsp, ws_bytes);
  if (s) return s;
  int64_t* host = nullptr;
  if ((s = pinned(&host))) return s;
  LV_HIP(hipMemsetAsync(ws.ctr, 0, sizeof(int64_t) * CTR_COUNT, st));
  LV_HIP(hipMemsetAsync(g->row_len, 0, sizeof(int32_t) * static_cast<size_t>(g->n), st));
  launch_build_count(*e, g->n, g->row_len, ws.ctr, st);
  launch_row_capacity(g->row_len, ws.i64tmp, g->n, slack_frac, slack_min, st);
  exclusive_scan_i64(ws.i64tmp, g->row_start, g->n, ws, st);
  LV_CHECK_LAUNCH();
  if ((s = read_counters(host, ws, CTR_COUNT, st))) return s;
  if (host[CTR_ERR]) return fail(static_cast<lv_status>(host[CTR_ERR]), "edge list has a bad id, self-loop or weight");
  if (host[CTR_TOTAL] >= (int64_t(1) << 31)) return fail(LV_EOVERFLOW, "total arc weight 2m >= 2^31");
  int64_t need = 0;
  if ((s = read_i64(&need, g->row_start + g->n, st))) return s;
  if (need > g->cap) return fail(LV_ENOSLACK, "graph capacity too small for the edge list and slack");
  LV_HIP(hipMemsetAsync(g->row_len, 0, sizeof(int32_t) * static_cast<size_t>(g->n), st));
  LV_HIP(hipMemsetAsync(g->two_m, 0, sizeof(int64_t), st));
  launch_build_scatter(*e, g->row_start, g->row_len, g->col, g->w, g->two_m, st);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

lv_status lv_graph_relayout(const lv_graph* src, lv_graph* dst, float slack_frac, int32_t slack_min, void* wsp,
                            size_t ws_bytes, void* stream) {
  if (!graph_ok(src) || !graph_ok(dst) || src->n != dst->n) return fail(LV_EINVAL, "invalid graphs");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace ws;
  lv_status s = setup_ws(ws, dst, wsp, ws_bytes);
  if (s) return s;
  launch_row_capacity(src->row_len, ws.i64tmp, src->n, slack_frac, slack_min, st);
  exclusive_scan_i64(ws.i64tmp, dst->row_start, src->n, ws, st);
  LV_CHECK_LAUNCH();
  int64_t need = 0;
  if ((s = read_i64(&need, dst->row_start + dst->n, st))) return s;
  if (need > dst->cap) return fail(LV_ENOSLACK, "destination capacity too small");
  launch_relayout_copy(*src, dst->row_start, dst->row_len, dst->col, dst->w, st);
  LV_HIP(hipMemcpyAsync(dst->two_m, src->two_m, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  LV_CHECK_LAUNCH();
  return LV_OK;
}

namespace {

// Enqueues the whole batch edit (both phases; phase 2 is gated on the
// device by the error slot) without waiting.  Host-side failures only.
lv_status enqueue_batch(lv_graph* g, const lv_edges* del, const lv_edges* ins, Workspace& ws, hipStream_t st) {
  if (del->count + ins->count == 0) return LV_OK;
  const int64_t U = del->count + ins->count, E = 2 * U;
  BatchScratch b;
  b.size = static_cast<int64_t>(pow2_at_least(2 * U + 2));
  b.dirs = E;
  const int64_t chunks = batch_chunks_bound(E, g->cap);
  size_t need = 0;
  auto room = [&](size_t bytes) { need += align_up(bytes); };
  room(8ull * b.size);
  room(4ull * b.size);
  room(4ull * b.size);
  room(16ull * b.size);
  room(4ull * U);
  for (int k = 0; k < 11; ++k) room(4ull * E);
  room(8ull * ins->count + 4);
  room(sizeof(BatchScratch::Chunk) * chunks);
  if (need > static_cast<size_t>(ws.pool_slots) * 4) return fail(LV_EWORKSPACE, "batch too large for the workspace pool");
  char* p = reinterpret_cast<char*>(ws.pool_keys);
  auto grab = [&](size_t bytes) {
    char* q = p;
    p += align_up(bytes);
    return q;
  };
  b.keys = reinterpret_cast<uint64_t*>(grab(8ull * b.size));
  b.dw = reinterpret_cast<int32_t*>(grab(4ull * b.size));
  b.iw = reinterpret_cast<int32_t*>(grab(4ull * b.size));
  b.pos = reinterpret_cast<int64_t*>(grab(16ull * b.size));
  b.slot = reinterpret_cast<int32_t*>(grab(4ull * U));
  int32_t** per_dir[11] = {&b.row_of, &b.r_len,  &b.r_cnt, &b.r_pbase, &b.r_zero, &b.r_app,
                           &b.r_hole, &b.d_rank, &b.part,  &b.tcol,    &b.tw};
  for (int k = 0; k < 11; ++k) *per_dir[k] = reinterpret_cast<int32_t*>(grab(4ull * E));
  b.kind = reinterpret_cast<int32_t*>(grab(8ull * ins->count + 4));
  b.chunk = reinterpret_cast<BatchScratch::Chunk*>(grab(sizeof(BatchScratch::Chunk) * chunks));
  b.tag = ws.dE;
  b.row_slot = ws.ccount;
  // phase 2 is gated on the device by the error slot, so the whole update
  // is enqueued at once and the host waits a single time
  launch_batch_phase1(*g, *del, *ins, b, ws.words, ws.ctr, st);
  launch_batch_phase2(*g, *del, *ins, b, ws.ctr, st);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

}  // namespace

lv_status apply_batch(lv_graph* g, const lv_edges* del, const lv_edges* ins, void* wsp, size_t ws_bytes,
                      void* stream) {
  if (!graph_ok(g) || !edges_ok(del) || !edges_ok(ins)) return fail(LV_EINVAL, "invalid graph or batch");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace ws;
  lv_status s = setup_ws(ws, g, wsp, ws_bytes);
  if (s) return s;
  int64_t* host = nullptr;
  if ((s = pinned(&host))) return s;
  if (del->count + ins->count == 0) return LV_OK;
  if ((s = enqueue_batch(g, del, ins, ws, st))) return s;
  if ((s = read_counters(host, ws, CTR_COUNT, st))) return s;
  if (host[CTR_ERR]) return batch_error(host[CTR_ERR]);
  return LV_OK;
}

lv_status louvain_static(const lv_graph* g, const lv_params* p, lv_state* out, void* ws, size_t ws_bytes,
                         lv_stats* stats, void* stream) {
  return run_louvain(A_STATIC, g, nullptr, nullptr, p, out, ws, ws_bytes, stats, stream);
}

lv_status louvain_nd(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                     lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream) {
  return run_louvain(A_ND, g, del, ins, p, state, ws, ws_bytes, stats, stream);
}

lv_status louvain_ds(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                     lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream) {
  return run_louvain(A_DS, g, del, ins, p, state, ws, ws_bytes, stats, stream);
}

lv_status louvain_df(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                     lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream) {
  return run_louvain(A_DF, g, del, ins, p, state, ws, ws_bytes, stats, stream);
}

lv_status louvain_df_apply(lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                           lv_state* state, void* wsp, size_t ws_bytes, lv_stats* stats, void* stream) {
  if (!graph_ok(g) || !edges_ok(del) || !edges_ok(ins)) return fail(LV_EINVAL, "invalid graph or batch");
  if (!params_ok(p)) return fail(LV_EINVAL, "invalid parameters");
  if (!state || !state->C || !state->K || !state->Sigma) return fail(LV_EINVAL, "invalid state");
  if (p->recompute_weights) {  // K and Sigma come from the edited rows: the edit must be complete
    const lv_status s = apply_batch(g, del, ins, wsp, ws_bytes, stream);
    return s ? s : run_louvain(A_DF, g, del, ins, p, state, wsp, ws_bytes, stats, stream);
  }
  Workspace ws;
  lv_status s = setup_ws(ws, g, wsp, ws_bytes);
  if (s) return s;
  if ((s = enqueue_batch(g, del, ins, ws, static_cast<hipStream_t>(stream)))) return s;
  return run_louvain(A_DF, g, del, ins, p, state, wsp, ws_bytes, stats, stream, 0, true);
}

size_t lv_many_scratch_bytes(int32_t n, int32_t max_updates) { return many_scratch_bytes(n, max_updates); }

size_t lv_many_desc_bytes(int32_t count) {
  return kManyHeader + sizeof(ManyItem) * static_cast<size_t>(count > 0 ? count : 1);
}

}  // extern "C"

namespace lv {
namespace {

// Host side of a batched call: item descriptors (LV_ETOOLARGE marks items
// the kernel must leave to the single-graph path).
lv_status many_prepare(const lv_item* items, int32_t count, std::vector<ManyItem>& h) {
  h.assign(static_cast<size_t>(count), ManyItem{});
  for (int32_t k = 0; k < count; ++k) {
    const lv_item& x = items[k];
    ManyItem& m = h[k];
    std::memset(&m, 0, sizeof(ManyItem));
    if (!graph_ok(&x.g) || !x.state.C || !x.state.K || !x.state.Sigma || !x.state.size || !edges_ok(&x.del) ||
        !edges_ok(&x.ins) || !x.scratch)
      return fail(LV_EINVAL, "invalid item");
    m.row_start = x.g.row_start;
    m.row_len = x.g.row_len;
    m.col = x.g.col;
    m.w = x.g.w;
    m.two_m = x.g.two_m;
    m.n = x.g.n;
    m.max_updates = x.max_updates;
    m.C = x.state.C;
    m.K = x.state.K;
    m.Sigma = x.state.Sigma;
    m.size = x.state.size;
    m.du = x.del.u;
    m.dv = x.del.v;
    m.dw = x.del.w;
    m.iu = x.ins.u;
    m.iv = x.ins.v;
    m.iw = x.ins.w;
    m.nd = static_cast<int32_t>(x.del.count);
    m.ni = static_cast<int32_t>(x.ins.count);
    m.scratch = x.scratch;
    // outside the kernel's limits: the single-graph path takes it
    if (x.del.count + x.ins.count > x.max_updates || x.del.count + x.ins.count > LV_MANY_MAX_UPDATES ||
        x.max_updates <= 0 || x.g.n <= 0)
      m.status = LV_ETOOLARGE;
  }
  return LV_OK;
}

// After the batched kernel: statuses and statistics, the single-graph path
// for items outside the kernel's limits, and aggregation with later passes
// for graphs whose pass 0 iterated more than once (Alg. 4).
void many_finish(const lv_item* items, int32_t count, const std::vector<ManyItem>& h, const lv_params* p, void* ws,
                 size_t ws_bytes, int32_t* status, lv_stats* stats, void* stream, double batched_s) {
  for (int32_t k = 0; k < count; ++k) {
    const ManyItem& m = h[k];
    const lv_item& x = items[k];
    lv_stats local;
    lv_stats& S = stats ? stats[k] : local;
    std::memset(&S, 0, sizeof(lv_stats));
    status[k] = m.status;
    if (m.status == LV_ETOOLARGE) {  // single-graph path from the start
      if (!ws) {
        status[k] = LV_EWORKSPACE;
        continue;
      }
      lv_graph g = x.g;
      lv_state state = x.state;
      lv_status s = apply_batch(&g, &x.del, &x.ins, ws, ws_bytes, stream);
      if (s == LV_OK) s = run_louvain(A_DF, &g, &x.del, &x.ins, p, &state, ws, ws_bytes, &S, stream);
      status[k] = s;
      continue;
    }
    if (m.status != LV_OK) continue;
    if (m.iterations > 1) {  // aggregation and further passes (Alg. 4)
      if (!ws) {
        status[k] = LV_EWORKSPACE;
        continue;
      }
      lv_graph g = x.g;
      lv_state state = x.state;
      const lv_status s = run_louvain(A_DF, &g, &x.del, &x.ins, p, &state, ws, ws_bytes, &S, stream, m.iterations);
      status[k] = s;
    } else {
      S.passes = 1;
    }
    S.iterations[0] = m.iterations;
    S.moves += m.moves;
    S.arcs_scanned += m.arcs_scanned;
    S.vertices_affected = m.vertices_affected;
    for (int t = 0; t < m.iterations && t < kManyIters && t < LV_MAX_ITERS; ++t) {
      S.iter_moves[0][t] = m.iter_moves[t];
      S.iter_gain[0][t] = m.iter_gain[t];
    }
    S.seconds += batched_s;
  }
}

int32_t many_size_class(const std::vector<ManyItem>& h) {
  if (h.empty()) return 0;
  double sum = 0.0;
  for (const ManyItem& m : h) sum += static_cast<double>(m.n);
  const double mean = sum / static_cast<double>(h.size());
  int32_t k = 0;
  while (k + 1 < LV_MANY_CLASSES && mean > static_cast<double>(int64_t(1) << (k + 9))) ++k;
  return k;
}

lv_status many_check(int32_t count, const lv_item* items, const int32_t* status, const void* desc, const lv_params* p,
                     size_t desc_bytes) {
  if (count < 0 || (count > 0 && (!items || !status || !desc))) return fail(LV_EINVAL, "invalid arguments");
  if (!params_ok(p)) return fail(LV_EINVAL, "invalid parameters");
  if (p->recompute_weights) return fail(LV_EINVAL, "the batched launch updates K and Sigma incrementally only");
  if (desc_bytes < lv_many_desc_bytes(count)) return fail(LV_EWORKSPACE, "descriptor buffer too small");
  return LV_OK;
}

}  // namespace
}  // namespace lv

extern "C" {

void lv_get_many_tuning(int32_t size_class, lv_many_tuning* t) {
  if (t && size_class >= 0 && size_class < LV_MANY_CLASSES) *t = g_many_tuning[size_class];
}

void lv_set_many_tuning(int32_t size_class, const lv_many_tuning* t) {
  if (t && size_class >= 0 && size_class < LV_MANY_CLASSES) g_many_tuning[size_class] = clamp_many(*t);
}

int32_t lv_many_size_class(const lv_item* items, int32_t count) {
  if (!items || count <= 0) return 0;
  std::vector<ManyItem> h(static_cast<size_t>(count));
  for (int32_t k = 0; k < count; ++k) h[k].n = items[k].g.n;
  return many_size_class(h);
}

lv_status louvain_df_many(const lv_item* items, int32_t count, const lv_params* p, void* desc, size_t desc_bytes,
                          void* ws, size_t ws_bytes, int32_t* status, lv_stats* stats, void* stream) {
  lv_status s = many_check(count, items, status, desc, p, desc_bytes);
  if (s) return s;
  if (count == 0) return LV_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t_start = std::chrono::steady_clock::now();
  std::vector<ManyItem> h;
  if ((s = many_prepare(items, count, h))) return s;
  const lv_many_tuning tu = clamp_many(g_many_tuning[many_size_class(h)]);
  ManyGraph* mg = nullptr;
  if ((s = many_graph(desc, desc_bytes, count, *p, tu, &mg))) return s;
  *reinterpret_cast<int32_t*>(mg->host) = count;
  std::memcpy(mg->host + kManyHeader, h.data(), sizeof(ManyItem) * h.size());
  LV_HIP(hipGraphLaunch(mg->exec, st));
  LV_HIP(hipStreamSynchronize(st));
  std::memcpy(h.data(), mg->host + kManyHeader, sizeof(ManyItem) * h.size());
  const double batched_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  many_finish(items, count, h, p, ws, ws_bytes, status, stats, stream, batched_s);
  return LV_OK;
}

lv_status lv_autotune_many(const lv_item* items, int32_t count, const lv_params* p, void* desc, size_t desc_bytes,
                           void* ws, size_t ws_bytes, int32_t* status, lv_stats* stats, lv_many_tuning* best,
                           void* stream) {
  lv_status s = many_check(count, items, status, desc, p, desc_bytes);
  if (s) return s;
  if (count == 0) return LV_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t_start = std::chrono::steady_clock::now();
  std::vector<ManyItem> h;
  if ((s = many_prepare(items, count, h))) return s;
  const int32_t cls = many_size_class(h);
  // one graph per workgroup (the hardware hands workgroups to free compute
  // units, which balances graphs of uneven size); the candidates differ in
  // the wavefront / workgroup split and the LDS table size it implies
  static const int32_t waves[] = {32, 64, 128, 256};
  const int32_t grid_cap = g_many_tuning[cls].grid;
  std::vector<lv_many_tuning> cand;
  for (int32_t w : waves) cand.push_back(lv_many_tuning{w, grid_cap});
  const int32_t nc = static_cast<int32_t>(cand.size());
  // items by size, dealt round-robin: every candidate gets a like share of
  // small and large graphs (a launch lasts as long as its largest graph)
  std::vector<int32_t> order(static_cast<size_t>(count));
  for (int32_t k = 0; k < count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return static_cast<int64_t>(h[a].n) + h[a].nd + h[a].ni > static_cast<int64_t>(h[b].n) + h[b].nd + h[b].ni;
  });
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LV_HIP(hipEventCreate(&e0));
  LV_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  char* d = static_cast<char*>(desc);
  // the kernel's code is loaded by a first launch with no items
  int32_t zero = 0;
  LV_HIP(hipMemcpyAsync(d, &zero, sizeof(int32_t), hipMemcpyHostToDevice, st));
  launch_many_df(reinterpret_cast<const int32_t*>(d), reinterpret_cast<ManyItem*>(d + kManyHeader), 1, *p,
                 cand[0].wave_max_degree, st);
  LV_CHECK_LAUNCH();
  LV_HIP(hipStreamSynchronize(st));
  double best_t = 0.0;
  int32_t best_k = -1;
  std::vector<ManyItem> grp;
  for (int32_t c = 0; c < nc; ++c) {
    grp.clear();
    for (int32_t k = c; k < count; k += nc) grp.push_back(h[order[k]]);
    if (grp.empty()) continue;
    const int32_t gn = static_cast<int32_t>(grp.size());
    LV_HIP(hipMemcpyAsync(d, &gn, sizeof(int32_t), hipMemcpyHostToDevice, st));
    LV_HIP(hipMemcpyAsync(d + kManyHeader, grp.data(), sizeof(ManyItem) * grp.size(), hipMemcpyHostToDevice, st));
    LV_HIP(hipEventRecord(e0, st));
    launch_many_df(reinterpret_cast<const int32_t*>(d), reinterpret_cast<ManyItem*>(d + kManyHeader),
                   std::min(gn, cand[c].grid), *p, cand[c].wave_max_degree, st);
    LV_CHECK_LAUNCH();
    LV_HIP(hipEventRecord(e1, st));
    LV_HIP(hipMemcpyAsync(grp.data(), d + kManyHeader, sizeof(ManyItem) * grp.size(), hipMemcpyDeviceToHost, st));
    LV_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    LV_HIP(hipEventElapsedTime(&ms, e0, e1));
    for (int32_t k = c, q = 0; k < count; k += nc, ++q) h[order[k]] = grp[q];
    const double per_item = static_cast<double>(ms) / gn;
    if (best_k < 0 || per_item < best_t) {
      best_t = per_item;
      best_k = c;
    }
  }
  if (best_k >= 0) {
    g_many_tuning[cls] = clamp_many(cand[best_k]);
    if (best) *best = g_many_tuning[cls];
  }
  const double batched_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  many_finish(items, count, h, p, ws, ws_bytes, status, stats, stream, batched_s);
  return LV_OK;
}

lv_status modularity(const lv_graph* g, const int32_t* C, double* q_host, void* wsp, size_t ws_bytes, void* stream) {
  if (!graph_ok(g) || !C || !q_host) return fail(LV_EINVAL, "invalid arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace ws;
  lv_status s = setup_ws(ws, g, wsp, ws_bytes);
  if (s) return s;
  int64_t* host = nullptr;
  if ((s = pinned(&host))) return s;
  LevelGraph L;
  L.n = g->n;
  L.row_start = g->row_start;
  L.row_len = g->row_len;
  L.col = g->col;
  L.w = g->w;
  LV_HIP(hipMemsetAsync(ws.ctr, 0, sizeof(int64_t) * CTR_COUNT, st));
  LV_HIP(hipMemsetAsync(ws.i64tmp, 0, sizeof(int64_t) * (static_cast<size_t>(g->n) + 1), st));
  // K_i and the intra-community arc weight (ctr[AUX0]), then Σ_c and Σ_c^2
  launch_row_sums(L, C, ws.lK, nullptr, nullptr, nullptr, ws, st);
  launch_accumulate(C, g->n, nullptr, ws.lK, nullptr, ws.i64tmp, st);
  LV_HIP(hipMemsetAsync(ws.ctr + CTR_AUX1, 0, sizeof(int64_t), st));
  launch_sum_squares(ws.i64tmp, g->n, ws.ctr + CTR_AUX1, st);
  LV_CHECK_LAUNCH();
  int64_t two_m = 0;
  if ((s = read_i64(&two_m, g->two_m, st))) return s;
  if ((s = read_counters(host, ws, CTR_COUNT, st))) return s;
  if (two_m <= 0) return fail(LV_EEMPTY, "graph has no edges (2m = 0)");
  if (two_m >= (int64_t(1) << 31)) return fail(LV_EOVERFLOW, "total arc weight 2m >= 2^31");
  // Q = (2m Σσ_c - Σ_c Σ_c^2) / (2m)^2; the numerator is exact in int64
  const int64_t qnum = two_m * stat(host + CTR_STATS0, ST_INTRA) - host[CTR_AUX1];
  *q_host = static_cast<double>(qnum) / (static_cast<double>(two_m) * static_cast<double>(two_m));
  return LV_OK;
}

lv_status lv_set_timing(uint32_t mask) {
  if (mask >> LV_NTIMED) return fail(LV_EINVAL, "unknown kernel for timing");
  g_timed_mask.store(mask);
  return LV_OK;
}

void lv_set_tuning(const lv_tuning* t) {
  if (t) g_tuning = *t;
}

void lv_get_tuning(lv_tuning* t) {
  if (t) *t = effective_tuning();
}

lv_status lv_autotune(const lv_graph* g, lv_state* scratch, void* ws, size_t ws_bytes, int32_t repeats,
                      lv_tuning* best, void* stream) {
  if (!graph_ok(g)) return fail(LV_EINVAL, "invalid graph");
  if (!scratch || !scratch->C || !scratch->K || !scratch->Sigma) return fail(LV_EINVAL, "invalid scratch state");
  const lv_tuning base = g_tuning;
  lv_params p;
  lv_default_params(&p);
  p.mode = LV_SYNC;
  p.max_iterations = 1;
  p.max_passes = 1;
  static const int32_t kCandidates[] = {64, 128, 256, 512};
  // the threshold in force stays unless a candidate is faster by more than
  // kAutotuneMargin (run-to-run timing noise is a few per cent)
  constexpr float kAutotuneMargin = 0.03f;
  const int32_t current = effective_tuning().wave_max_degree;
  float best_ms = 0.f, current_ms = -1.f;
  int32_t best_w = current;
  bool have = false;
  for (const int32_t w : kCandidates) {
    lv_tuning t = base;
    t.wave_max_degree = w;
    g_tuning = t;
    float ms = 0.f;
    for (int32_t r = 0; r < std::max(1, repeats); ++r) {
      lv_stats S;
      lv_state st = *scratch;
      const lv_status s = run_louvain(A_STATIC, g, nullptr, nullptr, &p, &st, ws, ws_bytes, &S, stream);
      if (s != LV_OK) {
        g_tuning = base;
        return s;
      }
      if (r == 0 || S.ms_move < ms) ms = S.ms_move;
    }
    if (w == current) current_ms = ms;
    if (!have || ms < best_ms) {
      have = true;
      best_ms = ms;
      best_w = w;
    }
  }
  if (current_ms >= 0.f && best_ms > current_ms * (1.f - kAutotuneMargin)) best_w = current;
  lv_tuning t = base;
  t.wave_max_degree = best_w;
  g_tuning = t;
  if (best) *best = effective_tuning();
  return LV_OK;
}

const char* lv_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
