/*
 * louvain.h -- C interface of the MI355X (gfx950) DF Louvain library.
 *
 * The library implements the data-parallel hot path of Dynamic Frontier
 * (DF) Louvain (Sahu, "DF Louvain: Fast Incrementally Expanding Approach for
 * Community Detection on Dynamic Graphs", arXiv 2404.19634) together with
 * the static, Naive-dynamic (ND) and Delta-screening (DS) variants that the
 * paper compares it with.  Every step runs in hand-written HIP kernels.
 *
 * General conventions
 *  - Pointers inside lv_graph, lv_edges and lv_state, and the `ws`
 *    workspace, are HIP DEVICE pointers owned by the caller.  The library
 *    never allocates or frees caller memory; it keeps no device memory of
 *    its own apart from a small pinned host buffer for status readback
 *    (one per host thread, kept until the process ends).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work is enqueued on it.  Entry points that must return a
 *    status which depends on device data (validation, convergence) wait for
 *    the stream before returning; everything they enqueued is then done.
 *  - Graphs are undirected and stored with both arc directions.  Vertex ids
 *    are int32, weights positive int32, weighted degrees K and community
 *    totals Sigma int64.  The total arc weight 2m must stay below 2^31 so
 *    that every gain fits in int64 (LV_EOVERFLOW otherwise).
 *  - Nothing throws across this interface.  A negative status is an
 *    error; lv_last_error() describes the last one on the calling thread.
 *    Validation errors leave all caller data untouched.  LV_EHIP means a
 *    HIP call failed; caller data may then be partially updated.
 *  - Calls that share a workspace must not overlap (same stream or
 *    explicitly ordered).
 */
#ifndef LOUVAIN_H
#define LOUVAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lv_status;
#define LV_OK 0
#define LV_EINVAL (-1)      /* bad argument, id out of range, self-loop, w <= 0, duplicate pair */
#define LV_ENOEDGE (-2)     /* a deletion names a missing edge or more weight than present */
#define LV_ENOSLACK (-3)    /* a row lacks free capacity; nothing was changed */
#define LV_EOVERFLOW (-4)   /* total arc weight 2m >= 2^31 */
#define LV_EEMPTY (-5)      /* graph without edges (2m = 0) */
#define LV_EHIP (-6)        /* a HIP runtime call failed */
#define LV_EWORKSPACE (-7)  /* workspace smaller than lv_workspace_bytes() */
#define LV_ETOOLARGE (-8)   /* louvain_df_many: item outside the batched kernel's limits */

#define LV_SYNC 0   /* Jacobi moves: every vertex decides on the iteration-start state */
#define LV_ASYNC 1  /* moves applied as they are decided (racy, as in the paper's loop) */

#define LV_MAX_PASSES 16
#define LV_MAX_ITERS 32

/*
 * Slack-padded CSR (the paper's "holey" CSR of its aggregation phase,
 * Alg. 6, used here for the input graph too so that batch updates edit it
 * in place).  Row i occupies col/w[row_start[i] .. row_start[i] +
 * row_len[i]) and may grow up to row_start[i+1].  row_start[n] is the used
 * capacity.  *two_m (device) is the total arc weight, tracked across
 * batches as the paper assumes (Section 5.1.5).
 */
typedef struct {
  int32_t n;          /* number of vertices */
  int64_t cap;        /* allocated length of col and w */
  int64_t* row_start; /* device int64[n + 1] */
  int32_t* row_len;   /* device int32[n] */
  int32_t* col;       /* device int32[cap] */
  int32_t* w;         /* device int32[cap] */
  int64_t* two_m;     /* device int64[1] */
} lv_graph;

/* A list of undirected edges or updates, each given once (device arrays). */
typedef struct {
  const int32_t* u;
  const int32_t* v;
  const int32_t* w;
  int64_t count;
} lv_edges;

/* Community membership C, weighted degrees K, community totals Sigma
 * (Sigma indexed by community id).  Device arrays of length n.
 *
 * `size` is optional (NULL allowed): the member count of every community
 * id, size[c] = |{i : C_i = c}|.  Like Sigma it is auxiliary information
 * carried from one batch to the next (Section 4.1 keeps K and Sigma for
 * the same reason): the swap guard needs it, and recounting it costs a
 * pass over all n vertices per call.  When non-NULL, the dynamic entry
 * points trust it on entry and return it updated; louvain_static fills it.
 * When NULL, the library counts it in the workspace as needed. */
typedef struct {
  int32_t* C;
  int64_t* K;
  int64_t* Sigma;
  int32_t* size;
} lv_state;

/* Parameters; lv_default_params() gives the paper's values (Section
 * 5.1.2): tolerance 1e-2, drop 10, 20 iterations, 10 passes,
 * aggregation tolerance 0.8. */
typedef struct {
  double tolerance;             /* iteration tolerance tau on the summed ΔQ */
  double tolerance_drop;        /* tau is divided by this after each pass */
  double aggregation_tolerance; /* stop when |communities| / |vertices| exceeds it */
  int32_t max_iterations;       /* 1 .. LV_MAX_ITERS */
  int32_t max_passes;           /* 1 .. LV_MAX_PASSES */
  int32_t mode;                 /* LV_SYNC or LV_ASYNC */
  int32_t swap_guard;           /* 1: a singleton never joins a singleton of larger id */
  int32_t recompute_weights;    /* 1: the dynamic calls recompute K^t (row sums of G^t) and Sigma^t
                                   (from C^{t-1}) instead of updating K^{t-1}, Sigma^{t-1} by the
                                   batch: the variant without auxiliary information (Section 4.2).
                                   Same results, more work.  0 (default) for the incremental update;
                                   louvain_df_many accepts 0 only. */
  int32_t reserved;             /* must be 0 */
} lv_params;

/* Degree bins of the local-moving scan: rows of up to 4, 8, 16, 32 arcs
 * (lane groups), up to the wavefront threshold (one wavefront, LDS table),
 * up to 2048 arcs (one workgroup, LDS table), and longer hub rows (several
 * workgroups, global table). */
enum { LV_BIN_G4 = 0, LV_BIN_G8, LV_BIN_G16, LV_BIN_G32, LV_BIN_WAVE, LV_BIN_BLOCK, LV_BIN_HUB, LV_NBINS };
/* Kernels the measurement hook can time: the fused local-moving scan (all
 * degree bins and the hub-row inserts of a sub-round in one launch), the
 * frontier binning, and the hub-row table clear and decision kernels. */
enum { LV_TIME_SCAN = 0, LV_TIME_BINNING, LV_TIME_HUB_CLEAR, LV_TIME_HUB_DECIDE, LV_NTIMED };

/* Per-run statistics.  The first block matches the oracle's layout. */
typedef struct {
  int32_t passes;
  int32_t iterations[LV_MAX_PASSES];   /* iterations run in each pass */
  int64_t communities[LV_MAX_PASSES];  /* communities after a pass's moves (when counted) */
  int64_t moves;                       /* vertex moves over all passes */
  int64_t arcs_scanned;                /* sum of row lengths of processed vertices */
  int64_t vertices_affected;           /* distinct vertices processed in pass 0 */
  int64_t iter_moves[LV_MAX_PASSES][LV_MAX_ITERS];
  int64_t iter_gain[LV_MAX_PASSES][LV_MAX_ITERS]; /* sum of movers' gains (2m^2 ΔQ) */
  double seconds;                      /* host wall time of the call */
  /* GPU-side breakdown (hipEvent), milliseconds */
  float ms_mark;       /* initial marking + updateWeights */
  float ms_move;       /* local-moving iterations */
  float ms_aggregate;  /* renumber, lookup, aggregation */
  float ms_other;      /* output consistency, setup */
  int64_t arcs_aggregated; /* arcs read by aggregation */
  /* Local-moving work per degree bin (index LV_BIN_*): vertices processed,
   * arcs scanned, and the sub-rounds whose scan launch served the bin.
   * Summed over every iteration, pass and sub-round. */
  int64_t bin_vertices[LV_NBINS];
  int64_t bin_arcs[LV_NBINS];
  int32_t bin_launches[LV_NBINS];
  /* Launches bracketed by timing events (lv_set_timing) and their summed
   * GPU time, per timed kernel (index LV_TIME_*); zero for kernels that are
   * not timed. */
  int32_t timed_launches[LV_NTIMED];
  double timed_ms[LV_NTIMED];
} lv_stats;

/* Tunables chosen by the autotuner (degree-bin thresholds and launch
 * shapes).  Zero fields take built-in defaults, except the async_rounds,
 * fuse and defer fields, where 0 is a value (lv_get_tuning reports the
 * values in use). */
typedef struct {
  int32_t wave_max_degree;   /* rows up to this length go to one wavefront with an LDS table */
  int32_t blocks_small;      /* persistent grid size of the sub-wave kernels */
  int32_t blocks_wave;       /* persistent grid size of the wavefront kernel */
  int32_t blocks_hub;        /* persistent grid size of the workgroup kernel */
  int32_t async_rounds_log2; /* LV_ASYNC: each iteration runs 2^k hash-partitioned sub-rounds */
  int32_t async_rounds_min_frontier; /* ... when the frontier may exceed this many vertices */
  int32_t async_round_order; /* sub-rounds by 0: hash of the vertex id; 1: contiguous id ranges;
                                2: degree classes (highest first), hashed within a class */
  int32_t fuse_max_frontier; /* a sub-round scans all degree bins in one launch when its frontier
                                bound is at most this and an eighth of the level's vertices at
                                most (else one launch per bin); -1: never */
  int32_t defer_totals;      /* LV_ASYNC: 1 sums a workgroup's Sigma/size changes in LDS and applies
                                them when it ends; 0 applies each move's changes at once */
  int32_t revisit_min_degree; /* LV_ASYNC, degree-class order: each iteration visits the degree classes
                                 whose rows are all longer than this twice in a row (the second visit
                                 sees the first one's moves); 0: every class once */
} lv_tuning;

/* The paper's parameter values (Section 5.1.2). */
void lv_default_params(lv_params* p);

/* Bytes of device workspace needed by every call on a graph with n
 * vertices and capacity cap (the bound covers all passes and levels). */
size_t lv_workspace_bytes(int32_t n, int64_t cap);

/* Upper bound of the capacity lv_graph_build needs for m undirected edges
 * on n vertices with the given slack (so the caller can size col and w). */
int64_t lv_graph_capacity_bound(int32_t n, int64_t m, float slack_frac, int32_t slack_min);

/*
 * Build the slack CSR from an undirected edge list (each edge once, no
 * duplicate pairs).  Row capacity = deg + max(slack_min, ceil(slack_frac *
 * deg)).  g->n, g->cap and the device arrays must be set by the caller;
 * on return row_start, row_len, col, w and *two_m are filled.  Errors:
 * LV_EINVAL (id out of range, self-loop, w <= 0), LV_ENOSLACK (g->cap too
 * small), LV_EOVERFLOW.
 */
lv_status lv_graph_build(lv_graph* g, const lv_edges* edges, float slack_frac, int32_t slack_min,
                         void* ws, size_t ws_bytes, void* stream);

/* Copy `src` into `dst` (same n) with new slack; used after LV_ENOSLACK. */
lv_status lv_graph_relayout(const lv_graph* src, lv_graph* dst, float slack_frac, int32_t slack_min,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * apply_batch -- turn G^{t-1} into G^t in place (Section 3.4: the batch
 * holds deletions Δ- and insertions Δ+; Section 5.1.4: batches are
 * undirected).  Each update names an undirected pair once and applies to
 * both arcs.  Deletions run first and subtract w (an arc reaching weight 0
 * is removed); insertions then add w to an existing arc or append one into
 * the row's slack.  *two_m changes by 2(Σw_ins - Σw_del).
 * Everything is validated before anything changes: LV_EINVAL (id out of
 * range, self-loop, w <= 0, a pair repeated within Δ- or within Δ+),
 * LV_ENOEDGE (deleting a missing pair or more weight than present),
 * LV_ENOSLACK (a row would overflow its capacity).
 */
lv_status apply_batch(lv_graph* g, const lv_edges* del, const lv_edges* ins, void* ws, size_t ws_bytes,
                      void* stream);

/*
 * louvain_static -- Louvain from singleton communities (the paper's static
 * baseline, Alg. 4 with every vertex affected): K is computed from the
 * graph, Sigma = K, then passes of local-moving (Alg. 5) and aggregation
 * (Alg. 6).  Writes C, K, Sigma (and size, when non-NULL) of `out`.
 */
lv_status louvain_static(const lv_graph* g, const lv_params* p, lv_state* out, void* ws, size_t ws_bytes,
                         lv_stats* stats, void* stream);

/*
 * louvain_nd / louvain_ds / louvain_df -- dynamic Louvain after a batch
 * (Alg. 2 / Alg. 3 / Alg. 1).  `g` is G^t (apply_batch already ran);
 * `del` and `ins` are the batch.  `state` holds C^{t-1}, K^{t-1},
 * Sigma^{t-1} (and the matching size, when non-NULL) on entry and C^t,
 * K^t, Sigma^t (size^t) on return.  K and Sigma are
 * updated from the batch (Alg. 7) rather than recomputed; the initial
 * affected set is every vertex (ND), the delta-screening set (DS) or the
 * endpoints of intra-community deletions and cross-community insertions
 * (DF), which then grows by the neighbours of every moved vertex.
 * Community ids stay in [0, n) but are not made dense.
 */
lv_status louvain_nd(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                     lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream);
lv_status louvain_ds(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                     lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream);
lv_status louvain_df(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                     lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream);

/*
 * One dynamic update (Section 3.4, then Alg. 1): apply_batch(g, del, ins)
 * followed by louvain_df on the edited graph, enqueued together so that the
 * host waits once, at the end of the first local-moving iteration, instead
 * of also after the edit.  Same arguments, results and statistics as the two
 * calls in sequence.  Errors of the edit (LV_EINVAL, LV_ENOEDGE, LV_ENOSLACK,
 * LV_EOVERFLOW) are returned by this call with graph and state untouched;
 * the other errors are louvain_df's.  With p->recompute_weights = 1 the two
 * calls are made one after the other (K and Sigma are then read from the
 * edited rows).
 */
lv_status louvain_df_apply(lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                           lv_state* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream);

/*
 * louvain_df_noalloc -- louvain_df for callers that cannot allocate device
 * or host memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same computation and results, with
 * no workspace argument.  Its scratch is a device array inside the library
 * of lv_noalloc_scratch_bytes() bytes (64 MiB), held on each GPU the library
 * runs on until the process ends; the call allocates nothing (no hipMalloc,
 * no pinned buffer, no events: the ms_* fields and timed launches of
 * `stats` stay 0).  Graphs whose lv_workspace_bytes(n, cap) exceeds that size
 * get LV_EWORKSPACE and are left untouched.  The device is the current one;
 * `stream` must belong to it.  Every call on a GPU shares that GPU's array,
 * so calls that overlap on one GPU (other threads or streams) race: the
 * caller serialises them.  Other arguments and errors as louvain_df.
 */
size_t lv_noalloc_scratch_bytes(void);
lv_status louvain_df_noalloc(const lv_graph* g, const lv_edges* del, const lv_edges* ins, const lv_params* p,
                             lv_state* state, lv_stats* stats, void* stream);

/*
 * modularity -- Eq. 1: Q = Σ_c [σ_c/2m - (Σ_c/2m)^2] for membership C
 * (device int32[n], ids in [0, n)).  σ_c and Σ_c are exact int64 sums;
 * the host forms the FP64 quotient.  Waits for the stream.
 */
lv_status modularity(const lv_graph* g, const int32_t* C, double* q_host, void* ws, size_t ws_bytes,
                     void* stream);

/* Set or read the tuning table used by the calls above (process-wide). */
/*
 * louvain_df_many -- apply_batch followed by louvain_df (Section 3.4,
 * Alg. 1) on many independent graphs at once, in one persistent launch:
 * a workgroup takes a graph, edits it in place, updates K and Sigma, marks
 * the DF frontier and runs the local-moving iterations of pass 0.  A graph
 * whose pass 0 needs more than one iteration (so Alg. 4 aggregates and
 * goes on) continues on the single-graph path afterwards, as does an item
 * outside the kernel's limits (rows longer than 2048 arcs after its batch,
 * or a batch of more than LV_MANY_MAX_UPDATES updates, whose frontier is
 * too large for one workgroup).
 * Results are those of apply_batch + louvain_df on each graph alone
 * (bit-exact in LV_SYNC mode).
 *
 *   items      host array of `count` items; each names its graph, its state
 *              (size is required: member counts carried with the state),
 *              its batch, and its scratch: lv_many_scratch_bytes(n,
 *              max_updates) bytes of device memory, zero before its first
 *              use; each call leaves it ready for the next (keep one per
 *              graph); del.count + ins.count must not exceed max_updates.
 *   desc       device buffer of at least lv_many_desc_bytes(count) bytes
 *              (item count, item descriptors and results).  Keep one per
 *              calling thread: the call replays a HIP graph captured for
 *              this buffer (copy in, the persistent kernel, copy out; one
 *              graph per power-of-two size class of count that fits the
 *              buffer), and calls on one buffer must not overlap.
 *   ws         a workspace for the single-graph path, lv_workspace_bytes()
 *              of the largest graph that may need it; may be NULL, and then
 *              such items report LV_EWORKSPACE.
 *   status     host array of `count`: LV_OK or the item's own error
 *              (LV_EINVAL, LV_ENOEDGE, LV_ENOSLACK, LV_EOVERFLOW: nothing of
 *              that graph was changed; LV_EEMPTY after the edit).
 *   stats      host array of `count` lv_stats, or NULL.
 * Returns LV_OK unless a HIP call failed or an argument is invalid.
 * Synchronises `stream`.  Items must name distinct graphs.
 */
#define LV_MANY_MAX_UPDATES 4096

typedef struct {
  lv_graph g;
  lv_state state;
  lv_edges del;
  lv_edges ins;
  void* scratch;
  int32_t max_updates;
} lv_item;

size_t lv_many_scratch_bytes(int32_t n, int32_t max_updates);
size_t lv_many_desc_bytes(int32_t count);
lv_status louvain_df_many(const lv_item* items, int32_t count, const lv_params* p, void* desc, size_t desc_bytes,
                          void* ws, size_t ws_bytes, int32_t* status, lv_stats* stats, void* stream);

/*
 * Tuning of the batched launch, one entry per size class of graphs: a call
 * of louvain_df_many falls in class k when its graphs average at most
 * 2^(k+9) vertices (k = 0 .. LV_MANY_CLASSES-1; the last class takes all
 * larger ones).  The entry sets the mapping of the persistent kernel: rows
 * up to wave_max_degree arcs are scanned by one wavefront each with an LDS
 * table of twice that many slots, longer rows (up to 2048 arcs) by the
 * whole workgroup; grid is the number of workgroups the launch holds (one
 * graph at a time each).  Process-wide; lv_get/lv_set_many_tuning read and
 * restore the table (so a caller can persist it), lv_many_size_class names
 * the class of a set of items.
 */
#define LV_MANY_CLASSES 12
typedef struct {
  int32_t wave_max_degree; /* 1 .. 256 (default 256) */
  int32_t grid;            /* most workgroups of a launch, 1 .. 65535 (default 65535: one per graph) */
} lv_many_tuning;
void lv_get_many_tuning(int32_t size_class, lv_many_tuning* t);
void lv_set_many_tuning(int32_t size_class, const lv_many_tuning* t);
int32_t lv_many_size_class(const lv_item* items, int32_t count);

/*
 * lv_autotune_many -- louvain_df_many on `items` (same arguments, same
 * results and statistics per item) that also tunes the batched launch for
 * their size class.  The items, ordered by size, are dealt round-robin to
 * the candidate mappings (wave_max_degree 32, 64, 128, 256; the class's
 * grid), so each candidate gets a like mix of small and large graphs; each
 * runs its share in one launch timed with HIP events, and the one with the
 * least time per item becomes the class's entry (and *best when non-null).
 * Needs at least one item per candidate to time them all (fewer items: the
 * untimed candidates are skipped).  SYNC results do not depend on the
 * tuning.  Not to be called while other batched calls run.
 */
lv_status lv_autotune_many(const lv_item* items, int32_t count, const lv_params* p, void* desc, size_t desc_bytes,
                           void* ws, size_t ws_bytes, int32_t* status, lv_stats* stats, lv_many_tuning* best,
                           void* stream);

/*
 * Paper precision (Section 5.1.2: float32 edge weights, FP64 hashtable
 * values, sums and modularity).  The same slack CSR with float32 weights,
 * FP64 K, Sigma and 2m, and Eq. 2 evaluated as printed in FP64:
 *     ΔQ(i: d -> c) = (K_{i->c} - K_{i->d}) / m - K_i (K_i + Σ_c - Σ_d) / (2 m^2)
 * The best community has the largest ΔQ (lowest id on ties) and a vertex
 * moves only for ΔQ > 0; iterations stop when the movers' ΔQ sum to at most
 * the tolerance.  LV_ASYNC mode only (the results depend on the order of
 * floating-point sums, so there is no bit-exact SYNC contract); the
 * parameters, the swap guard, the sub-round schedule and the pass control
 * are the integer path's.  Aggregated arc weights are summed in FP64 and
 * stored as float32.  lv_stats reports passes, iterations, moves and arcs;
 * iter_gain stays 0 (the ΔQ sums are FP64).  Weights must be finite and
 * positive (LV_EINVAL).  No 2^31 bound applies.
 */
typedef struct {
  int32_t n;
  int64_t cap;
  int64_t* row_start; /* device int64[n + 1] */
  int32_t* row_len;   /* device int32[n] */
  int32_t* col;       /* device int32[cap] */
  float* w;           /* device float32[cap] */
  double* two_m;      /* device double[1]: total arc weight */
} lv_graph_f;

typedef struct {
  const int32_t* u;
  const int32_t* v;
  const float* w;
  int64_t count;
} lv_edges_f;

typedef struct {
  int32_t* C;
  double* K;
  double* Sigma;
  int32_t* size; /* optional, as in lv_state */
} lv_state_f;

size_t lv_workspace_bytes_f(int32_t n, int64_t cap);
/* As lv_graph_build (capacity bound: lv_graph_capacity_bound). */
lv_status lv_graph_build_f(lv_graph_f* g, const lv_edges_f* edges, float slack_frac, int32_t slack_min, void* ws,
                           size_t ws_bytes, void* stream);
/* As apply_batch (Section 3.4): deletions subtract (an arc whose weight
 * reaches 0 is removed; LV_ENOEDGE for a missing pair or more weight than
 * present), insertions add or append; all-or-nothing; *two_m moves by
 * 2(Σw_ins - Σw_del) in FP64. */
lv_status apply_batch_f(lv_graph_f* g, const lv_edges_f* del, const lv_edges_f* ins, void* ws, size_t ws_bytes,
                        void* stream);
/* Static Louvain (Alg. 4 from singletons) in the paper's precision. */
lv_status louvain_static_f(const lv_graph_f* g, const lv_params* p, lv_state_f* out, void* ws, size_t ws_bytes,
                           lv_stats* stats, void* stream);
/* DF Louvain (Alg. 1, updateWeights Alg. 7 in FP64) after apply_batch_f. */
lv_status louvain_df_f(const lv_graph_f* g, const lv_edges_f* del, const lv_edges_f* ins, const lv_params* p,
                       lv_state_f* state, void* ws, size_t ws_bytes, lv_stats* stats, void* stream);
/* Eq. 1 in FP64.  Waits for the stream. */
lv_status modularity_f(const lv_graph_f* g, const int32_t* C, double* q_host, void* ws, size_t ws_bytes,
                       void* stream);

/* Measurement hook.  lv_set_timing(mask) makes every later louvain_* call
 * time each launch of the kernels whose bit k is set in `mask` (k =
 * LV_TIME_*) with a pair of HIP events that the launch itself stamps with
 * the kernel's begin and end (hipExtLaunchKernel), and report their count
 * and summed time in lv_stats.  Up to 4096 launches per call are timed;
 * mask 0 turns timing off.  Process-wide setting; LV_EINVAL for unknown
 * bits. */
lv_status lv_set_timing(uint32_t mask);

void lv_set_tuning(const lv_tuning* t);
void lv_get_tuning(lv_tuning* t);

/*
 * lv_autotune -- picks the degree-bin threshold between the wavefront and
 * the workgroup mapping of the local-moving scan (Alg. 5) for graph g: for
 * each wave_max_degree in {64, 128, 256, 512} it times, with HIP events,
 * `repeats` SYNC local-moving sweeps of g from singletons (every vertex
 * scanned once) and keeps the fastest, unless the threshold in force is
 * within 3% of it (then that one stays).  The other tuning fields stay as
 * they are.  The result becomes the process-wide tuning (as lv_set_tuning)
 * and is written to *best when non-null.
 *   scratch  device C/K/Sigma arrays of g->n entries (contents overwritten;
 *            size may be NULL)
 *   ws       lv_workspace_bytes(g->n, g->cap) bytes of device memory
 * The graph is not modified.  Synchronises `stream`.  Not to be called
 * while other calls of this library run (they read the tuning).
 * Returns LV_OK, LV_EINVAL, LV_EWORKSPACE or LV_EHIP (tuning then as
 * before the call).
 */
lv_status lv_autotune(const lv_graph* g, lv_state* scratch, void* ws, size_t ws_bytes, int32_t repeats,
                      lv_tuning* best, void* stream);

/* Message for the last non-OK status returned on this thread. */
const char* lv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LOUVAIN_H */
