// Sequential reference ("oracle") for the DF Louvain hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test suite, the package smoke check and the
// benchmark's CPU-baseline leg do.  It shares no code, header, table or
// constant with the GPU implementation.
//
// It follows "DF Louvain: Fast Incrementally Expanding Approach for
// Community Detection on Dynamic Graphs" (arXiv 2404.19634) step by step:
//   * modularity                -- Eq. 1 (community form), FP64
//   * move gain                 -- Eq. 2, scaled by 2m^2 to an exact integer
//   * batch update              -- Section 3.4 (deletions, then insertions)
//   * updateWeights             -- Alg. 7
//   * DF / ND / DS marking      -- Alg. 1 / Alg. 2 / Alg. 3
//   * Louvain driver            -- Alg. 4
//   * local-moving phase        -- Alg. 5 (louvainMove, scanCommunities)
//   * aggregation phase         -- Alg. 6
// Readings of points the paper leaves open (sync/async move modes, tie
// breaks, the swap guard, convergence arithmetic) are listed in the design
// notes; each is applied here at the step it concerns.
//
// Plain data structures on purpose: adjacency lists, a dense per-call
// accumulator for the community hashtable (the paper's collision-free
// hashtable), sequential loops.  Integer weights, 64-bit sums.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <unordered_set>
#include <vector>

namespace {

enum : int32_t { OK = 0, E_INVAL = -1, E_NOEDGE = -2, E_OVERFLOW = -4, E_EMPTY = -5 };
enum : int32_t { STATIC = 0, ND = 1, DS = 2, DF = 3 };
enum : int32_t { SYNC = 0, ASYNC = 1 };

constexpr int kMaxPasses = 16;
constexpr int kMaxIters = 32;

struct Arc {
  int32_t j;
  int64_t w;
};
using Adj = std::vector<std::vector<Arc>>;

struct Graph {
  int32_t n = 0;
  Adj adj;
  int64_t two_m = 0;  // total arc weight = 2m (paper's m is half of it)
};

struct Params {
  double tolerance;
  double tolerance_drop;
  double aggregation_tolerance;
  int32_t max_iterations;
  int32_t max_passes;
  int32_t mode;
  int32_t swap_guard;
};

struct Stats {
  int32_t passes;
  int32_t iterations[kMaxPasses];
  int64_t communities[kMaxPasses];
  int64_t moves;
  int64_t arcs_scanned;
  int64_t vertices_affected;
  int64_t iter_moves[kMaxPasses][kMaxIters];
  int64_t iter_gain[kMaxPasses][kMaxIters];
  double seconds;
};

// Batch: each undirected update is listed once and applies to both arcs.
struct Batch {
  int64_t nd;
  const int32_t *du, *dv, *dw;
  int64_t ni;
  const int32_t *iu, *iv, *iw;
};

// Weighted degree K_i: sum of the row's arc weights (Section 3; a self-loop
// arc, which only super-vertices carry, counts once).
int64_t row_weight(const std::vector<Arc>& row) {
  int64_t s = 0;
  for (const Arc& a : row) s += a.w;
  return s;
}

Arc* find_arc(std::vector<Arc>& row, int32_t j) {
  for (Arc& a : row)
    if (a.j == j) return &a;
  return nullptr;
}

uint64_t pair_key(int32_t a, int32_t b) {
  uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
  return ((uint64_t)lo << 32) | hi;
}

// ---------------------------------------------------------------------------
// Batch update (Section 3.4): deletions Δ- then insertions Δ+, both arc
// directions.  All checks happen before any change.
// ---------------------------------------------------------------------------
int32_t apply_batch(Graph& g, const Batch& b) {
  const int32_t n = g.n;
  std::unordered_set<uint64_t> dels, inss;
  for (int64_t k = 0; k < b.nd; ++k) {
    int32_t u = b.du[k], v = b.dv[k], w = b.dw[k];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v || w <= 0) return E_INVAL;
    if (!dels.insert(pair_key(u, v)).second) return E_INVAL;
    Arc* a = find_arc(g.adj[u], v);
    if (!a || a->w < w) return E_NOEDGE;
  }
  for (int64_t k = 0; k < b.ni; ++k) {
    int32_t u = b.iu[k], v = b.iv[k], w = b.iw[k];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v || w <= 0) return E_INVAL;
    if (!inss.insert(pair_key(u, v)).second) return E_INVAL;
  }
  for (int64_t k = 0; k < b.nd; ++k) {
    int32_t ends[2][2] = {{b.du[k], b.dv[k]}, {b.dv[k], b.du[k]}};
    for (auto& e : ends) {
      std::vector<Arc>& row = g.adj[e[0]];
      for (size_t t = 0; t < row.size(); ++t) {
        if (row[t].j != e[1]) continue;
        row[t].w -= b.dw[k];
        if (row[t].w == 0) row.erase(row.begin() + t);
        break;
      }
    }
    g.two_m -= 2 * (int64_t)b.dw[k];
  }
  for (int64_t k = 0; k < b.ni; ++k) {
    int32_t ends[2][2] = {{b.iu[k], b.iv[k]}, {b.iv[k], b.iu[k]}};
    for (auto& e : ends) {
      Arc* a = find_arc(g.adj[e[0]], e[1]);
      if (a)
        a->w += b.iw[k];
      else
        g.adj[e[0]].push_back(Arc{e[1], (int64_t)b.iw[k]});
    }
    g.two_m += 2 * (int64_t)b.iw[k];
  }
  return OK;
}

// ---------------------------------------------------------------------------
// updateWeights (Alg. 7): K and Σ move by the batch's weights, with Σ keyed
// by the endpoint's previous community.  Both endpoints of every undirected
// update are updated, since the batch holds both directions.
// ---------------------------------------------------------------------------
void update_weights(const Batch& b, const int32_t* Cprev, std::vector<int64_t>& K,
                    std::vector<int64_t>& Sig) {
  for (int64_t k = 0; k < b.nd; ++k) {
    int32_t u = b.du[k], v = b.dv[k];
    int64_t w = b.dw[k];
    K[u] -= w;
    K[v] -= w;
    Sig[Cprev[u]] -= w;
    Sig[Cprev[v]] -= w;
  }
  for (int64_t k = 0; k < b.ni; ++k) {
    int32_t u = b.iu[k], v = b.iv[k];
    int64_t w = b.iw[k];
    K[u] += w;
    K[v] += w;
    Sig[Cprev[u]] += w;
    Sig[Cprev[v]] += w;
  }
}

// ---------------------------------------------------------------------------
// Initial marking of affected vertices.
//  DF (Alg. 1): endpoints of deletions inside a community and of
//               insertions across communities.
//  ND (Alg. 2): every vertex.
//  DS (Alg. 3): δV/δE/δC from intra-community deletions and, per insertion
//               source, the best linked community; then neighbours of δE
//               vertices and members of δC communities join δV.  The DS
//               frontier is also its affected range.
// `two_m_prev` is 2m before the batch; all values used here precede
// updateWeights, as in Alg. 3.
// ---------------------------------------------------------------------------
void mark(const Graph& g, int32_t approach, const Batch& b, const int32_t* C, const int64_t* K,
          const int64_t* Sig, int64_t two_m_prev, std::vector<char>& frontier,
          std::vector<char>& in_range, bool& use_range) {
  const int32_t n = g.n;
  frontier.assign(n, 0);
  in_range.assign(n, 1);
  use_range = false;
  if (approach == ND || approach == STATIC) {
    frontier.assign(n, 1);
    return;
  }
  if (approach == DF) {
    for (int64_t k = 0; k < b.nd; ++k)
      if (C[b.du[k]] == C[b.dv[k]]) frontier[b.du[k]] = frontier[b.dv[k]] = 1;
    for (int64_t k = 0; k < b.ni; ++k)
      if (C[b.iu[k]] != C[b.iv[k]]) frontier[b.iu[k]] = frontier[b.iv[k]] = 1;
    return;
  }
  // DS
  std::vector<char> dV(n, 0), dE(n, 0), dC(n, 0);
  for (int64_t k = 0; k < b.nd; ++k) {
    int32_t u = b.du[k], v = b.dv[k];
    if (C[u] != C[v]) continue;
    dV[u] = dE[u] = 1;
    dV[v] = dE[v] = 1;
    dC[C[u]] = 1;
  }
  // insertion arcs grouped by source (both directions of every update)
  std::vector<std::vector<std::pair<int32_t, int64_t>>> by_src(n);
  for (int64_t k = 0; k < b.ni; ++k) {
    by_src[b.iu[k]].push_back({b.iv[k], (int64_t)b.iw[k]});
    by_src[b.iv[k]].push_back({b.iu[k], (int64_t)b.iw[k]});
  }
  std::vector<int64_t> H(n, 0);
  std::vector<int32_t> keys;
  for (int32_t i = 0; i < n; ++i) {
    if (by_src[i].empty()) continue;
    keys.clear();
    for (auto& jw : by_src[i]) {
      int32_t c = C[jw.first];
      if (c == C[i]) continue;
      if (H[c] == 0) keys.push_back(c);
      H[c] += jw.second;
    }
    if (keys.empty()) continue;
    // best linked community by Eq. 2 with K_{i->c} := H[c]; the terms that do
    // not depend on c are dropped, ties go to the lowest community id
    int32_t best = -1;
    int64_t best_s = 0;
    for (int32_t c : keys) {
      int64_t s = two_m_prev * H[c] - K[i] * Sig[c];
      if (best < 0 || s > best_s || (s == best_s && c < best)) {
        best = c;
        best_s = s;
      }
    }
    for (int32_t c : keys) H[c] = 0;
    dV[i] = dE[i] = 1;
    dC[best] = 1;
  }
  for (int32_t i = 0; i < n; ++i) {
    if (dE[i])
      for (const Arc& a : g.adj[i]) dV[a.j] = 1;
    if (dC[C[i]]) dV[i] = 1;
  }
  frontier = dV;
  in_range = dV;
  use_range = true;
}

// ---------------------------------------------------------------------------
// One vertex's local-moving decision (Alg. 5, scanCommunities + best
// community).  K_{i->c} sums the weights of i's arcs into community c,
// skipping a self-loop.  For each neighbouring community c != d = C_i the
// gain is Eq. 2 multiplied by 2m^2:
//     g(c) = 2m (K_{i->c} - K_{i->d}) - K_i (Σ_c - Σ_d + K_i)
// The best c has the largest gain, lowest id on ties; i moves only for a
// strictly positive gain.  The swap guard (on request) keeps a singleton
// from moving into another singleton with a larger id.
// ---------------------------------------------------------------------------
struct Accum {
  std::vector<int64_t> val;
  std::vector<char> seen;
  std::vector<int32_t> keys;
  explicit Accum(int32_t n) : val(n, 0), seen(n, 0) {}
  void add(int32_t c, int64_t w) {
    if (!seen[c]) {
      seen[c] = 1;
      keys.push_back(c);
    }
    val[c] += w;
  }
  void clear() {
    for (int32_t c : keys) {
      val[c] = 0;
      seen[c] = 0;
    }
    keys.clear();
  }
};

struct Choice {
  int32_t c;
  int64_t g;
  bool move;
};

Choice decide(const Graph& g, int32_t i, const std::vector<int32_t>& C,
              const std::vector<int64_t>& K, const std::vector<int64_t>& Sig,
              const std::vector<int32_t>& size, int64_t two_m, bool guard, Accum& H) {
  for (const Arc& a : g.adj[i])
    if (a.j != i) H.add(C[a.j], a.w);
  const int32_t d = C[i];
  const int64_t Kid = H.seen[d] ? H.val[d] : 0;
  Choice best{-1, 0, false};
  for (int32_t c : H.keys) {
    if (c == d) continue;
    int64_t gain = two_m * (H.val[c] - Kid) - K[i] * (Sig[c] - Sig[d] + K[i]);
    if (best.c < 0 || gain > best.g || (gain == best.g && c < best.c)) {
      best.c = c;
      best.g = gain;
    }
  }
  H.clear();
  best.move = best.c >= 0 && best.g > 0;
  if (best.move && guard && size[d] == 1 && size[best.c] == 1 && best.c > d) best.move = false;
  return best;
}

// ---------------------------------------------------------------------------
// louvainMove (Alg. 5).  Each iteration takes the unprocessed vertices
// (the frontier), marks them processed, skips those outside the affected
// range, and lets the rest choose.  A mover updates Σ of both communities,
// changes C and marks its neighbours (other than itself) unprocessed; that
// is the incremental frontier expansion of DF (Section 4.1).
//   SYNC : all choices read the state at iteration start; moves are applied
//          after every choice is made.
//   ASYNC: vertices go in ascending id order and see earlier moves.
// The iteration's ΔQ is the sum of the movers' gains; the phase stops when
// ΔQ <= τ.  Returns the number of iterations run, the stopping one included.
// ---------------------------------------------------------------------------
int32_t local_move(const Graph& g, std::vector<int32_t>& C, const std::vector<int64_t>& K,
                   std::vector<int64_t>& Sig, std::vector<int32_t>& size,
                   std::vector<char>& unprocessed, const std::vector<char>* in_range, double tau,
                   const Params& P, Stats& st, int pass, std::vector<char>* ever) {
  const int32_t n = g.n;
  const bool guard = P.swap_guard != 0;
  Accum H(n);
  std::vector<int32_t> S;
  std::vector<Choice> choice;
  for (int32_t it = 0; it < P.max_iterations; ++it) {
    S.clear();
    for (int32_t i = 0; i < n; ++i) {
      if (!unprocessed[i]) continue;
      unprocessed[i] = 0;
      if (in_range && !(*in_range)[i]) continue;
      S.push_back(i);
    }
    int64_t gain_sum = 0, movers = 0;
    auto apply = [&](int32_t i, const Choice& ch) {
      const int32_t d = C[i];
      Sig[d] -= K[i];
      Sig[ch.c] += K[i];
      size[d] -= 1;
      size[ch.c] += 1;
      C[i] = ch.c;
      gain_sum += ch.g;
      movers += 1;
      for (const Arc& a : g.adj[i])
        if (a.j != i) unprocessed[a.j] = 1;
    };
    for (int32_t i : S) {
      st.arcs_scanned += (int64_t)g.adj[i].size();
      if (ever) (*ever)[i] = 1;
    }
    if (P.mode == SYNC) {
      choice.assign(S.size(), Choice{-1, 0, false});
      for (size_t t = 0; t < S.size(); ++t) choice[t] = decide(g, S[t], C, K, Sig, size, g.two_m, guard, H);
      for (size_t t = 0; t < S.size(); ++t)
        if (choice[t].move) apply(S[t], choice[t]);
    } else {
      for (int32_t i : S) {
        Choice ch = decide(g, i, C, K, Sig, size, g.two_m, guard, H);
        if (ch.move) apply(i, ch);
      }
    }
    st.moves += movers;
    if (pass < kMaxPasses && it < kMaxIters) {
      st.iter_moves[pass][it] = movers;
      st.iter_gain[pass][it] = gain_sum;
    }
    // ΔQ of the iteration = Σ gains / (2m^2) = 2 Σ gains / (2m)^2, in FP64
    const double two_m_d = (double)g.two_m;
    const double dq = (2.0 * (double)gain_sum) / (two_m_d * two_m_d);
    if (dq <= tau) return it + 1;
  }
  return P.max_iterations;
}

// Renumber communities to [0, |Γ|) in ascending order of the old ids (Alg. 4).
int32_t renumber(const std::vector<int32_t>& C, std::vector<int32_t>& newid) {
  const int32_t n = (int32_t)C.size();
  std::vector<char> exists(n, 0);
  for (int32_t c : C) exists[c] = 1;
  newid.assign(n, -1);
  int32_t k = 0;
  for (int32_t c = 0; c < n; ++c)
    if (exists[c]) newid[c] = k++;
  return k;
}

// ---------------------------------------------------------------------------
// Aggregation (Alg. 6): super-vertex c gets one arc to every community d
// linked from any member, weighted by the sum over the members' arcs
// (self-loops included, so the arc (c, c) carries the intra weight).
// ---------------------------------------------------------------------------
Graph aggregate(const Graph& g, const std::vector<int32_t>& C, int32_t nc) {
  std::vector<std::vector<int32_t>> members(nc);
  for (int32_t i = 0; i < g.n; ++i) members[C[i]].push_back(i);
  Graph out;
  out.n = nc;
  out.adj.assign(nc, {});
  out.two_m = g.two_m;
  Accum H(nc);
  for (int32_t c = 0; c < nc; ++c) {
    for (int32_t i : members[c])
      for (const Arc& a : g.adj[i]) H.add(C[a.j], a.w);
    for (int32_t d : H.keys) out.adj[c].push_back(Arc{d, H.val[d]});
    H.clear();
  }
  return out;
}

void now(double& t) {
  t = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Louvain driver (Alg. 4) with the initial steps of Alg. 1-3, or the static
// start (singletons, K from the graph, Σ = K, all vertices affected).
// C, K, Sig hold C^{t-1}, K^{t-1}, Σ^{t-1} on entry (ignored for STATIC) and
// C^t, K^t, Σ^t on return.
// ---------------------------------------------------------------------------
int32_t louvain(const Graph& g0, int32_t approach, const Params& P, const Batch& b, int32_t* Cio,
                int64_t* Kio, int64_t* Sio, Stats& st) {
  double t0, t1;
  now(t0);
  const int32_t n = g0.n;
  if (g0.two_m <= 0) return E_EMPTY;
  if (g0.two_m >= ((int64_t)1 << 31)) return E_OVERFLOW;
  if (P.max_passes < 1 || P.max_passes > kMaxPasses || P.max_iterations < 1 ||
      P.max_iterations > kMaxIters)
    return E_INVAL;
  std::memset(&st, 0, sizeof(Stats));
  std::vector<int32_t> C(n);
  std::vector<int64_t> K(n), Sig(n);
  std::vector<char> frontier, in_range;
  bool use_range = false;
  if (approach == STATIC) {
    for (int32_t i = 0; i < n; ++i) {
      C[i] = i;
      K[i] = row_weight(g0.adj[i]);
      Sig[i] = K[i];
    }
    frontier.assign(n, 1);
  } else {
    for (int32_t i = 0; i < n; ++i) {
      C[i] = Cio[i];
      K[i] = Kio[i];
      Sig[i] = Sio[i];
      if (C[i] < 0 || C[i] >= n) return E_INVAL;
    }
    int64_t ins = 0, del = 0;
    for (int64_t k = 0; k < b.ni; ++k) ins += b.iw[k];
    for (int64_t k = 0; k < b.nd; ++k) del += b.dw[k];
    const int64_t two_m_prev = g0.two_m - 2 * ins + 2 * del;
    mark(g0, approach, b, C.data(), K.data(), Sig.data(), two_m_prev, frontier, in_range,
         use_range);
    update_weights(b, C.data(), K, Sig);
  }
  std::vector<int32_t> size(n, 0);
  for (int32_t i = 0; i < n; ++i) size[C[i]] += 1;

  // Alg. 4: C_top starts as the identity; level 0 is the input graph with
  // C' = C^{t-1}, K' = K^t, Σ' = Σ^t.
  std::vector<int32_t> Ctop(n);
  for (int32_t i = 0; i < n; ++i) Ctop[i] = i;
  Graph level;  // levels >= 1
  const Graph* G = &g0;
  std::vector<int32_t> Cl = C;
  std::vector<int64_t> Kl = K, Sl = Sig;
  std::vector<char> ever(n, 0);
  double tau = P.tolerance;
  bool aggregated = false;
  for (int32_t p = 0; p < P.max_passes; ++p) {
    const std::vector<char>* range = (p == 0 && use_range) ? &in_range : nullptr;
    int32_t li = local_move(*G, Cl, Kl, Sl, size, frontier, range, tau, P, st, p,
                            p == 0 ? &ever : nullptr);
    st.passes = p + 1;
    st.iterations[p] = li;
    if (li <= 1) break;  // converged within one iteration
    std::vector<int32_t> newid;
    const int32_t nc = renumber(Cl, newid);
    st.communities[p] = nc;
    if ((double)nc / (double)G->n > P.aggregation_tolerance) break;  // low shrink
    for (int32_t& c : Cl) c = newid[c];
    for (int32_t& c : Ctop) c = Cl[c];
    Graph next = aggregate(*G, Cl, nc);
    level = std::move(next);
    G = &level;
    Kl.assign(nc, 0);
    for (int32_t c = 0; c < nc; ++c) Kl[c] = row_weight(level.adj[c]);
    Sl = Kl;
    Cl.resize(nc);
    for (int32_t c = 0; c < nc; ++c) Cl[c] = c;
    size.assign(nc, 1);
    frontier.assign(nc, 1);
    tau = tau / P.tolerance_drop;
    aggregated = true;
  }
  for (int32_t& c : Ctop) c = Cl[c];
  for (int32_t i = 0; i < n; ++i) {
    Cio[i] = Ctop[i];
    Kio[i] = K[i];
  }
  if (aggregated) {
    for (int32_t i = 0; i < n; ++i) Sio[i] = 0;
    for (int32_t i = 0; i < n; ++i) Sio[Ctop[i]] += K[i];
  } else {
    for (int32_t i = 0; i < n; ++i) Sio[i] = Sl[i];
  }
  int64_t aff = 0;
  for (char e : ever) aff += e;
  st.vertices_affected = aff;
  now(t1);
  st.seconds = t1 - t0;
  return OK;
}

}  // namespace

// ===========================================================================
// C interface for the tests (ctypes).  Host memory only.
// ===========================================================================
extern "C" {

void* orc_graph_new(int32_t n, int64_t m, const int32_t* u, const int32_t* v, const int32_t* w,
                    int32_t* status) {
  *status = OK;
  if (n < 0) {
    *status = E_INVAL;
    return nullptr;
  }
  Graph* g = new Graph();
  g->n = n;
  g->adj.assign(n, {});
  {  // exact row capacities first (memory only: large inputs would double it)
    std::vector<int64_t> deg(n, 0);
    for (int64_t k = 0; k < m; ++k) {
      if (u[k] >= 0 && u[k] < n) deg[u[k]] += 1;
      if (v[k] >= 0 && v[k] < n) deg[v[k]] += 1;
    }
    for (int32_t i = 0; i < n; ++i) g->adj[i].reserve(deg[i]);
  }
  for (int64_t k = 0; k < m; ++k) {
    if (u[k] < 0 || v[k] < 0 || u[k] >= n || v[k] >= n || u[k] == v[k] || w[k] <= 0) {
      *status = E_INVAL;
      delete g;
      return nullptr;
    }
    g->adj[u[k]].push_back(Arc{v[k], (int64_t)w[k]});
    g->adj[v[k]].push_back(Arc{u[k], (int64_t)w[k]});
    g->two_m += 2 * (int64_t)w[k];
  }
  return g;
}

void orc_graph_free(void* h) { delete static_cast<Graph*>(h); }

int32_t orc_graph_n(void* h) { return static_cast<Graph*>(h)->n; }

int64_t orc_two_m(void* h) { return static_cast<Graph*>(h)->two_m; }

int64_t orc_arc_count(void* h) {
  int64_t s = 0;
  for (auto& r : static_cast<Graph*>(h)->adj) s += (int64_t)r.size();
  return s;
}

// Rows exported sorted by neighbour id: offsets[n+1], col[arcs], w[arcs].
void orc_export(void* h, int64_t* offsets, int32_t* col, int64_t* w) {
  Graph* g = static_cast<Graph*>(h);
  int64_t p = 0;
  for (int32_t i = 0; i < g->n; ++i) {
    offsets[i] = p;
    std::vector<Arc> row = g->adj[i];
    std::sort(row.begin(), row.end(), [](const Arc& a, const Arc& b) { return a.j < b.j; });
    for (const Arc& a : row) {
      col[p] = a.j;
      w[p] = a.w;
      ++p;
    }
  }
  offsets[g->n] = p;
}

int32_t orc_apply_batch(void* h, int64_t nd, const int32_t* du, const int32_t* dv, const int32_t* dw,
                        int64_t ni, const int32_t* iu, const int32_t* iv, const int32_t* iw) {
  Batch b{nd, du, dv, dw, ni, iu, iv, iw};
  return apply_batch(*static_cast<Graph*>(h), b);
}

void orc_weighted_degrees(void* h, int64_t* K) {
  Graph* g = static_cast<Graph*>(h);
  for (int32_t i = 0; i < g->n; ++i) K[i] = row_weight(g->adj[i]);
}

// Eq. 1, community form: Q = Σ_c [σ_c/2m - (Σ_c/2m)^2], evaluated in FP64.
// σ_c sums the arcs whose endpoints both lie in c (an undirected edge is two
// arcs, a self-loop one); Σ_c sums the weighted degrees of c's members.
double orc_modularity(void* h, const int32_t* C) {
  Graph* g = static_cast<Graph*>(h);
  const int32_t n = g->n;
  std::vector<double> sigma_in(n, 0.0), sigma_tot(n, 0.0);
  for (int32_t i = 0; i < n; ++i)
    for (const Arc& a : g->adj[i]) {
      sigma_tot[C[i]] += (double)a.w;
      if (C[a.j] == C[i]) sigma_in[C[i]] += (double)a.w;
    }
  const double two_m = (double)g->two_m;
  double q = 0.0;
  for (int32_t c = 0; c < n; ++c) {
    if (sigma_tot[c] == 0.0 && sigma_in[c] == 0.0) continue;
    const double f = sigma_tot[c] / two_m;
    q += sigma_in[c] / two_m - f * f;
  }
  return q;
}

int32_t orc_mark(void* h, int32_t approach, int64_t nd, const int32_t* du, const int32_t* dv,
                 const int32_t* dw, int64_t ni, const int32_t* iu, const int32_t* iv,
                 const int32_t* iw, const int32_t* C, const int64_t* K, const int64_t* Sig,
                 uint8_t* frontier_out, uint8_t* in_range_out) {
  Graph* g = static_cast<Graph*>(h);
  Batch b{nd, du, dv, dw, ni, iu, iv, iw};
  int64_t ins = 0, del = 0;
  for (int64_t k = 0; k < ni; ++k) ins += iw[k];
  for (int64_t k = 0; k < nd; ++k) del += dw[k];
  std::vector<char> f, r;
  bool use_range;
  mark(*g, approach, b, C, K, Sig, g->two_m - 2 * ins + 2 * del, f, r, use_range);
  for (int32_t i = 0; i < g->n; ++i) {
    frontier_out[i] = (uint8_t)f[i];
    in_range_out[i] = (uint8_t)(use_range ? r[i] : 1);
  }
  return OK;
}

void orc_update_weights(int32_t n, int64_t nd, const int32_t* du, const int32_t* dv,
                        const int32_t* dw, int64_t ni, const int32_t* iu, const int32_t* iv,
                        const int32_t* iw, const int32_t* C, int64_t* K, int64_t* Sig) {
  Batch b{nd, du, dv, dw, ni, iu, iv, iw};
  std::vector<int64_t> Kv(K, K + n), Sv(Sig, Sig + n);
  update_weights(b, C, Kv, Sv);
  std::copy(Kv.begin(), Kv.end(), K);
  std::copy(Sv.begin(), Sv.end(), Sig);
}

int32_t orc_louvain(void* h, int32_t approach, const Params* P, int64_t nd, const int32_t* du,
                    const int32_t* dv, const int32_t* dw, int64_t ni, const int32_t* iu,
                    const int32_t* iv, const int32_t* iw, int32_t* C, int64_t* K, int64_t* Sig,
                    Stats* st) {
  Batch b{nd, du, dv, dw, ni, iu, iv, iw};
  return louvain(*static_cast<Graph*>(h), approach, *P, b, C, K, Sig, *st);
}

// Single local-moving decisions for the listed vertices against a given
// state (used to check sampled vertices of large graphs).
int32_t orc_decide(void* h, const int32_t* C, const int64_t* K, const int64_t* Sig,
                   const int32_t* size, int32_t guard, int64_t count, const int32_t* verts,
                   int32_t* out_c, int64_t* out_g, uint8_t* out_move) {
  Graph* g = static_cast<Graph*>(h);
  const int32_t n = g->n;
  std::vector<int32_t> Cv(C, C + n), Zv(size, size + n);
  std::vector<int64_t> Kv(K, K + n), Sv(Sig, Sig + n);
  Accum H(n);
  for (int64_t t = 0; t < count; ++t) {
    Choice ch = decide(*g, verts[t], Cv, Kv, Sv, Zv, g->two_m, guard != 0, H);
    out_c[t] = ch.c;
    out_g[t] = ch.g;
    out_move[t] = ch.move ? 1 : 0;
  }
  return OK;
}

// Aggregation of a level graph under a dense membership (Alg. 6); returns a
// new graph handle.
void* orc_aggregate(void* h, const int32_t* C, int32_t nc) {
  Graph* g = static_cast<Graph*>(h);
  std::vector<int32_t> Cv(C, C + g->n);
  return new Graph(aggregate(*g, Cv, nc));
}

// Graph from explicit arcs (each arc given; used for aggregated levels with
// self-loops in tests).
void* orc_graph_from_arcs(int32_t n, int64_t arcs, const int32_t* src, const int32_t* dst,
                          const int64_t* w) {
  Graph* g = new Graph();
  g->n = n;
  g->adj.assign(n, {});
  for (int64_t k = 0; k < arcs; ++k) {
    g->adj[src[k]].push_back(Arc{dst[k], w[k]});
    g->two_m += w[k];
  }
  return g;
}

int32_t orc_stats_size(void) { return (int32_t)sizeof(Stats); }
int32_t orc_params_size(void) { return (int32_t)sizeof(Params); }

}  // extern "C"
