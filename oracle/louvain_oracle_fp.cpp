// Sequential reference ("oracle") in the paper's own precision.
//
// TEST INFRASTRUCTURE ONLY, like louvain_oracle.cpp beside it: nothing in the
// product library links, loads or calls this file, and it shares no code
// with the GPU implementation (nor with the integer oracle).
//
// The paper runs with 32-bit floating-point edge weights and 64-bit
// floating-point hashtable values, sums and modularity (Section 5.1.2).
// This file follows the same steps as the integer oracle in that precision:
//   * modularity    -- Eq. 1, community form, sums in FP64;
//   * move gain     -- Eq. 2 as printed: ΔQ(i: d -> c) = (K_{i->c} - K_{i->d}) / m
//                      - K_i (K_i + Σ_c - Σ_d) / (2 m^2), in FP64;
//   * batch update  -- Section 3.4 (deletions, then insertions; weights are
//                      float32, an arc whose weight reaches 0 is removed);
//   * updateWeights -- Alg. 7 (K and Σ in FP64);
//   * DF marking    -- Alg. 1;
//   * driver        -- Alg. 4;
//   * local moving  -- Alg. 5 (SYNC: all decide on the iteration-start
//                      state; ASYNC: ascending id order, each sees earlier
//                      moves);
//   * aggregation   -- Alg. 6: super-vertex arc weights are summed in FP64
//                      (the hashtable) and stored as float32 edge weights.
// The best community has the largest ΔQ, the lowest id on ties; a vertex
// moves only for ΔQ > 0; a singleton does not join a singleton of larger id
// (the same swap guard as the integer oracle).  The iteration stops when the
// movers' ΔQ sum to at most τ.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_set>
#include <vector>

namespace {

enum : int32_t { OK = 0, E_INVAL = -1, E_NOEDGE = -2, E_EMPTY = -5 };
enum : int32_t { STATIC = 0, DF = 3 };
enum : int32_t { SYNC = 0, ASYNC = 1 };
constexpr int kMaxPasses = 16;
constexpr int kMaxIters = 32;

struct ArcF {
  int32_t j;
  float w;
};

struct GraphF {
  int32_t n = 0;
  std::vector<std::vector<ArcF>> adj;
  double two_m = 0.0;  // Σ of arc weights (both directions), FP64
};

struct ParamsF {
  double tolerance;
  double tolerance_drop;
  double aggregation_tolerance;
  int32_t max_iterations;
  int32_t max_passes;
  int32_t mode;
  int32_t swap_guard;
};

struct StatsF {
  int32_t passes;
  int32_t iterations[kMaxPasses];
  int64_t communities[kMaxPasses];
  int64_t moves;
  int64_t arcs_scanned;
  int64_t iter_moves[kMaxPasses][kMaxIters];
  double iter_dq[kMaxPasses][kMaxIters];
  double seconds;
};

// K_i: the row's weights summed in FP64 (a self-loop counts once).
double row_sum(const std::vector<ArcF>& row) {
  double s = 0.0;
  for (const ArcF& a : row) s += static_cast<double>(a.w);
  return s;
}

double total_weight(const GraphF& g) {
  double s = 0.0;
  for (const auto& row : g.adj) s += row_sum(row);
  return s;
}

ArcF* find(std::vector<ArcF>& row, int32_t j) {
  for (ArcF& a : row)
    if (a.j == j) return &a;
  return nullptr;
}

bool weight_ok(float w) { return std::isfinite(w) && w > 0.0f; }

// Section 3.4 in float32 weights: every check first, then deletions, then
// insertions, both directions; 2m is the FP64 total of the arc weights.
int32_t apply_batch_f(GraphF& g, int64_t nd, const int32_t* du, const int32_t* dv, const float* dw, int64_t ni,
                      const int32_t* iu, const int32_t* iv, const float* iw) {
  std::unordered_set<uint64_t> seen_d, seen_i;
  auto key = [](int32_t a, int32_t b) {
    return (static_cast<uint64_t>(static_cast<uint32_t>(std::min(a, b))) << 32) | static_cast<uint32_t>(std::max(a, b));
  };
  for (int64_t k = 0; k < nd; ++k) {
    if (du[k] < 0 || dv[k] < 0 || du[k] >= g.n || dv[k] >= g.n || du[k] == dv[k] || !weight_ok(dw[k])) return E_INVAL;
    if (!seen_d.insert(key(du[k], dv[k])).second) return E_INVAL;
    ArcF* a = find(g.adj[du[k]], dv[k]);
    if (!a || a->w < dw[k]) return E_NOEDGE;
  }
  for (int64_t k = 0; k < ni; ++k) {
    if (iu[k] < 0 || iv[k] < 0 || iu[k] >= g.n || iv[k] >= g.n || iu[k] == iv[k] || !weight_ok(iw[k])) return E_INVAL;
    if (!seen_i.insert(key(iu[k], iv[k])).second) return E_INVAL;
  }
  for (int64_t k = 0; k < nd; ++k) {
    const int32_t ends[2][2] = {{du[k], dv[k]}, {dv[k], du[k]}};
    for (auto& e : ends) {
      auto& row = g.adj[e[0]];
      for (size_t t = 0; t < row.size(); ++t) {
        if (row[t].j != e[1]) continue;
        row[t].w -= dw[k];
        if (row[t].w <= 0.0f) row.erase(row.begin() + static_cast<long>(t));
        break;
      }
    }
  }
  for (int64_t k = 0; k < ni; ++k) {
    const int32_t ends[2][2] = {{iu[k], iv[k]}, {iv[k], iu[k]}};
    for (auto& e : ends) {
      ArcF* a = find(g.adj[e[0]], e[1]);
      if (a)
        a->w += iw[k];
      else
        g.adj[e[0]].push_back(ArcF{e[1], iw[k]});
    }
  }
  g.two_m = total_weight(g);
  return OK;
}

// Dense accumulator (the paper's collision-free hashtable), FP64 values.
struct AccF {
  std::vector<double> val;
  std::vector<char> seen;
  std::vector<int32_t> keys;
  explicit AccF(int32_t n) : val(n, 0.0), seen(n, 0) {}
  void add(int32_t c, double w) {
    if (!seen[c]) {
      seen[c] = 1;
      keys.push_back(c);
    }
    val[c] += w;
  }
  void clear() {
    for (int32_t c : keys) {
      val[c] = 0.0;
      seen[c] = 0;
    }
    keys.clear();
  }
};

struct ChoiceF {
  int32_t c;
  double dq;
  bool move;
};

// Alg. 5 for one vertex with Eq. 2 in FP64.
ChoiceF decide_f(const GraphF& g, int32_t i, const std::vector<int32_t>& C, const std::vector<double>& K,
                 const std::vector<double>& Sig, const std::vector<int32_t>& size, bool guard, AccF& H) {
  for (const ArcF& a : g.adj[i])
    if (a.j != i) H.add(C[a.j], static_cast<double>(a.w));
  const int32_t d = C[i];
  const double kid = H.seen[d] ? H.val[d] : 0.0;
  const double m = g.two_m / 2.0;
  ChoiceF best{-1, 0.0, false};
  for (int32_t c : H.keys) {
    if (c == d) continue;
    const double dq = (H.val[c] - kid) / m - K[i] * (K[i] + Sig[c] - Sig[d]) / (2.0 * m * m);
    if (best.c < 0 || dq > best.dq || (dq == best.dq && c < best.c)) {
      best.c = c;
      best.dq = dq;
    }
  }
  H.clear();
  best.move = best.c >= 0 && best.dq > 0.0;
  if (best.move && guard && size[d] == 1 && size[best.c] == 1 && best.c > d) best.move = false;
  return best;
}

int32_t local_move_f(const GraphF& g, std::vector<int32_t>& C, const std::vector<double>& K, std::vector<double>& Sig,
                     std::vector<int32_t>& size, std::vector<char>& unprocessed, double tau, const ParamsF& P,
                     StatsF& st, int pass) {
  const int32_t n = g.n;
  AccF H(n);
  std::vector<int32_t> S;
  std::vector<ChoiceF> choice;
  for (int32_t it = 0; it < P.max_iterations; ++it) {
    S.clear();
    for (int32_t i = 0; i < n; ++i)
      if (unprocessed[i]) {
        unprocessed[i] = 0;
        S.push_back(i);
      }
    double dq_sum = 0.0;
    int64_t movers = 0;
    auto apply = [&](int32_t i, const ChoiceF& ch) {
      const int32_t d = C[i];
      Sig[d] -= K[i];
      Sig[ch.c] += K[i];
      size[d] -= 1;
      size[ch.c] += 1;
      C[i] = ch.c;
      dq_sum += ch.dq;
      movers += 1;
      for (const ArcF& a : g.adj[i])
        if (a.j != i) unprocessed[a.j] = 1;
    };
    for (int32_t i : S) st.arcs_scanned += static_cast<int64_t>(g.adj[i].size());
    if (P.mode == SYNC) {
      choice.assign(S.size(), ChoiceF{-1, 0.0, false});
      for (size_t t = 0; t < S.size(); ++t) choice[t] = decide_f(g, S[t], C, K, Sig, size, P.swap_guard != 0, H);
      for (size_t t = 0; t < S.size(); ++t)
        if (choice[t].move) apply(S[t], choice[t]);
    } else {
      for (int32_t i : S) {
        const ChoiceF ch = decide_f(g, i, C, K, Sig, size, P.swap_guard != 0, H);
        if (ch.move) apply(i, ch);
      }
    }
    st.moves += movers;
    if (pass < kMaxPasses && it < kMaxIters) {
      st.iter_moves[pass][it] = movers;
      st.iter_dq[pass][it] = dq_sum;
    }
    if (dq_sum <= tau) return it + 1;
  }
  return P.max_iterations;
}

// Alg. 6: super-vertex c's arc to d weighs the FP64 sum over its members'
// arcs (self-loops included), stored as a float32 edge weight.
GraphF aggregate_f(const GraphF& g, const std::vector<int32_t>& C, int32_t nc) {
  std::vector<std::vector<int32_t>> members(nc);
  for (int32_t i = 0; i < g.n; ++i) members[C[i]].push_back(i);
  GraphF out;
  out.n = nc;
  out.adj.assign(nc, {});
  AccF H(nc);
  for (int32_t c = 0; c < nc; ++c) {
    for (int32_t i : members[c])
      for (const ArcF& a : g.adj[i]) H.add(C[a.j], static_cast<double>(a.w));
    for (int32_t d : H.keys) out.adj[c].push_back(ArcF{d, static_cast<float>(H.val[d])});
    H.clear();
  }
  out.two_m = total_weight(out);
  return out;
}

int32_t louvain_f(const GraphF& g0, int32_t approach, const ParamsF& P, int64_t nd, const int32_t* du,
                  const int32_t* dv, const float* dw, int64_t ni, const int32_t* iu, const int32_t* iv,
                  const float* iw, int32_t* Cio, double* Kio, double* Sio, StatsF& st) {
  const auto t0 = std::chrono::steady_clock::now();
  const int32_t n = g0.n;
  if (!(g0.two_m > 0.0)) return E_EMPTY;
  if (P.max_passes < 1 || P.max_passes > kMaxPasses || P.max_iterations < 1 || P.max_iterations > kMaxIters)
    return E_INVAL;
  std::memset(&st, 0, sizeof(StatsF));
  std::vector<int32_t> C(n);
  std::vector<double> K(n), Sig(n);
  std::vector<char> frontier(n, 0);
  if (approach == STATIC) {
    for (int32_t i = 0; i < n; ++i) {
      C[i] = i;
      K[i] = row_sum(g0.adj[i]);
      Sig[i] = K[i];
      frontier[i] = 1;
    }
  } else {
    for (int32_t i = 0; i < n; ++i) {
      C[i] = Cio[i];
      K[i] = Kio[i];
      Sig[i] = Sio[i];
      if (C[i] < 0 || C[i] >= n) return E_INVAL;
    }
    // DF marking (Alg. 1) and updateWeights (Alg. 7), both on C^{t-1}
    for (int64_t k = 0; k < nd; ++k) {
      if (C[du[k]] == C[dv[k]]) frontier[du[k]] = frontier[dv[k]] = 1;
      K[du[k]] -= dw[k];
      K[dv[k]] -= dw[k];
      Sig[C[du[k]]] -= dw[k];
      Sig[C[dv[k]]] -= dw[k];
    }
    for (int64_t k = 0; k < ni; ++k) {
      if (C[iu[k]] != C[iv[k]]) frontier[iu[k]] = frontier[iv[k]] = 1;
      K[iu[k]] += iw[k];
      K[iv[k]] += iw[k];
      Sig[C[iu[k]]] += iw[k];
      Sig[C[iv[k]]] += iw[k];
    }
  }
  std::vector<int32_t> size(n, 0);
  for (int32_t i = 0; i < n; ++i) size[C[i]] += 1;
  std::vector<int32_t> Ctop(n);
  for (int32_t i = 0; i < n; ++i) Ctop[i] = i;
  GraphF level;
  const GraphF* G = &g0;
  std::vector<int32_t> Cl = C;
  std::vector<double> Kl = K, Sl = Sig;
  double tau = P.tolerance;
  bool aggregated = false;
  for (int32_t p = 0; p < P.max_passes; ++p) {
    const int32_t li = local_move_f(*G, Cl, Kl, Sl, size, frontier, tau, P, st, p);
    st.passes = p + 1;
    st.iterations[p] = li;
    if (li <= 1) break;
    std::vector<char> exists(G->n, 0);
    for (int32_t c : Cl) exists[c] = 1;
    std::vector<int32_t> newid(G->n, -1);
    int32_t nc = 0;
    for (int32_t c = 0; c < G->n; ++c)
      if (exists[c]) newid[c] = nc++;
    st.communities[p] = nc;
    if (static_cast<double>(nc) / static_cast<double>(G->n) > P.aggregation_tolerance) break;
    for (int32_t& c : Cl) c = newid[c];
    for (int32_t& c : Ctop) c = Cl[c];
    level = aggregate_f(*G, Cl, nc);
    G = &level;
    Kl.assign(nc, 0.0);
    for (int32_t c = 0; c < nc; ++c) Kl[c] = row_sum(level.adj[c]);
    Sl = Kl;
    Cl.resize(nc);
    for (int32_t c = 0; c < nc; ++c) Cl[c] = c;
    size.assign(nc, 1);
    frontier.assign(nc, 1);
    tau /= P.tolerance_drop;
    aggregated = true;
  }
  for (int32_t i = 0; i < n; ++i) {
    Cio[i] = Cl[Ctop[i]];
    Kio[i] = K[i];
  }
  if (aggregated) {
    for (int32_t i = 0; i < n; ++i) Sio[i] = 0.0;
    for (int32_t i = 0; i < n; ++i) Sio[Cio[i]] += K[i];
  } else {
    for (int32_t i = 0; i < n; ++i) Sio[i] = Sl[i];
  }
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return OK;
}

}  // namespace

extern "C" {

void* orcf_graph_new(int32_t n, int64_t m, const int32_t* u, const int32_t* v, const float* w, int32_t* status) {
  *status = OK;
  for (int64_t k = 0; k < m; ++k)
    if (u[k] < 0 || v[k] < 0 || u[k] >= n || v[k] >= n || u[k] == v[k] || !weight_ok(w[k])) {
      *status = E_INVAL;
      return nullptr;
    }
  GraphF* g = new GraphF();
  g->n = n;
  g->adj.assign(n, {});
  for (int64_t k = 0; k < m; ++k) {
    g->adj[u[k]].push_back(ArcF{v[k], w[k]});
    g->adj[v[k]].push_back(ArcF{u[k], w[k]});
  }
  g->two_m = total_weight(*g);
  return g;
}

void orcf_graph_free(void* h) { delete static_cast<GraphF*>(h); }

double orcf_two_m(void* h) { return static_cast<GraphF*>(h)->two_m; }

int32_t orcf_apply_batch(void* h, int64_t nd, const int32_t* du, const int32_t* dv, const float* dw, int64_t ni,
                         const int32_t* iu, const int32_t* iv, const float* iw) {
  return apply_batch_f(*static_cast<GraphF*>(h), nd, du, dv, dw, ni, iu, iv, iw);
}

void orcf_degrees(void* h, double* K) {
  const GraphF& g = *static_cast<GraphF*>(h);
  for (int32_t i = 0; i < g.n; ++i) K[i] = row_sum(g.adj[i]);
}

// Eq. 1 (community form): Q = Σ_c [σ_c / 2m - (Σ_c / 2m)^2], sums in FP64.
double orcf_modularity(void* h, const int32_t* C) {
  const GraphF& g = *static_cast<GraphF*>(h);
  std::vector<double> in(g.n, 0.0), tot(g.n, 0.0);
  for (int32_t i = 0; i < g.n; ++i)
    for (const ArcF& a : g.adj[i]) {
      tot[C[i]] += static_cast<double>(a.w);
      if (C[a.j] == C[i]) in[C[i]] += static_cast<double>(a.w);
    }
  double q = 0.0;
  for (int32_t c = 0; c < g.n; ++c) {
    const double f = tot[c] / g.two_m;
    q += in[c] / g.two_m - f * f;
  }
  return q;
}

// Single decisions against a given state: target, ΔQ and whether it moves.
void orcf_decide(void* h, const int32_t* C, const double* K, const double* Sig, const int32_t* size, int32_t guard,
                 int64_t count, const int32_t* verts, int32_t* out_c, double* out_dq, uint8_t* out_move) {
  const GraphF& g = *static_cast<GraphF*>(h);
  std::vector<int32_t> Cv(C, C + g.n), Zv(size, size + g.n);
  std::vector<double> Kv(K, K + g.n), Sv(Sig, Sig + g.n);
  AccF H(g.n);
  for (int64_t t = 0; t < count; ++t) {
    const ChoiceF ch = decide_f(g, verts[t], Cv, Kv, Sv, Zv, guard != 0, H);
    out_c[t] = ch.c;
    out_dq[t] = ch.dq;
    out_move[t] = ch.move ? 1 : 0;
  }
}

int32_t orcf_louvain(void* h, int32_t approach, const ParamsF* P, int64_t nd, const int32_t* du, const int32_t* dv,
                     const float* dw, int64_t ni, const int32_t* iu, const int32_t* iv, const float* iw, int32_t* C,
                     double* K, double* Sig, StatsF* st) {
  if (approach != STATIC && approach != DF) return E_INVAL;
  return louvain_f(*static_cast<GraphF*>(h), approach, *P, nd, du, dv, dw, ni, iu, iv, iw, C, K, Sig, *st);
}

int32_t orcf_stats_size(void) { return static_cast<int32_t>(sizeof(StatsF)); }

int64_t orcf_arc_count(void* h) {
  int64_t a = 0;
  for (const auto& row : static_cast<GraphF*>(h)->adj) a += static_cast<int64_t>(row.size());
  return a;
}

// The adjacency as CSR, every row sorted by neighbour.
void orcf_export(void* h, int64_t* off, int32_t* col, float* w) {
  const GraphF& g = *static_cast<GraphF*>(h);
  off[0] = 0;
  for (int32_t i = 0; i < g.n; ++i) {
    std::vector<ArcF> row = g.adj[i];
    std::sort(row.begin(), row.end(), [](const ArcF& a, const ArcF& b) { return a.j < b.j; });
    int64_t o = off[i];
    for (const ArcF& a : row) {
      col[o] = a.j;
      w[o] = a.w;
      ++o;
    }
    off[i + 1] = o;
  }
}

}  // extern "C"
