"""Pins of the paper-precision oracle (float32 weights, FP64 sums:
oracle/louvain_oracle_fp.cpp) against what the paper and the mathematics
fix, independently of its own code:

* Eq. 1: closed forms of two cliques joined by a bridge and of a ring of
  cliques (modularity is invariant under a uniform weight scale), and
  Newman's pairwise form in exact rationals of the float32 weights;
* Eq. 2: for single moves from random states, the predicted ΔQ equals the
  change of Eq. 1 modularity;
* Louvain: below the brute-force maximum on tiny weighted graphs, and it
  finds the cliques of a weighted two-clique graph;
* integer-valued weights: the same modularity as the integer oracle;
* batches and updateWeights: K and Sigma equal a recomputation from the
  updated edge list."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from paper_2404_19634_amd import workloads as W


def _scaled(e, s):
    return W.Edges(e.n, e.u, e.v, (e.w.astype(np.float64) * s).astype(np.float32))


def _pairwise_q(e, C):
    """Newman's pairwise form (1/2m) Σ_ij [A_ij - K_i K_j / 2m] δ(C_i, C_j),
    exact rationals of the float32 weights."""
    n = e.n
    A = {}
    K = [Fraction(0)] * n
    for u, v, w in zip(e.u.tolist(), e.v.tolist(), np.asarray(e.w, np.float32).tolist()):
        x = Fraction(float(np.float32(w)))
        A[(u, v)] = A.get((u, v), 0) + x
        A[(v, u)] = A.get((v, u), 0) + x
        K[u] += x
        K[v] += x
    two_m = sum(K)
    q = Fraction(0)
    for i in range(n):
        for j in range(n):
            if C[i] == C[j]:
                q += A.get((i, j), 0) - K[i] * K[j] / two_m
    return q / two_m


@pytest.mark.parametrize("scale", [1.0, 0.37, 5.5])
def test_modularity_closed_forms(orc, scale):
    k = 5
    e = _scaled(W.two_cliques_bridge(k), scale)
    G = orc.GraphF.from_edges(e)
    m = k * (k - 1) + 1
    C = np.array([0] * k + [1] * k, dtype=np.int32)
    assert abs(G.modularity(C) - (0.5 - 1.0 / m)) <= 1e-12
    r = 10
    e = _scaled(W.ring_of_cliques(r, k), scale)
    G = orc.GraphF.from_edges(e)
    C = (np.arange(r * k) // k).astype(np.int32)
    assert abs(G.modularity(C) - (1 - 2 / (k * (k - 1) + 2) - 1 / r)) <= 1e-12


def test_modularity_pairwise_form(orc):
    rng = np.random.default_rng(3)
    for t in range(4):
        e = W.real_weights(W.random_small_graph(12, 30, 40 + t), 50 + t)
        G = orc.GraphF.from_edges(e)
        C = rng.integers(0, 4, e.n).astype(np.int32)
        assert abs(G.modularity(C) - float(_pairwise_q(e, C))) <= 1e-12


def test_integer_weights_give_the_integer_oracles_modularity(orc):
    rng = np.random.default_rng(5)
    e = W.random_small_graph(300, 1500, 6, max_w=5)
    ef = W.Edges(e.n, e.u, e.v, e.w.astype(np.float32))
    for _ in range(3):
        C = rng.integers(0, 20, e.n).astype(np.int32)
        assert abs(orc.GraphF.from_edges(ef).modularity(C) - orc.Graph.from_edges(e).modularity(C)) <= 1e-12


def test_gain_equals_modularity_change(orc):
    """Eq. 2 against Eq. 1: for single moves out of random states (with
    Sigma consistent with the state), the predicted ΔQ is the change of
    modularity."""
    rng = np.random.default_rng(7)
    e = W.real_weights(W.random_small_graph(200, 900, 8), 9)
    G = orc.GraphF.from_edges(e)
    K = G.degrees()
    checked = 0
    for trial in range(5):
        C = rng.integers(0, 25, e.n).astype(np.int32)
        S = np.bincount(C, weights=K, minlength=e.n)
        size = np.bincount(C, minlength=e.n).astype(np.int32)
        verts = rng.choice(e.n, 40, replace=False).astype(np.int32)
        oc, odq, om = G.decide(C, K, S, size, verts, guard=0)
        q0 = G.modularity(C)
        for v, c, dq, mv in zip(verts, oc, odq, om):
            if c < 0:
                continue
            C2 = C.copy()
            C2[v] = c
            assert abs((G.modularity(C2) - q0) - dq) <= 1e-12, (v, c)
            checked += 1
    assert checked > 50


def _brute_max(e):
    best = -1.0
    n = e.n
    G = None
    import oracle
    G = oracle.GraphF.from_edges(e)
    # every set partition via restricted growth strings
    def rgs(k, a, m):
        if k == n:
            yield a[:]
            return
        for x in range(m + 2):
            a.append(x)
            yield from rgs(k + 1, a, max(m, x))
            a.pop()
    for a in rgs(1, [0], 0):
        best = max(best, G.modularity(np.array(a, dtype=np.int32)))
    return best


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_louvain_below_brute_force_maximum(orc, seed):
    e = W.real_weights(W.random_small_graph(8, 14, 60 + seed), 70 + seed)
    G = orc.GraphF.from_edges(e)
    qmax = _brute_max(e)
    for mode in ("sync", "async"):
        C = G.louvain("static", mode=mode, tolerance=0.0)[0]
        assert G.modularity(C) <= qmax + 1e-12


def test_louvain_finds_weighted_cliques(orc):
    k = 6
    e = W.two_cliques_bridge(k)
    w = np.where((e.u < k) == (e.v < k), 2.5, 0.3).astype(np.float32)
    e = W.Edges(e.n, e.u, e.v, w)
    G = orc.GraphF.from_edges(e)
    for mode in ("sync", "async"):
        C = G.louvain("static", mode=mode)[0]
        assert len(set(C[:k].tolist())) == 1 and len(set(C[k:].tolist())) == 1 and C[0] != C[k]


def test_batches_and_weight_updates(orc):
    e = W.real_weights(W.random_small_graph(400, 1600, 11), 12)
    G = orc.GraphF.from_edges(e)
    C, K, S, _ = G.louvain("static", mode="async")
    cur = e
    for t in range(3):
        b = W.real_batch(W.random_batch(cur, 60, 20 + t), cur, 30 + t)
        assert G.apply_batch(b) == 0
        C, K, S, st = G.louvain("df", batch=b, state=(C, K, S), mode="async")
        cur = W.apply_batch_np(cur, b)
        Kref = (np.bincount(cur.u, weights=cur.w.astype(np.float64), minlength=e.n) +
                np.bincount(cur.v, weights=cur.w.astype(np.float64), minlength=e.n))
        assert np.allclose(K, Kref, rtol=1e-9, atol=1e-9)
        assert np.allclose(G.degrees(), Kref, rtol=1e-9, atol=1e-9)
        assert np.allclose(S, np.bincount(C, weights=K, minlength=e.n), rtol=1e-9, atol=1e-9)
        assert abs(G.two_m - Kref.sum()) <= 1e-9 * Kref.sum()
    # errors leave the graph as it was
    z, zf = np.zeros(0, np.int32), np.zeros(0, np.float32)
    present = set(zip(cur.u.tolist(), cur.v.tolist()))
    a, c = next((a, c) for a in range(400) for c in range(a + 1, 400) if (a, c) not in present)
    bad = W.Batch(np.array([a], np.int32), np.array([c], np.int32), np.array([1.0], np.float32), z, z, zf)
    two_m = G.two_m
    assert G.apply_batch(bad) == orc.E_NOEDGE and G.two_m == two_m
