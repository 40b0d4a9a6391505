"""Pins of the sequential oracle against what the paper and the mathematics
fix: closed-form modularities, the pairwise (Newman) form of Eq. 1, the
exact single-move identity behind Eq. 2, exhaustive maximum modularity on
tiny graphs, the marking rules of Alg. 1-3, the weight updates of Alg. 7 and
the invariants of aggregation (Alg. 6)."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2404_19634_amd import workloads as W
from tests import exact as X


def _graph(orc, e):
    return orc.Graph.from_edges(e)


# --------------------------------------------------------------------------
# Eq. 1
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_modularity_matches_pairwise_form(orc, seed):
    rng = np.random.default_rng(seed)
    e = W.random_small_graph(12, 25, seed, max_w=5)
    G = _graph(orc, e)
    src, dst, w = X.arcs_of(e)
    for _ in range(4):
        C = rng.integers(0, 4, e.n)
        q = G.modularity(C)
        assert abs(q - float(X.modularity_pairwise(e.n, src, dst, w, C))) < 1e-13


def test_modularity_singletons_and_one_community(orc):
    e = W.random_small_graph(20, 60, 3, max_w=3)
    G = _graph(orc, e)
    src, dst, w = X.arcs_of(e)
    K = X.degrees(e.n, src, w)
    two_m = int(K.sum())
    q_single = G.modularity(np.arange(e.n))
    assert q_single == pytest.approx(-float((K.astype(np.float64) ** 2).sum()) / two_m ** 2, abs=1e-15)
    assert abs(G.modularity(np.zeros(e.n, dtype=np.int32))) < 1e-15


@pytest.mark.parametrize("k", [3, 5, 8])
def test_modularity_two_cliques_bridge_closed_form(orc, k):
    e = W.two_cliques_bridge(k)
    G = _graph(orc, e)
    m = k * (k - 1) + 1
    C = np.repeat([0, 1], k)
    assert G.modularity(C) == pytest.approx(0.5 - 1.0 / m, abs=1e-15)


@pytest.mark.parametrize("r,k", [(10, 5), (6, 4), (12, 6)])
def test_modularity_ring_of_cliques_closed_form(orc, r, k):
    e = W.ring_of_cliques(r, k)
    G = _graph(orc, e)
    C = np.repeat(np.arange(r), k)
    assert G.modularity(C) == pytest.approx(1 - 2.0 / (k * (k - 1) + 2) - 1.0 / r, abs=1e-14)
    if r % 2 == 0:
        Cp = np.repeat(np.arange(r) // 2, k)
        assert G.modularity(Cp) == pytest.approx(1 - 1.0 / (k * (k - 1) + 2) - 2.0 / r, abs=1e-14)


# --------------------------------------------------------------------------
# Eq. 2: the integer gain is 2m^2 ΔQ exactly, and the chosen community is
# the exact argmax over neighbouring communities.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_gain_identity_and_argmax(orc, seed):
    rng = np.random.default_rng(100 + seed)
    e = W.random_small_graph(14, 30, seed, max_w=4)
    G = _graph(orc, e)
    src, dst, w = X.arcs_of(e)
    K = X.degrees(e.n, src, w)
    two_m = int(K.sum())
    C = rng.integers(0, 5, e.n).astype(np.int32)
    Sig = np.bincount(C, weights=K, minlength=e.n).astype(np.int64)
    size = np.bincount(C, minlength=e.n).astype(np.int32)
    verts = np.arange(e.n, dtype=np.int32)
    oc, og, om = G.decide(C, K, Sig, size, verts, guard=0)
    q0 = X.qnum(e.n, src, dst, w, C)
    for i in range(e.n):
        nbr = set(int(C[j]) for j in dst[src == i]) - {int(C[i])}
        if not nbr:
            assert oc[i] == -1 and not om[i]
            continue
        # exact ΔQ·(2m)^2 for every candidate, by recomputing Q
        best_c, best_d = None, None
        for c in sorted(nbr):
            C2 = C.copy()
            C2[i] = c
            d = X.qnum(e.n, src, dst, w, C2) - q0
            if best_d is None or d > best_d:
                best_c, best_d = c, d
        assert oc[i] == best_c
        assert 2 * int(og[i]) == best_d          # Qnum' - Qnum = 2 g
        assert bool(om[i]) == (best_d > 0)


def test_swap_guard_blocks_only_singleton_to_larger_singleton(orc):
    # path 0-1-2, all singletons: 0 prefers 1's community but 1 > 0 -> blocked;
    # 2 prefers 1 < 2 -> allowed
    e = W.Edges(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1, 1], np.int32))
    G = _graph(orc, e)
    K = np.array([1, 2, 1], np.int64)
    C = np.arange(3, dtype=np.int32)
    oc, og, om = G.decide(C, K, K.copy(), np.ones(3, np.int32), np.arange(3, dtype=np.int32), guard=1)
    assert oc.tolist() == [1, 0, 1]
    assert om.tolist() == [False, True, True]
    oc2, og2, om2 = G.decide(C, K, K.copy(), np.ones(3, np.int32), np.arange(3, dtype=np.int32), guard=0)
    assert om2.tolist() == [True, True, True]


# --------------------------------------------------------------------------
# Local-moving and the whole driver on graphs with known optima
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("k", [4, 5, 7])
def test_two_cliques_bridge_found(orc, mode, k):
    e = W.two_cliques_bridge(k)
    G = _graph(orc, e)
    C, K, S, st = G.louvain("static", mode=mode)
    assert len(set(C[:k].tolist())) == 1 and len(set(C[k:].tolist())) == 1 and C[0] != C[-1]
    assert G.modularity(C) == pytest.approx(0.5 - 1.0 / (k * (k - 1) + 1), abs=1e-15)


@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("r,k", [(10, 5), (8, 6), (5, 4)])
def test_ring_of_cliques_found(orc, mode, r, k):
    assert r < k * (k - 1) + 2
    e = W.ring_of_cliques(r, k)
    G = _graph(orc, e)
    C, K, S, st = G.louvain("static", mode=mode)
    labels = C.reshape(r, k)
    assert all(len(set(row.tolist())) == 1 for row in labels)
    assert len(set(labels[:, 0].tolist())) == r
    assert G.modularity(C) == pytest.approx(1 - 2.0 / (k * (k - 1) + 2) - 1.0 / r, abs=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_tiny_graphs_vs_bruteforce_maximum(orc, seed):
    n = 8 + seed % 2
    e = W.random_small_graph(n, 14, 40 + seed, max_w=3)
    G = _graph(orc, e)
    src, dst, w = X.arcs_of(e)
    qmax, lab = X.max_modularity_bruteforce(n, src, dst, w)
    assert float(qmax) == pytest.approx(G.modularity(lab), abs=1e-14)
    for mode in ("sync", "async"):
        C, K, S, st = G.louvain("static", mode=mode, tolerance=0.0)
        q = G.modularity(C)
        assert q <= float(qmax) + 1e-14
        assert q > 0.6 * float(qmax)


@pytest.mark.parametrize("guard", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_async_pass_gain_sum_is_exact_modularity_change(orc, seed, guard):
    """In ASYNC mode every move is applied to the current state, so over a
    single pass the exact change of Q·(2m)^2 equals twice the sum of the
    recorded gains (Eq. 2 scaled by 2m^2), iteration by iteration."""
    e = W.random_small_graph(30, 70, 70 + seed, max_w=3)
    G = _graph(orc, e)
    src, dst, w = X.arcs_of(e)
    q_prev = X.qnum(e.n, src, dst, w, np.arange(e.n))
    for t in range(1, 8):
        C, K, S, st = G.louvain("static", mode="async", tolerance=0.0, max_passes=1,
                                max_iterations=t, swap_guard=guard)
        gains = st["iter_gain"][0]
        q = X.qnum(e.n, src, dst, w, C)
        assert q - X.qnum(e.n, src, dst, w, np.arange(e.n)) == 2 * sum(gains)
        assert q >= q_prev
        q_prev = q
        if st["iterations"][0] < t:
            break


@pytest.mark.parametrize("seed", range(4))
def test_sync_first_iteration_is_jacobi(orc, seed):
    """One SYNC iteration from singletons moves exactly the vertices whose
    exact best ΔQ is positive (and not vetoed by the swap guard), each to
    its exact best community, all decided on the initial state."""
    e = W.random_small_graph(16, 30, 90 + seed, max_w=3)
    G = _graph(orc, e)
    src, dst, w = X.arcs_of(e)
    C, K, S, st = G.louvain("static", mode="sync", max_iterations=1, max_passes=1)
    C0 = np.arange(e.n)
    q0 = X.qnum(e.n, src, dst, w, C0)
    for i in range(e.n):
        best_c, best_d = int(i), 0
        for c in sorted(set(int(j) for j in dst[src == i])):
            C2 = C0.copy()
            C2[i] = c
            d = X.qnum(e.n, src, dst, w, C2) - q0
            if best_c == i or d > best_d:
                best_c, best_d = c, d
        moves = best_c != i and best_d > 0 and not (best_c > i)   # all singletons: guard
        assert C[i] == (best_c if moves else i)


def test_gain_sum_and_convergence_rule(orc):
    e = W.config1_sbm()
    G = _graph(orc, e)
    for mode in ("sync", "async"):
        C, K, S, st = G.louvain("static", mode=mode)
        tau = 1e-2
        for p in range(st["passes"]):
            gains = st["iter_gain"][p]
            assert sum(st["iter_moves"][p]) >= 0
            for t, g in enumerate(gains):
                dq = 2.0 * g / float(G.two_m) ** 2
                if t < len(gains) - 1:
                    assert dq > tau
                elif st["iterations"][p] < 20:
                    assert dq <= tau
            tau /= 10
        assert st["moves"] == sum(sum(x) for x in st["iter_moves"])


def test_sbm_planted_partition_recovered(orc):
    e = W.config1_sbm()
    G = _graph(orc, e)
    planted = np.arange(e.n) // 200
    qp = G.modularity(planted)
    assert 0.75 < qp < 0.80
    for mode in ("sync", "async"):
        C, K, S, st = G.louvain("static", mode=mode)
        assert G.modularity(C) >= qp - 1e-3


# --------------------------------------------------------------------------
# Batch update, Alg. 7, invariants
# --------------------------------------------------------------------------

def test_apply_batch_matches_edge_list_update(orc):
    e = W.config1_sbm()
    b = W.random_batch(e, 100, 11)
    G = _graph(orc, e)
    assert G.apply_batch(b) == orc.OK
    e2 = W.apply_batch_np(e, b)
    G2 = _graph(orc, e2)
    o1, c1, w1 = G.csr()
    o2, c2, w2 = G2.csr()
    assert np.array_equal(o1, o2) and np.array_equal(c1, c2) and np.array_equal(w1, w2)
    assert G.two_m == 2 * int(e2.w.sum())


def test_apply_batch_rejects_without_change(orc):
    e = W.random_small_graph(20, 40, 5)
    G = _graph(orc, e)
    before = G.csr()
    bad_del = W.Batch(np.array([0], np.int32), np.array([0], np.int32), np.array([1], np.int32),
                      *[np.zeros(0, np.int32)] * 3)
    assert G.apply_batch(bad_del) == orc.E_INVAL            # self loop
    missing = W.random_batch(e, 5, 1)
    key = set(zip(e.u.tolist(), e.v.tolist()))
    a, b = next((a, b) for a in range(20) for b in range(a + 1, 20) if (a, b) not in key)
    nodel = W.Batch(np.array([a], np.int32), np.array([b], np.int32), np.array([1], np.int32),
                    missing.ins_u, missing.ins_v, missing.ins_w)
    assert G.apply_batch(nodel) == orc.E_NOEDGE
    heavy = W.Batch(e.u[:1], e.v[:1], e.w[:1] + 1, *[np.zeros(0, np.int32)] * 3)
    assert G.apply_batch(heavy) == orc.E_NOEDGE
    dup = W.Batch(*[np.zeros(0, np.int32)] * 3, np.array([a, b], np.int32), np.array([b, a], np.int32),
                  np.array([1, 1], np.int32))
    assert G.apply_batch(dup) == orc.E_INVAL
    after = G.csr()
    assert all(np.array_equal(x, y) for x, y in zip(before, after))


@pytest.mark.parametrize("seed", range(3))
def test_update_weights_equals_recompute(orc, seed):
    e = W.rmat(10, 8, 0.57, 0.19, 0.19, seed)
    rng = np.random.default_rng(seed)
    G = _graph(orc, e)
    C = rng.integers(0, 50, e.n).astype(np.int32)
    K = G.degrees()
    S = np.bincount(C, weights=K, minlength=e.n).astype(np.int64)
    b = W.random_batch(e, 300, seed)
    K2, S2 = orc.update_weights(e.n, b, C, K, S)
    assert G.apply_batch(b) == orc.OK
    Kr = G.degrees()
    assert np.array_equal(K2, Kr)
    assert np.array_equal(S2, np.bincount(C, weights=Kr, minlength=e.n).astype(np.int64))
    assert int(Kr.sum()) == G.two_m


def _run_dynamic(orc, approach, e, b, mode="sync"):
    G = _graph(orc, e)
    C, K, S, _ = G.louvain("static", mode=mode)
    assert G.apply_batch(b) == orc.OK
    C2, K2, S2, st = G.louvain(approach, batch=b, state=(C, K, S), mode=mode)
    return G, (C, K, S), (C2, K2, S2), st


@pytest.mark.parametrize("approach", ["nd", "ds", "df"])
@pytest.mark.parametrize("mode", ["sync", "async"])
def test_dynamic_outputs_consistent(orc, approach, mode):
    e = W.config1_sbm()
    b = W.random_batch(e, 100, 3)
    G, _, (C, K, S), st = _run_dynamic(orc, approach, e, b, mode)
    assert np.array_equal(K, G.degrees())
    assert np.array_equal(S, np.bincount(C, weights=K, minlength=e.n).astype(np.int64))
    assert C.min() >= 0 and C.max() < e.n


def test_dynamic_modularity_close_to_static(orc):
    e = W.config1_sbm()
    b = W.random_batch(e, 100, 3)
    G = _graph(orc, e)
    C, K, S, _ = G.louvain("static", mode="async")
    assert G.apply_batch(b) == orc.OK
    Cs, _, _, _ = G.louvain("static", mode="async")
    qs = G.modularity(Cs)
    for ap in ("nd", "ds", "df"):
        Cd, _, _, _ = G.louvain(ap, batch=b, state=(C, K, S), mode="async")
        assert G.modularity(Cd) >= qs - 1e-3


# --------------------------------------------------------------------------
# Marking (Alg. 1, Alg. 2, Alg. 3)
# --------------------------------------------------------------------------

def _edges(n, pairs):
    a = np.array(pairs, dtype=np.int32).reshape(-1, 2)
    return W.Edges(n, a[:, 0].copy(), a[:, 1].copy(), np.ones(a.shape[0], np.int32))


def _batch(dels=(), ins=()):
    d = np.array(dels, dtype=np.int32).reshape(-1, 2)
    i = np.array(ins, dtype=np.int32).reshape(-1, 2)
    return W.Batch(d[:, 0].copy(), d[:, 1].copy(), np.ones(d.shape[0], np.int32),
                   i[:, 0].copy(), i[:, 1].copy(), np.ones(i.shape[0], np.int32))


def test_df_marking_rule_table(orc):
    # communities {0,1,2} {3,4,5}; edges inside and one across (2,3)
    e = _edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)])
    G = _graph(orc, e)
    C = np.array([0, 0, 0, 3, 3, 3], np.int32)
    K = G.degrees()
    S = np.bincount(C, weights=K, minlength=6).astype(np.int64)
    cases = [
        (_batch(dels=[(0, 1)]), {0, 1}),      # deletion inside a community: marked
        (_batch(dels=[(2, 3)]), set()),       # deletion across: ignored
        (_batch(ins=[(1, 4)]), {1, 4}),       # insertion across: marked
        (_batch(ins=[(3, 5)]), set()),        # insertion inside (merge): ignored
    ]
    for b, want in cases:
        f, r = G.mark("df", b, C, K, S)
        assert set(np.nonzero(f)[0].tolist()) == want
        assert r.all()
    f, r = G.mark("nd", cases[0][0], C, K, S)
    assert f.all() and r.all()


def test_ds_marking_hand_case(orc):
    # communities A={0,1,2}, B={3,4,5}, D={6,7}; 8 isolated in its own
    e = _edges(9, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (6, 7), (2, 3)])
    G = _graph(orc, e)
    C = np.array([0, 0, 0, 3, 3, 3, 6, 6, 8], np.int32)
    K = G.degrees()
    S = np.bincount(C, weights=K, minlength=9).astype(np.int64)
    # deletion inside A: 0 and 1 and their neighbours, plus every member of A
    f, r = G.mark("ds", _batch(dels=[(0, 1)]), C, K, S)
    assert set(np.nonzero(f)[0].tolist()) == {0, 1, 2}
    assert np.array_equal(f, r)
    # insertion 6-0 (across): source 6 links to A, source 0 links to D.
    # Each source marks itself, its neighbours and its best linked community.
    f, r = G.mark("ds", _batch(ins=[(6, 0)]), C, K, S)
    assert set(np.nonzero(f)[0].tolist()) == {0, 1, 2, 6, 7}
    # insertion inside a community: ignored
    f, r = G.mark("ds", _batch(ins=[(3, 5)]), C, K, S)
    assert not f.any()


def test_ds_best_community_uses_eq2_score(orc):
    # A={0,9}, B={1,2,3,4,7}, D={5,6,8}.  Insertions (0,2) and (0,5) give
    # source 0 weight 1 towards B and towards D.  Σ_D < Σ_B, so D scores
    # higher (2m H[c] - K_0 Σ_c) and only D's members are marked as a
    # community: 8 (D, not adjacent to a source) is marked, 7 (B, not
    # adjacent to a source) is not.
    e = _edges(10, [(1, 2), (2, 3), (1, 3), (3, 4), (1, 4), (2, 4), (1, 7), (5, 6), (6, 8), (0, 9)])
    G = _graph(orc, e)
    C = np.array([0, 1, 1, 1, 1, 5, 5, 1, 5, 0], np.int32)
    K = G.degrees()
    S = np.bincount(C, weights=K, minlength=10).astype(np.int64)
    f, r = G.mark("ds", _batch(ins=[(0, 2), (0, 5)]), C, K, S)
    assert set(np.nonzero(f)[0].tolist()) == {0, 1, 2, 3, 4, 5, 6, 8, 9}
    assert np.array_equal(f, r)


def test_empty_and_ignorable_batches_change_nothing(orc):
    e = W.config1_sbm()
    G = _graph(orc, e)
    C, K, S, _ = G.louvain("static")
    # cross-community deletion and intra-community insertion only
    cross = np.nonzero(C[e.u] != C[e.v])[0][:3]
    intra_pairs = []
    present = set(zip(e.u.tolist(), e.v.tolist()))
    comm0 = np.nonzero(C == C[0])[0]
    for a in comm0:
        for bb in comm0:
            if a < bb and (a, bb) not in present:
                intra_pairs.append((a, bb))
            if len(intra_pairs) == 3:
                break
        if len(intra_pairs) == 3:
            break
    b = W.Batch(e.u[cross], e.v[cross], e.w[cross],
                np.array([p[0] for p in intra_pairs], np.int32),
                np.array([p[1] for p in intra_pairs], np.int32), np.ones(3, np.int32))
    assert G.apply_batch(b) == orc.OK
    for mode in ("sync", "async"):
        C2, K2, S2, st = G.louvain("df", batch=b, state=(C, K, S), mode=mode)
        assert st["passes"] == 1 and st["iterations"] == [1] and st["moves"] == 0
        assert st["vertices_affected"] == 0
        assert np.array_equal(C2, C)
        assert np.array_equal(K2, G.degrees())
    empty = _batch()
    C3, _, _, st = G.louvain("df", batch=empty, state=(C, K2, S2))
    assert np.array_equal(C3, C) and st["iterations"] == [1]


# --------------------------------------------------------------------------
# Aggregation (Alg. 6)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_aggregation_preserves_modularity_and_weight(orc, seed):
    e = W.rmat(9, 8, 0.57, 0.19, 0.19, 10 + seed)
    rng = np.random.default_rng(seed)
    G = _graph(orc, e)
    nc = 40
    C = rng.integers(0, nc, e.n).astype(np.int32)
    # make ids dense
    uniq, C = np.unique(C, return_inverse=True)
    C = C.astype(np.int32)
    nc = uniq.shape[0]
    A = G.aggregate(C, nc)
    assert A.two_m == G.two_m
    KA = A.degrees()
    K = G.degrees()
    assert np.array_equal(KA, np.bincount(C, weights=K, minlength=nc).astype(np.int64))
    assert A.modularity(np.arange(nc)) == pytest.approx(G.modularity(C), abs=1e-13)
    # and for a coarser partition of the super-vertices
    D = rng.integers(0, 7, nc).astype(np.int32)
    assert A.modularity(D) == pytest.approx(G.modularity(D[C]), abs=1e-13)
    # the self-loop of c is its intra weight σ_c
    off, col, w = A.csr()
    for c in range(0, nc, 7):
        row = slice(off[c], off[c + 1])
        self_w = w[row][col[row] == c]
        sig_in = int(e.w[(C[e.u] == c) & (C[e.v] == c)].sum()) * 2
        assert (self_w.sum() if self_w.size else 0) == sig_in


# --------------------------------------------------------------------------
# Alg. 4: the aggregation stop and the renumbering of communities
# --------------------------------------------------------------------------


def test_aggregation_tolerance_boundary(orc):
    """Alg. 4 stops when the pass leaves more than τ_agg of the vertices as
    communities (|communities| / |vertices| > τ_agg); at equality it
    aggregates.  A ring of 4 cliques of 5 ends pass 0 as its 4 cliques:
    the ratio is 4/20 = 0.2 exactly."""
    e = W.ring_of_cliques(4, 5)
    G = _graph(orc, e)
    _, _, _, st = G.louvain("static", mode="async", aggregation_tolerance=0.2)
    assert st["communities"][0] == 4
    assert st["passes"] == 2  # equal ratio: aggregated, then level 1 runs
    _, _, _, st = G.louvain("static", mode="async", aggregation_tolerance=float(np.nextafter(0.2, 0.0)))
    assert st["communities"][0] == 4
    assert st["passes"] == 1  # ratio above: stopped before aggregating


def test_renumbering_is_ascending_old_id(orc):
    """Communities are renumbered in ascending order of their old ids (the
    reading the implementations share), worked by hand on 10 vertices:
    a 5-clique {1..5} (weights 1), an edge 6-7 (weight 1), and a triangle
    0-8 (1), 0-9 (1), 8-9 (3); 2m = 32.  ASYNC visits ascending ids; the
    integer gain is 2m (K_i->c - K_i->d) - K_i (Σ_c - Σ_d + K_i).

    Iteration 1: vertex 0 prefers 8 (gain 24, tied with 9, lower id) but
    the swap guard keeps a singleton from joining a larger singleton; 1
    likewise stays, 2..5 join 1; 6 stays, 7 joins 6; 8 prefers 9 (gain 80)
    and is blocked; 9 joins 8 (gain 80).  Iteration 2 (neighbours of
    movers): 0 joins community 8, now of size 2 (gain 64 - 16 = 48).  So
    the old labels are 1 for {1..5}, 6 for {6, 7} and 8 for {0, 8, 9}, and
    ascending old id gives 0, 1 and 2.  Level 1 has three isolated
    super-vertices: no moves, so the labels are final.  Numbering by first
    member would instead give {0, 8, 9} the label 0."""
    pairs = [(a, b, 1) for a in range(1, 6) for b in range(a + 1, 6)] + [(6, 7, 1), (0, 8, 1), (0, 9, 1),
                                                                        (8, 9, 3)]
    u, v, w = (np.array(x, dtype=np.int32) for x in zip(*pairs))
    G = _graph(orc, W.Edges(10, u, v, w))
    C, _, _, st = G.louvain("static", mode="async")
    assert C.tolist() == [2, 0, 0, 0, 0, 0, 1, 1, 2, 2]
    assert st["passes"] == 2 and st["communities"][0] == 3
