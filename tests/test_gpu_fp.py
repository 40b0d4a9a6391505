"""GPU parity of the paper-precision path (float32 edge weights, FP64 sums
and Eq. 2 in FP64; Section 5.1.2) against the paper-precision oracle.

Exact where the arithmetic fixes the result: the built and edited graphs
(arc for arc, float32 weights bit-equal: every arc weight is the same
float32 sum in both), and the error codes of invalid batches.  FP64 sums
whose order differs (K, 2m, Sigma, modularity) agree to a relative 1e-12.
The ASYNC results depend on the order of floating-point sums and moves, so
the memberships are checked for consistency (Sigma and K recomputed from
them) and for quality: modularity within 1e-3 of the oracle's ASYNC run on
the same input, and the planted partitions of clique graphs recovered.
"""
import numpy as np
import pytest
import torch

from paper_2404_19634_amd import workloads as W

pytestmark = pytest.mark.gpu

Q_TOL = 1e-3


@pytest.fixture(scope="module")
def lib():
    from paper_2404_19634_amd import lib as L
    L.load()
    L.set_tuning()
    return L


def _weighted(e, seed):
    return W.real_weights(e, seed)


def _cases():
    return {
        "sbm": lambda: _weighted(W.config1_sbm(), 11),
        "rmat12": lambda: _weighted(W.rmat(12, 16, 0.57, 0.19, 0.19, 5), 12),
        "star_plus": lambda: _weighted(_star_plus(), 13),
    }


def _star_plus(seed=3):
    # a 3000-arc hub, a 600-arc vertex, a ring and random chords: rows in
    # the wavefront, workgroup and pooled-table bins
    rng = np.random.default_rng(seed)
    n = 3301
    pairs = set((0, v) for v in range(1, 3001))
    pairs.update((1, v) for v in range(3001, 3301))
    pairs.update((v, v + 1) for v in range(1, 3000))
    while len(pairs) < 9000:
        a, b = rng.integers(1, n, 2)
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    a = np.array(sorted(pairs), dtype=np.int32)
    return W.Edges(n, a[:, 0].copy(), a[:, 1].copy(), np.ones(a.shape[0], np.int32))


def _graph(lib, e, **kw):
    return lib.GraphF.build(e.n, e.u, e.v, np.asarray(e.w, np.float32), **kw)


def _same_csr(g, G):
    off, col, w = g.csr_host()
    o2, c2, w2 = G.csr()
    assert np.array_equal(off, o2)
    assert np.array_equal(col, c2)
    assert np.array_equal(w.view(np.uint32), w2.view(np.uint32))


def _close(a, b, rel=1e-12):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = max(1.0, float(np.max(np.abs(b))) if b.size else 1.0)
    assert np.max(np.abs(a - b), initial=0.0) <= rel * scale


def _consistent(G, C, K, S, two_m):
    """K equals the oracle's row sums; Sigma equals the totals of C."""
    n = G.n
    assert C.min() >= 0 and C.max() < n
    _close(K, G.degrees())
    tot = np.zeros(n, np.float64)
    np.add.at(tot, C, K)
    _close(S, tot, rel=1e-9)


@pytest.mark.parametrize("name", list(_cases()))
def test_build_matches_oracle(lib, orc, name):
    e = _cases()[name]()
    g = _graph(lib, e)
    G = orc.GraphF.from_edges(e)
    _same_csr(g, G)
    assert abs(g.two_m - G.two_m) <= 1e-12 * G.two_m


@pytest.mark.parametrize("name", list(_cases()))
def test_modularity_matches_oracle(lib, orc, name):
    e = _cases()[name]()
    g = _graph(lib, e)
    G = orc.GraphF.from_edges(e)
    rng = np.random.default_rng(5)
    for parts in (1, 7, 64, e.n):
        C = rng.integers(0, parts, e.n).astype(np.int32)
        q = lib.modularity_f(g, torch.from_numpy(C).cuda())
        assert abs(q - G.modularity(C)) <= 1e-12


@pytest.mark.parametrize("name", list(_cases()))
def test_static_quality(lib, orc, name):
    e = _cases()[name]()
    g = _graph(lib, e)
    G = orc.GraphF.from_edges(e)
    st, stats = lib.louvain_static_f(g)
    C, K, S = st.host()
    _consistent(G, C, K, S, g.two_m)
    size = st.size.cpu().numpy()
    assert np.array_equal(size, np.bincount(C, minlength=e.n))
    q = lib.modularity_f(g, st.C)
    assert abs(q - G.modularity(C)) <= 1e-12
    Co, _, _, so = G.louvain("static", mode="async")
    qo = G.modularity(Co)
    assert q >= qo - Q_TOL, (q, qo)
    assert stats["passes"] >= 1 and stats["moves"] > 0


def test_static_sync_rejected(lib):
    e = _weighted(W.two_cliques_bridge(5), 1)
    g = _graph(lib, e)
    with pytest.raises(lib.LouvainError) as ex:
        lib.louvain_static_f(g, mode="sync")
    assert ex.value.code == lib.LV_EINVAL


@pytest.mark.parametrize("scale", [1.0, 0.37])
def test_planted_cliques(lib, orc, scale):
    # a ring of 24 cliques of 6, uniform weight: the optimum is the cliques
    e = W.ring_of_cliques(24, 6)
    e = W.Edges(e.n, e.u, e.v, np.full(e.m, scale, np.float32))
    g = _graph(lib, e)
    st, _ = lib.louvain_static_f(g)
    C = st.C.cpu().numpy()
    truth = np.arange(e.n) // 6
    # the same partition up to labels
    pairs = set(zip(C.tolist(), truth.tolist()))
    assert len(pairs) == len(set(C.tolist())) == 24
    G = orc.GraphF.from_edges(e)
    assert abs(lib.modularity_f(g, st.C) - G.modularity(truth.astype(np.int32))) <= 1e-12


def _edit_batch(e, seed):
    """Whole and half deletions, insertions of absent pairs and of present
    ones (merges), including a pair deleted whole and re-inserted."""
    rng = np.random.default_rng(seed)
    m = e.m
    pick = rng.choice(m, size=min(m, 120), replace=False)
    whole, half = pick[:60], pick[60:100]
    merge = pick[100:]
    du = np.concatenate([e.u[whole], e.u[half]])
    dv = np.concatenate([e.v[whole], e.v[half]])
    dw = np.concatenate([e.w[whole], (e.w[half] * np.float32(0.5)).astype(np.float32)]).astype(np.float32)
    b = W.random_batch(W.Edges(e.n, e.u, e.v, np.ones(m, np.int32)), 100, seed + 1, ins_frac=1.0)
    iu = np.concatenate([b.ins_u, e.u[merge], e.u[whole[:5]]])
    iv = np.concatenate([b.ins_v, e.v[merge], e.v[whole[:5]]])
    iw = rng.uniform(0.25, 4.0, iu.shape[0]).astype(np.float32)
    return W.Batch(du.astype(np.int32), dv.astype(np.int32), dw, iu.astype(np.int32), iv.astype(np.int32), iw)


@pytest.mark.parametrize("name", ["sbm", "star_plus"])
def test_apply_batch_matches_oracle(lib, orc, name):
    e = _cases()[name]()
    g = _graph(lib, e, slack_frac=0.5, slack_min=8)
    G = orc.GraphF.from_edges(e)
    for s in range(3):
        b = _edit_batch(W.Edges(e.n, *G_edges(G)), 100 + s)
        assert G.apply_batch(b) == 0
        lib.apply_batch_f(g, lib.BatchF.from_host(b))
        _same_csr(g, G)
        assert abs(g.two_m - G.two_m) <= 1e-9 * G.two_m


def G_edges(G):
    off, col, w = G.csr()
    rows = np.repeat(np.arange(G.n), np.diff(off))
    keep = rows < col
    return rows[keep].astype(np.int32), col[keep].astype(np.int32), w[keep]


def test_apply_batch_errors_leave_graph(lib, orc):
    e = _cases()["sbm"]()
    g = _graph(lib, e, slack_frac=0.0, slack_min=0)
    before = g.csr_host()
    two_m = g.two_m
    u0, v0, w0 = int(e.u[0]), int(e.v[0]), float(e.w[0])
    nbrs = set(e.v[e.u == u0].tolist()) | set(e.u[e.v == u0].tolist())
    far = [v for v in range(e.n - 1, 0, -1) if v != u0 and v not in nbrs][0]
    z = np.zeros(0, np.int32)
    zf = np.zeros(0, np.float32)

    def one(u, v, x, ins):
        a = (np.array([u], np.int32), np.array([v], np.int32), np.array([x], np.float32))
        return W.Batch(*a, z, z, zf) if not ins else W.Batch(z, z, zf, *a)

    bad = {
        "missing": (one(u0, far, 1.0, False), lib.LV_ENOEDGE),
        "too_much": (one(u0, v0, 2 * w0, False), lib.LV_ENOEDGE),
        "dup": (W.Batch(z, z, zf, np.array([1, 2], np.int32), np.array([2, 1], np.int32),
                        np.array([1.0, 1.0], np.float32)), lib.LV_EINVAL),
        "dup_del": (W.Batch(np.array([u0, v0], np.int32), np.array([v0, u0], np.int32),
                            np.array([0.1, 0.1], np.float32), z, z, zf), lib.LV_EINVAL),
        "loop": (one(3, 3, 1.0, True), lib.LV_EINVAL),
        "nan": (one(3, 4, np.nan, True), lib.LV_EINVAL),
        "neg": (one(3, 4, -1.0, True), lib.LV_EINVAL),
        "range": (one(3, e.n, 1.0, True), lib.LV_EINVAL),
        # no slack: an append to a row overflows it
        "slack": (one(u0, far, 1.0, True), lib.LV_ENOSLACK),
    }
    for name, (b, code) in bad.items():
        with pytest.raises(lib.LouvainError) as ex:
            lib.apply_batch_f(g, lib.BatchF.from_host(b))
        assert ex.value.code == code, name
        after = g.csr_host()
        for x, y in zip(before, after):
            assert np.array_equal(x, y), name
        assert g.two_m == two_m


@pytest.mark.parametrize("name", list(_cases()))
def test_df_chain_quality(lib, orc, name):
    """Static, then batches of growing size with DF: the library's chain
    stays within Q_TOL of the oracle's own chains; K, Sigma and sizes stay
    exact.  ASYNC fixes no visiting order (the paper's loop runs under a
    dynamic schedule), and on graphs without planted structure equally
    valid orders differ by more than Q_TOL (the oracle's static Q on the
    4096-vertex R-MAT graph spans 1.8e-3 over vertex relabelings), so the
    reference at each step is the lowest of the oracle's chains under the
    identity and two seeded relabelings of the vertices."""
    e = _cases()[name]()
    g = _graph(lib, e, slack_frac=0.5, slack_min=8)
    G = orc.GraphF.from_edges(e)
    st, _ = lib.louvain_static_f(g)
    perms = [np.arange(e.n, dtype=np.int32)] + [np.random.default_rng(900 + s).permutation(e.n).astype(np.int32)
                                                for s in range(2)]
    refs = []
    for p in perms:
        Gp = orc.GraphF(e.n, p[e.u], p[e.v], e.w)
        refs.append([Gp, Gp.louvain("static", mode="async")[:3]])
    for k, frac in enumerate((1e-3, 1e-2, 5e-2)):
        size = max(4, int(frac * e.m))
        cur = W.Edges(e.n, *G_edges(G))
        b = W.real_batch(W.random_batch(W.Edges(e.n, cur.u, cur.v, np.ones(cur.m, np.int32)), size, 40 + k),
                         cur, 50 + k)
        assert G.apply_batch(b) == 0
        bf = lib.BatchF.from_host(b)
        lib.apply_batch_f(g, bf)
        st, stats = lib.louvain_df_f(g, bf, st)
        qos = []
        for p, ref in zip(perms, refs):
            Gp, state = ref
            bp = W.Batch(p[b.del_u], p[b.del_v], b.del_w, p[b.ins_u], p[b.ins_v], b.ins_w)
            assert Gp.apply_batch(bp) == 0
            ref[1] = Gp.louvain("df", batch=bp, state=state, mode="async")[:3]
            qos.append(Gp.modularity(ref[1][0]))
        C, K, S = st.host()
        _consistent(G, C, K, S, g.two_m)
        assert np.array_equal(st.size.cpu().numpy(), np.bincount(C, minlength=e.n))
        q = lib.modularity_f(g, st.C)
        assert abs(q - G.modularity(C)) <= 1e-12
        assert q >= min(qos) - Q_TOL, (k, q, qos)
        assert stats["vertices_affected"] > 0


def test_df_without_sizes_and_bad_state(lib, orc):
    e = _cases()["sbm"]()
    g = _graph(lib, e, slack_frac=0.5, slack_min=8)
    st, _ = lib.louvain_static_f(g)
    noz = lib.StateF(st.C.clone(), st.K.clone(), st.Sigma.clone(), None)
    b = lib.BatchF.from_host(W.Batch(*(np.zeros(0, t) for t in (np.int32, np.int32, np.float32,
                                                               np.int32, np.int32, np.float32))))
    out, stats = lib.louvain_df_f(g, b, noz)
    assert stats["moves"] == 0  # an empty batch marks nothing
    bad = noz.clone()
    bad.C[7] = e.n
    with pytest.raises(lib.LouvainError) as ex:
        lib.louvain_df_f(g, b, bad)
    assert ex.value.code == lib.LV_EINVAL
