"""GPU parity: the HIP library against the sequential oracle.

SYNC mode is bit-exact: memberships, weighted degrees, community totals and
every per-iteration statistic (moves, summed integer gains), on graphs that
span all degree bins (sub-wave groups, wavefront, workgroup) and ragged
sizes.  ASYNC mode is checked for consistency and modularity quality.
"""
import numpy as np
import pytest
import torch

from paper_2404_19634_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2404_19634_amd import lib as L
    L.load()
    L.set_tuning()
    return L


def _star_plus(seed=3):
    # one hub adjacent to 3000 leaves, a 600-degree vertex, a ring over the
    # leaves and a few random chords: rows in every bin
    rng = np.random.default_rng(seed)
    n = 3301
    pairs = set()
    for v in range(1, 3001):
        pairs.add((0, v))
    for v in range(3001, 3301):
        pairs.add((1, v) if v != 1 else (1, 2))
    for v in range(1, 3000):
        pairs.add((v, v + 1))
    while len(pairs) < 9000:
        a, b = rng.integers(1, n, 2)
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    for v in range(3001, 3301, 2):
        pairs.add((1, v))
    a = np.array(sorted(pairs), dtype=np.int32)
    return W.Edges(n, a[:, 0].copy(), a[:, 1].copy(), np.ones(a.shape[0], np.int32))


def _cases():
    return {
        "sbm": lambda: W.config1_sbm(),
        "rmat12": lambda: W.rmat(12, 16, 0.57, 0.19, 0.19, 5),
        "rmat14": lambda: W.rmat(14, 8, 0.57, 0.19, 0.19, 6),
        "weighted_ragged": lambda: W.random_small_graph(1037, 4000, 9, max_w=7),
        "ring_cliques": lambda: W.ring_of_cliques(30, 6),
        "star_plus": _star_plus,
    }


CASES = _cases()


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    return request.param, CASES[request.param]()


def _orc(e):
    import oracle
    return oracle.Graph.from_edges(e)


def _same_stats(gs, os_, keys=("passes", "iterations", "communities", "moves", "arcs_scanned",
                                "vertices_affected", "iter_moves", "iter_gain")):
    for k in keys:
        assert gs[k] == os_[k], (k, gs[k], os_[k])


def test_csr_build(lib, case):
    name, e = case
    g = lib.Graph.from_edges(e)
    off, col, w = g.csr_host()
    o_off, o_col, o_w = _orc(e).csr()
    assert np.array_equal(off, o_off) and np.array_equal(col, o_col) and np.array_equal(w, o_w)
    assert g.two_m == 2 * int(e.w.sum())


def test_modularity(lib, case):
    name, e = case
    g = lib.Graph.from_edges(e)
    G = _orc(e)
    rng = np.random.default_rng(1)
    for C in (np.arange(e.n), rng.integers(0, 17, e.n), np.zeros(e.n)):
        C = C.astype(np.int32)
        q = lib.modularity(g, torch.from_numpy(C).cuda())
        assert abs(q - G.modularity(C)) < 1e-12


@pytest.mark.parametrize("guard", [1, 0])
def test_static_sync_bit_exact(lib, case, guard):
    name, e = case
    g = lib.Graph.from_edges(e)
    st, gs = lib.louvain_static(g, mode="sync", swap_guard=guard)
    C, K, S = st.host()
    Co, Ko, So, os_ = _orc(e).louvain("static", mode="sync", swap_guard=guard)
    assert np.array_equal(K, Ko)
    assert np.array_equal(C, Co)
    assert np.array_equal(S, So)
    _same_stats(gs, os_)


@pytest.mark.parametrize("tuning", [dict(wave_max_degree=32), dict(wave_max_degree=512),
                                    dict(blocks_small=1, blocks_wave=1, blocks_hub=1)])
def test_static_sync_independent_of_mapping(lib, tuning):
    e = W.rmat(12, 16, 0.57, 0.19, 0.19, 5)
    Co, Ko, So, os_ = _orc(e).louvain("static", mode="sync")
    lib.set_tuning(**tuning)
    try:
        g = lib.Graph.from_edges(e)
        st, gs = lib.louvain_static(g, mode="sync")
    finally:
        lib.set_tuning()
    C, K, S = st.host()
    assert np.array_equal(C, Co) and np.array_equal(S, So)
    _same_stats(gs, os_)


def test_static_single_iteration(lib, case):
    name, e = case
    g = lib.Graph.from_edges(e)
    st, gs = lib.louvain_static(g, mode="sync", max_iterations=1, max_passes=1)
    Co, Ko, So, os_ = _orc(e).louvain("static", mode="sync", max_iterations=1, max_passes=1)
    C, K, S = st.host()
    assert np.array_equal(C, Co) and np.array_equal(S, So)
    _same_stats(gs, os_)


def _sizes(C, n):
    return np.bincount(np.asarray(C, np.int64), minlength=n).astype(np.int32)


@pytest.mark.parametrize("carry_size", [False, True])
@pytest.mark.parametrize("approach", ["nd", "ds", "df"])
def test_dynamic_sync_bit_exact(lib, case, approach, carry_size):
    name, e = case
    b = W.random_batch(e, max(10, e.m // 200), 77)
    G = _orc(e)
    state0 = G.louvain("static", mode="async")[:3]
    assert G.apply_batch(b) == 0
    Cd, Kd, Sd, os_ = G.louvain(approach, batch=b, state=state0, mode="sync")
    g = lib.Graph.from_edges(e)
    bb = lib.Batch.from_host(b)
    lib.apply_batch(g, bb)
    off, col, w = g.csr_host()
    o_off, o_col, o_w = G.csr()
    assert np.array_equal(off, o_off) and np.array_equal(col, o_col) and np.array_equal(w, o_w)
    assert g.two_m == G.two_m
    st = lib.State.from_host(*state0)
    if carry_size:  # member counts carried in from the previous state
        st.size = torch.from_numpy(_sizes(state0[0], e.n)).cuda()
    st, gs = getattr(lib, "louvain_" + approach)(g, bb, st, mode="sync")
    C, K, S = st.host()
    assert np.array_equal(K, Kd)
    assert np.array_equal(C, Cd)
    assert np.array_equal(S, Sd)
    _same_stats(gs, os_)
    if carry_size:
        assert np.array_equal(st.size.cpu().numpy(), _sizes(C, e.n))


@pytest.mark.parametrize("recompute", [0, 1])
def test_df_apply_one_call_sync_bit_exact(lib, case, recompute):
    """louvain_df_apply (the batch edit and DF in one call) gives the
    oracle's graph, state and statistics, as the two calls do."""
    name, e = case
    b = W.random_batch(e, max(10, e.m // 200), 79)
    G = _orc(e)
    state0 = G.louvain("static", mode="async")[:3]
    assert G.apply_batch(b) == 0
    Cd, Kd, Sd, os_ = G.louvain("df", batch=b, state=state0, mode="sync")
    g = lib.Graph.from_edges(e)
    st = lib.State.from_host(*state0)
    st.size = torch.from_numpy(_sizes(state0[0], e.n)).cuda()
    st, gs = lib.louvain_df_apply(g, lib.Batch.from_host(b), st, mode="sync", recompute_weights=recompute)
    assert all(np.array_equal(x, y) for x, y in zip(g.csr_host(), G.csr()))
    assert g.two_m == G.two_m
    C, K, S = st.host()
    assert np.array_equal(K, Kd) and np.array_equal(C, Cd) and np.array_equal(S, Sd)
    assert np.array_equal(st.size.cpu().numpy(), _sizes(C, e.n))
    _same_stats(gs, os_)


def test_df_apply_refused_batch_changes_nothing(lib):
    """An edit the batch cannot make (no slack, a missing edge, a repeated
    pair) is refused by louvain_df_apply with graph and state untouched;
    after a relayout the same call succeeds and matches the oracle."""
    e = W.random_small_graph(400, 1500, 12)
    G = _orc(e)
    state0 = G.louvain("static", mode="async")[:3]
    g = lib.Graph.from_edges(e, slack_frac=0.0, slack_min=0)
    present = set(zip(e.u.tolist(), e.v.tolist()))
    absent = [(a, c) for a in range(400) for c in range(a + 1, 400) if (a, c) not in present][:3]
    z = np.zeros(0, np.int32)
    iu, iv = (np.array(x, np.int32) for x in zip(*absent))
    cases = [
        (lib.LV_ENOSLACK, W.Batch(z, z, z, iu, iv, np.ones(3, np.int32))),
        (lib.LV_ENOEDGE, W.Batch(iu[:1], iv[:1], np.ones(1, np.int32), z, z, z)),
        (lib.LV_EINVAL, W.Batch(z, z, z, np.array([iu[0], iv[0]], np.int32), np.array([iv[0], iu[0]], np.int32),
                                np.ones(2, np.int32))),
    ]
    before = g.csr_host()
    st = lib.State.from_host(*state0)
    for code, b in cases:
        with pytest.raises(lib.LouvainError) as ex:
            lib.louvain_df_apply(g, lib.Batch.from_host(b), st, mode="sync")
        assert ex.value.code == code
        assert all(np.array_equal(x, y) for x, y in zip(before, g.csr_host()))
        assert g.two_m == 2 * int(e.w.sum())
        for x, y in zip(st.host(), state0):
            assert np.array_equal(x, y)
    b = cases[0][1]
    g = g.relayout(slack_frac=0.5, slack_min=8)
    st, gs = lib.louvain_df_apply(g, lib.Batch.from_host(b), st, mode="sync")
    assert G.apply_batch(b) == 0
    Cd, Kd, Sd, os_ = G.louvain("df", batch=b, state=state0, mode="sync")
    C, K, S = st.host()
    assert np.array_equal(C, Cd) and np.array_equal(K, Kd) and np.array_equal(S, Sd)
    _same_stats(gs, os_)


@pytest.mark.parametrize("approach", ["nd", "ds", "df"])
def test_without_auxiliary_information_sync_bit_exact(lib, case, approach):
    """recompute_weights=1 (Section 4.2's variant without auxiliary
    information): K^t and Sigma^t are recomputed from G^t and C^{t-1}, so
    every result equals the incremental run's, i.e. the oracle's.  ND and
    DF never read the carried K and Sigma then, so they get garbage ones
    (DS scores its marking with them, so it gets the true ones)."""
    name, e = case
    b = W.random_batch(e, max(10, e.m // 200), 78)
    G = _orc(e)
    state0 = G.louvain("static", mode="async")[:3]
    assert G.apply_batch(b) == 0
    Cd, Kd, Sd, os_ = G.louvain(approach, batch=b, state=state0, mode="sync")
    g = lib.Graph.from_edges(e)
    bb = lib.Batch.from_host(b)
    lib.apply_batch(g, bb)
    C0, K0, S0 = state0
    if approach != "ds":
        rng = np.random.default_rng(3)
        K0 = rng.integers(-1000, 1000, e.n).astype(np.int64)
        S0 = rng.integers(-1000, 1000, e.n).astype(np.int64)
    st, gs = getattr(lib, "louvain_" + approach)(g, bb, lib.State.from_host(C0, K0, S0), mode="sync",
                                                  recompute_weights=1)
    C, K, S = st.host()
    assert np.array_equal(K, Kd)
    assert np.array_equal(C, Cd)
    assert np.array_equal(S, Sd)
    _same_stats(gs, os_)


@pytest.mark.parametrize("approach", ["static", "nd", "ds", "df"])
def test_async_consistent_and_close_to_static(lib, approach):
    e = W.config1_sbm()
    b = W.random_batch(e, 100, 5)
    G = _orc(e)
    state0 = G.louvain("static", mode="async")[:3]
    assert G.apply_batch(b) == 0
    Cs = G.louvain("static", mode="async")[0]
    q_static = G.modularity(Cs)
    g = lib.Graph.from_edges(e)
    bb = lib.Batch.from_host(b)
    lib.apply_batch(g, bb)
    if approach == "static":
        st, gs = lib.louvain_static(g, mode="async")
    else:
        st, gs = getattr(lib, "louvain_" + approach)(g, bb, lib.State.from_host(*state0), mode="async")
    C, K, S = st.host()
    assert np.array_equal(K, G.degrees())
    assert np.array_equal(S, np.bincount(C, weights=K, minlength=e.n).astype(np.int64))
    q = lib.modularity(g, st.C)
    assert abs(q - G.modularity(C)) < 1e-12
    assert q >= q_static - 1e-3, (q, q_static)


def test_apply_batch_errors_leave_graph_unchanged(lib):
    e = W.random_small_graph(300, 900, 4)
    g = lib.Graph.from_edges(e, slack_frac=0.0, slack_min=0)
    before = g.csr_host()
    present = set(zip(e.u.tolist(), e.v.tolist()))
    a, c = next((a, c) for a in range(300) for c in range(a + 1, 300) if (a, c) not in present)
    z = np.zeros(0, np.int32)
    cases = [
        (lib.LV_ENOEDGE, W.Batch(np.array([a], np.int32), np.array([c], np.int32), np.array([1], np.int32), z, z, z)),
        (lib.LV_ENOEDGE, W.Batch(e.u[:1], e.v[:1], e.w[:1] + 1, z, z, z)),
        (lib.LV_EINVAL, W.Batch(z, z, z, np.array([a, c], np.int32), np.array([c, a], np.int32),
                                np.array([1, 1], np.int32))),
        (lib.LV_EINVAL, W.Batch(z, z, z, np.array([5], np.int32), np.array([5], np.int32), np.array([1], np.int32))),
        (lib.LV_EINVAL, W.Batch(z, z, z, np.array([5], np.int32), np.array([300], np.int32), np.array([1], np.int32))),
        (lib.LV_ENOSLACK, W.Batch(z, z, z, np.array([a], np.int32), np.array([c], np.int32), np.array([1], np.int32))),
    ]
    for code, b in cases:
        with pytest.raises(lib.LouvainError) as ex:
            lib.apply_batch(g, lib.Batch.from_host(b))
        assert ex.value.code == code
        after = g.csr_host()
        assert all(np.array_equal(x, y) for x, y in zip(before, after))
    # after LV_ENOSLACK: relayout with slack, retry, same result as the oracle
    g2 = g.relayout(slack_frac=0.5, slack_min=4)
    b = cases[-1][1]
    lib.apply_batch(g2, lib.Batch.from_host(b))
    G = _orc(e)
    assert G.apply_batch(b) == 0
    assert all(np.array_equal(x, y) for x, y in zip(g2.csr_host(), G.csr()))


@pytest.mark.parametrize("approach", ["nd", "ds", "df"])
def test_dynamic_calls_report_batches_outside_the_graph(lib, approach):
    """A batch that apply_batch would refuse (a vertex id outside [0, n), a
    self-loop), passed straight to a dynamic call, is reported as
    LV_EINVAL: the kernels check each update's ids before using them."""
    e = W.random_small_graph(300, 900, 4)
    g = lib.Graph.from_edges(e, slack_frac=0.5, slack_min=4)
    st0, _ = lib.louvain_static(g, mode="sync")
    z = np.zeros(0, np.int32)
    one = np.array([1], np.int32)
    bad = [W.Batch(z, z, z, np.array([5], np.int32), np.array([300], np.int32), one),
           W.Batch(np.array([-1], np.int32), np.array([7], np.int32), one, z, z, z),
           W.Batch(z, z, z, np.array([9], np.int32), np.array([9], np.int32), one)]
    for b in bad:
        with pytest.raises(lib.LouvainError) as ex:
            getattr(lib, "louvain_" + approach)(g, lib.Batch.from_host(b), st0.clone(), mode="sync")
        assert ex.value.code == lib.LV_EINVAL
    # the graph and a valid call are unaffected
    b = W.random_batch(e, 20, 5)
    lib.apply_batch(g, lib.Batch.from_host(b))
    st, _ = getattr(lib, "louvain_" + approach)(g, lib.Batch.from_host(b), st0.clone(), mode="sync")
    G = _orc(e)
    s0 = G.louvain("static", mode="sync")[:3]
    assert G.apply_batch(b) == 0
    Co, Ko, So, _ = G.louvain(approach, batch=b, state=s0, mode="sync")
    C, K, S = st.host()
    assert np.array_equal(C, Co) and np.array_equal(K, Ko) and np.array_equal(S, So)


def test_batch_deleting_and_reinserting_same_pair(lib):
    e = W.random_small_graph(200, 700, 8, max_w=4)
    z = np.zeros(0, np.int32)
    # delete three edges whole, one partially, and re-insert two of them
    d_u, d_v, d_w = e.u[:4].copy(), e.v[:4].copy(), e.w[:4].copy()
    d_w[3] = max(1, d_w[3] - 1) if e.w[3] > 1 else d_w[3]
    b = W.Batch(d_u, d_v, d_w, e.v[:2].copy(), e.u[:2].copy(), np.array([3, 5], np.int32))
    G = _orc(e)
    assert G.apply_batch(b) == 0
    g = lib.Graph.from_edges(e)
    lib.apply_batch(g, lib.Batch.from_host(b))
    assert all(np.array_equal(x, y) for x, y in zip(g.csr_host(), G.csr()))
    assert g.two_m == G.two_m


def test_empty_batch_and_degenerate_graphs(lib):
    e = W.config1_sbm()
    G = _orc(e)
    state0 = G.louvain("static", mode="sync")[:3]
    g = lib.Graph.from_edges(e)
    st, gs = lib.louvain_df(g, lib.Batch.empty(), lib.State.from_host(*state0), mode="sync")
    C, K, S = st.host()
    assert np.array_equal(C, state0[0]) and gs["iterations"] == [1] and gs["vertices_affected"] == 0
    # one edge among many isolated vertices
    one = W.Edges(97, np.array([3], np.int32), np.array([90], np.int32), np.array([2], np.int32))
    g1 = lib.Graph.from_edges(one)
    st1, s1 = lib.louvain_static(g1, mode="sync")
    Co, Ko, So, so = _orc(one).louvain("static", mode="sync")
    assert np.array_equal(st1.host()[0], Co) and np.array_equal(st1.host()[2], So)
    _same_stats(s1, so)
    # no edges at all
    none = W.Edges(10, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    g0 = lib.Graph.from_edges(none)
    with pytest.raises(lib.LouvainError) as ex:
        lib.louvain_static(g0, mode="sync")
    assert ex.value.code == lib.LV_EEMPTY


def test_graph_build_rejects_bad_edges(lib):
    bad = W.Edges(10, np.array([1, 2], np.int32), np.array([1, 3], np.int32), np.array([1, 1], np.int32))
    with pytest.raises(lib.LouvainError) as ex:
        lib.Graph.from_edges(bad)
    assert ex.value.code == lib.LV_EINVAL


def test_chained_batches_df_sync(lib):
    """Three consecutive DF updates stay bit-exact (state carried on both sides)."""
    e = W.rmat(13, 8, 0.57, 0.19, 0.19, 21)
    G = _orc(e)
    g = lib.Graph.from_edges(e)
    so = G.louvain("static", mode="sync")[:3]
    sg, _ = lib.louvain_static(g, mode="sync")
    cur = e
    for t in range(3):
        b = W.random_batch(cur, 60, 300 + t)
        cur = W.apply_batch_np(cur, b)
        assert G.apply_batch(b) == 0
        bb = lib.Batch.from_host(b)
        lib.apply_batch(g, bb)
        Co, Ko, Sto, os_ = G.louvain("df", batch=b, state=so, mode="sync")
        sg, gs = lib.louvain_df(g, bb, sg, mode="sync")
        C, K, S = sg.host()
        assert np.array_equal(C, Co) and np.array_equal(K, Ko) and np.array_equal(S, Sto)
        assert np.array_equal(sg.size.cpu().numpy(), _sizes(C, e.n))
        _same_stats(gs, os_)
        so = (Co, Ko, Sto)


def test_static_fills_sizes(lib, case):
    name, e = case
    g = lib.Graph.from_edges(e)
    for mode in ("sync", "async"):
        st, _ = lib.louvain_static(g, mode=mode)
        assert np.array_equal(st.size.cpu().numpy(), _sizes(st.host()[0], e.n))


def _hub_batches(e, seed):
    """Batches that hit the two hubs of the star graph hard: many whole and
    partial deletions on one row (holes in its head and its tail), merges,
    appends, and pairs deleted whole and re-inserted in the same batch."""
    rng = np.random.default_rng(seed)
    m = e.m
    hub = np.flatnonzero((e.u == 0) | (e.u == 1))
    pick = rng.choice(hub, size=len(hub) * 2 // 5, replace=False)
    d_w = e.w[pick].copy()
    part = rng.random(len(pick)) < 0.2
    d_w[part & (d_w > 1)] -= 1
    # re-insert a third of the whole deletions, append new pairs at the hub
    whole = pick[~part | (e.w[pick] == 1)]
    back = whole[: len(whole) // 3]
    present = set(zip(e.u.tolist(), e.v.tolist()))
    fresh = [(0, v) for v in range(3001, e.n) if (0, v) not in present][:150]
    merge = rng.choice(np.setdiff1d(np.arange(m), pick), size=80, replace=False)
    iu = np.concatenate([e.v[back], np.array([p[1] for p in fresh], np.int64), e.u[merge]]).astype(np.int32)
    iv = np.concatenate([e.u[back], np.array([p[0] for p in fresh], np.int64), e.v[merge]]).astype(np.int32)
    iw = rng.integers(1, 4, len(iu)).astype(np.int32)
    return W.Batch(e.u[pick].copy(), e.v[pick].copy(), d_w, iu, iv, iw)


def test_apply_batch_hub_rows(lib):
    """Row-centric batch editing on rows of thousands of arcs, applied twice
    in a row: CSR and 2m equal the oracle's after each batch."""
    e = _star_plus(11)
    G = _orc(e)
    g = lib.Graph.from_edges(e, slack_frac=0.5, slack_min=8)
    cur = e
    for t in range(2):
        b = _hub_batches(cur, 40 + t)
        assert G.apply_batch(b) == 0
        lib.apply_batch(g, lib.Batch.from_host(b))
        assert all(np.array_equal(x, y) for x, y in zip(g.csr_host(), G.csr()))
        assert g.two_m == G.two_m
        cur = W.apply_batch_np(cur, b)


def _segment_heavy_hub(n=60000, deg=12000, crowd=7000, seed=13):
    """Vertex 0 adjacent to `deg` others, `crowd` of which hash into the
    first of its ceil(2 deg / 4096) segments (multiplicative hash of the id,
    as in a SYNC sweep from singletons the community ids are the vertex
    ids): that segment then holds more keys than one decide pass takes.
    Plus a ring and random chords so the other rows have neighbours."""
    rng = np.random.default_rng(seed)
    ns = -(-2 * deg // 4096)
    ids = np.arange(1, n, dtype=np.uint64)
    h = (ids * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    seg = (h * np.uint64(ns)) >> np.uint64(32)
    first = ids[seg == 0].astype(np.int64)
    other = ids[seg != 0].astype(np.int64)
    nb = np.concatenate([rng.choice(first, crowd, replace=False), rng.choice(other, deg - crowd, replace=False)])
    pairs = {(0, int(v)) for v in nb}
    for v in range(1, n - 1):
        pairs.add((v, v + 1))
    while len(pairs) < deg + n + 20000:
        a, b = rng.integers(1, n, 2)
        if a != b:
            pairs.add((int(min(a, b)), int(max(a, b))))
    a = np.array(sorted(pairs), dtype=np.int32)
    return W.Edges(n, a[:, 0].copy(), a[:, 1].copy(), np.ones(a.shape[0], np.int32))


def _long_star(leaves=(1 << 20) + 5000, seed=17):
    """A hub row longer than 2^20 arcs (the global-table path), leaves in a
    ring with random chords."""
    rng = np.random.default_rng(seed)
    n = leaves + 1
    u = [np.zeros(leaves, np.int64), np.arange(1, n - 1, dtype=np.int64)]
    v = [np.arange(1, n, dtype=np.int64), np.arange(2, n, dtype=np.int64)]
    a, b = rng.integers(1, n, 200000), rng.integers(1, n, 200000)
    u.append(np.minimum(a, b))
    v.append(np.maximum(a, b))
    uu, vv = np.concatenate(u), np.concatenate(v)
    ok = uu != vv
    keys = np.unique(uu[ok] * n + vv[ok])
    return W.Edges(n, (keys // n).astype(np.int32), (keys % n).astype(np.int32), np.ones(keys.shape[0], np.int32))


@pytest.mark.parametrize("make", [_segment_heavy_hub, _long_star], ids=["segment_overflow", "global_table"])
def test_hub_paths_sync_bit_exact(lib, make):
    """The hub decide unit's multi-pass path (a segment with more keys than
    one pass holds) and the global-table path of rows above 2^20 arcs: one
    SYNC sweep from singletons and a full SYNC static run match the oracle
    bit for bit."""
    e = make()
    g = lib.Graph.from_edges(e)
    G = _orc(e)
    for kw in (dict(max_iterations=1, max_passes=1), dict()):
        st, gs = lib.louvain_static(g, mode="sync", **kw)
        C, K, S = st.host()
        Co, Ko, So, os_ = G.louvain("static", mode="sync", **kw)
        assert np.array_equal(C, Co) and np.array_equal(K, Ko) and np.array_equal(S, So)
        _same_stats(gs, os_)


def test_autotune_picks_a_candidate_and_keeps_results(lib):
    """The autotuner leaves one of its candidate thresholds in force, and
    SYNC results under it still match the oracle."""
    e = W.rmat(14, 8, 0.57, 0.19, 0.19, 6)
    g = lib.Graph.from_edges(e)
    try:
        t = lib.autotune(g, repeats=1)
        assert t["wave_max_degree"] in (64, 128, 256, 512)
        assert lib.get_tuning()["wave_max_degree"] == t["wave_max_degree"]
        st, gs = lib.louvain_static(g, mode="sync")
        Co, Ko, So, os_ = _orc(e).louvain("static", mode="sync")
        assert np.array_equal(st.C.cpu().numpy(), Co) and np.array_equal(st.Sigma.cpu().numpy(), So)
        _same_stats(gs, os_)
    finally:
        lib.set_tuning()


def test_bin_stats_and_timing_hook(lib):
    """Per-bin work adds up to the scan totals, and the event hook times
    exactly the launches it was asked for."""
    e = W.rmat(12, 16, 0.57, 0.19, 0.19, 5)
    g = lib.Graph.from_edges(e)
    _, s = lib.louvain_static(g, mode="sync")
    assert sum(s["bin_arcs"]) == s["arcs_scanned"]
    assert all(x == 0 for x in s["timed_launches"])
    lib.set_timing(range(lib.NTIMED))
    try:
        _, t = lib.louvain_static(g, mode="async")
    finally:
        lib.set_timing(())
    rounds = t["timed_launches"][lib.TIME_BINNING]
    assert rounds >= sum(t["iterations"])
    assert rounds <= t["timed_launches"][lib.TIME_SCAN] <= lib.NBINS * rounds  # fused, or one per bin
    assert t["timed_launches"][lib.TIME_HUB_DECIDE] == t["bin_launches"][lib.BINS.index("hub")]
    assert t["timed_launches"][lib.TIME_HUB_CLEAR] == t["bin_launches"][lib.BINS.index("hub")]
    assert all((t["timed_ms"][k] > 0) == (t["timed_launches"][k] > 0) for k in range(lib.NTIMED))
    _, u = lib.louvain_static(g, mode="async")
    assert all(x == 0 for x in u["timed_launches"])


# ---- many graphs in one launch ------------------------------------------------

def _many_cases():
    """Graphs of different sizes and shapes, each with its own batch; the
    star has a row longer than the batched kernel takes (single-graph path),
    and the big SBM batch makes pass 0 run several iterations (continuation
    with aggregation on the single-graph path)."""
    out = []
    for k, e in enumerate([W.config1_sbm(seed=5), W.rmat(11, 8, 0.57, 0.19, 0.19, 31),
                           W.random_small_graph(777, 3000, 41, max_w=5), W.ring_of_cliques(12, 5),
                           _star_plus(17), W.sbm([40] * 25, 0.3, 0.01, 8)]):
        size = max(6, e.m // 100) if k != 5 else e.m // 3
        out.append((e, W.random_batch(e, size, 500 + k)))
    return out


@pytest.mark.parametrize("mode,tol", [("sync", 1e-2), ("sync", 1e-4), ("async", 1e-2)])
def test_many_graphs_match_single_graph_results(lib, mode, tol):
    cases = _many_cases()
    cap = max(b.size for _, b in cases)
    graphs, batches, states, scratches, expect = [], [], [], [], []
    for e, b in cases:
        G = _orc(e)
        s0 = G.louvain("static", mode="sync")[:3]
        assert G.apply_batch(b) == 0
        Co, Ko, So, os_ = G.louvain("df", batch=b, state=s0, mode=mode, tolerance=tol)
        expect.append((G, Co, Ko, So, os_))
        g = lib.Graph.from_edges(e, slack_frac=1.0, slack_min=32)
        st = lib.State.from_host(*s0)
        st.size = torch.from_numpy(_sizes(s0[0], e.n)).cuda()
        graphs.append(g)
        batches.append(lib.Batch.from_host(b))
        states.append(st)
        scratches.append(lib.many_scratch(e.n, cap))
    ws = max(graphs, key=lambda g: g.n * 4 + g.cap).workspace
    status, stats = lib.louvain_df_many(graphs, batches, states, scratches, cap, ws=ws, mode=mode, tolerance=tol)
    assert status == [0] * len(cases), status
    if tol < 1e-2:  # pass 0 of the R-MAT graph iterates, so it continues with aggregation
        assert stats[1]["passes"] > 1
    for (G, Co, Ko, So, os_), g, st, s, (e, _) in zip(expect, graphs, states, stats, cases):
        assert all(np.array_equal(x, y) for x, y in zip(g.csr_host(), G.csr()))
        assert g.two_m == G.two_m
        C, K, S = st.host()
        assert np.array_equal(K, Ko)
        assert np.array_equal(st.size.cpu().numpy(), _sizes(C, e.n))
        assert np.array_equal(S, np.bincount(C, weights=K, minlength=e.n).astype(np.int64))
        if mode == "sync":
            assert np.array_equal(C, Co) and np.array_equal(S, So)
            _same_stats(s, os_)
        else:  # the oracle's ASYNC DF from the same state: the asynchronous mode's quality bar
            q = lib.modularity(g, st.C)
            assert q >= G.modularity(Co) - 1e-3
    # the call restores what the scratch needs: a second round on the same graphs works too
    b2 = [lib.Batch.from_host(W.random_batch(W.apply_batch_np(e, b), 8, 900 + k))
          for k, (e, b) in enumerate(cases)]
    status, _ = lib.louvain_df_many(graphs, b2, states, scratches, cap, ws=ws, mode=mode, tolerance=tol)
    assert status == [0] * len(cases), status


def test_many_graph_replays_match_eager_calls(lib):
    """Batched launches through one descriptor buffer replay a captured
    graph (the first call captures it).  Over a chain of SYNC batches, with
    eager apply_batch + louvain_df calls on twin graphs and synchronisations
    between the replays, every replay's graphs and states equal the twins'."""
    specs = W.multi_sbm_specs(6, 321, n_lo=500, n_hi=4000, b_lo=20, b_hi=300)
    edges = [W.multi_sbm_graph(n, b, sd) for n, b, sd in specs]
    chains, cap = [], 0
    for k, e in enumerate(edges):
        cur, bs = e, []
        for t in range(4):
            b = W.random_batch(cur, max(4, cur.m // 200), 500 + 10 * k + t)
            bs.append(b)
            cap = max(cap, b.size)
            cur = W.apply_batch_np(cur, b)
        chains.append(bs)
    graphs = [lib.Graph.from_edges(e, slack_frac=1.0, slack_min=32) for e in edges]
    twins = [lib.Graph.from_edges(e, slack_frac=1.0, slack_min=32) for e in edges]
    states = [lib.louvain_static(g, mode="sync")[0] for g in graphs]
    twin_states = [st.clone() for st in states]
    scratches = [lib.many_scratch(g.n, cap) for g in graphs]
    desc = torch.empty(int(lib.load().lv_many_desc_bytes(len(graphs))), dtype=torch.uint8, device="cuda")
    ws = max(graphs, key=lambda g: g.n * 4 + g.cap).workspace
    for t in range(4):
        bs = [lib.Batch.from_host(c[t]) for c in chains]
        status, _ = lib.louvain_df_many(graphs, bs, states, scratches, cap, ws=ws, desc=desc, mode="sync")
        assert status == [0] * len(graphs), (t, status)
        for k in range(len(graphs)):
            lib.apply_batch(twins[k], bs[k])
            twin_states[k], _ = lib.louvain_df(twins[k], bs[k], twin_states[k], mode="sync")
        torch.cuda.synchronize()
        for g, tw, st, ts in zip(graphs, twins, states, twin_states):
            assert all(np.array_equal(x, y) for x, y in zip(g.csr_host(), tw.csr_host())), t
            for x, y in zip(st.host(), ts.host()):
                assert np.array_equal(x, y), t
            assert np.array_equal(st.size.cpu().numpy(), ts.size.cpu().numpy()), t


def test_many_graphs_isolate_bad_batches(lib):
    good = [W.random_small_graph(300, 900, 60 + k) for k in range(3)]
    z = np.zeros(0, np.int32)
    e = good[1]
    bad = W.Batch(e.u[:1], e.v[:1], e.w[:1] + 1, z, z, z)  # deletes more weight than present
    batches_h = [W.random_batch(good[0], 20, 70), bad, W.random_batch(good[2], 20, 72)]
    graphs = [lib.Graph.from_edges(x) for x in good]
    before = graphs[1].csr_host()
    states = []
    for g, x in zip(graphs, good):
        st, _ = lib.louvain_static(g, mode="sync")
        states.append(st)
    C1 = states[1].C.clone()
    scratches = [lib.many_scratch(x.n, 32) for x in good]
    status, _ = lib.louvain_df_many(graphs, [lib.Batch.from_host(b) for b in batches_h], states, scratches, 32,
                                    mode="sync")
    assert status == [0, lib.LV_ENOEDGE, 0]
    assert all(np.array_equal(x, y) for x, y in zip(before, graphs[1].csr_host()))
    assert torch.equal(C1, states[1].C)


def test_autotune_many_keeps_results_and_sets_the_class_entry(lib):
    """lv_autotune_many deals its items to the candidate mappings of the
    batched launch (one timed launch each): every item's SYNC result is
    still the sequential oracle's, the chosen candidate becomes the entry
    of the items' size class, and a following louvain_df_many call (which
    uses that entry) stays bit-exact."""
    specs = W.multi_sbm_specs(24, 61, n_lo=400, n_hi=3000, b_lo=10, b_hi=300)
    graphs, states, scratches, orcs, first = [], [], [], [], []
    cap = 0
    cases = []
    for k, (n, b, sd) in enumerate(specs):
        e = W.multi_sbm_graph(int(n), int(b), int(sd))
        b1 = W.random_batch(e, max(4, e.m // 100), 700 + k)
        b2 = W.random_batch(W.apply_batch_np(e, b1), max(4, e.m // 100), 800 + k)
        cases.append((e, b1, b2))
        cap = max(cap, b1.size, b2.size)
    saved = lib.get_many_tuning()
    try:
        for e, b1, _ in cases:
            G = _orc(e)
            s0 = G.louvain("static", mode="sync")[:3]
            g = lib.Graph.from_edges(e, slack_frac=1.0, slack_min=32)
            st = lib.State.from_host(*s0)
            st.size = torch.from_numpy(_sizes(s0[0], e.n)).cuda()
            graphs.append(g)
            states.append(st)
            scratches.append(lib.many_scratch(e.n, cap))
            orcs.append((G, s0))
        ws = max(graphs, key=lambda g: g.n * 4 + g.cap).workspace
        cls = lib.many_size_class(graphs)
        status, stats, best = lib.autotune_many(graphs, [lib.Batch.from_host(c[1]) for c in cases], states,
                                                scratches, cap, ws=ws, mode="sync")
        assert status == [0] * len(cases), status
        assert best["wave_max_degree"] in (32, 64, 128, 256) and best["grid"] == saved[cls]["grid"]
        assert lib.get_many_tuning()[cls] == best
        for (G, s0), (e, b1, _), st in zip(orcs, cases, states):
            assert G.apply_batch(b1) == 0
            Co, Ko, So, _ = G.louvain("df", batch=b1, state=s0, mode="sync")
            C, K, S = st.host()
            assert np.array_equal(C, Co) and np.array_equal(K, Ko) and np.array_equal(S, So)
            first.append((Co, Ko, So))
        status, _ = lib.louvain_df_many(graphs, [lib.Batch.from_host(c[2]) for c in cases], states, scratches, cap,
                                        ws=ws, mode="sync")
        assert status == [0] * len(cases), status
        for (G, _), (e, _, b2), st, s1 in zip(orcs, cases, states, first):
            assert G.apply_batch(b2) == 0
            Co, Ko, So, _ = G.louvain("df", batch=b2, state=s1, mode="sync")
            C, K, S = st.host()
            assert np.array_equal(C, Co) and np.array_equal(K, Ko) and np.array_equal(S, So)
    finally:
        lib.set_many_tuning(saved)


@pytest.mark.gpu
def test_df_large_frontier_keeps_totals_and_sizes_exact(lib):
    """A DF update whose scan runs as one launch over a frontier bound of at
    least 65,536 (2 x 12,000 updates on 2M vertices: sparse, one sub-round):
    there the changes of communities with a total of at least 2m/1024 are
    deferred past the launch and summed per community afterwards.  Totals,
    sizes and degrees must still be exact, over several updates in a row."""
    e = W.chung_lu(2_000_000, 2.1, 8.0, 77, device="cuda")
    g = lib.Graph.from_edges(e, slack_frac=0.2, slack_min=8)
    lib.set_tuning(wave_max_degree=256)
    try:
        st, _ = lib.louvain_static(g, mode="async")
        batches = W.batch_sequence(e, [12000], 3, seed=91)
        for b in batches:
            st, s = lib.louvain_df_apply(g, lib.Batch.from_host(b), st, lib.params(mode="async"))
            assert s["passes"] >= 1
            C, K, S = st.host()
            size = st.size.cpu().numpy()
            deg = np.zeros(e.n, dtype=np.int64)
            rs = g.row_start.cpu().numpy()
            rl = g.row_len.cpu().numpy().astype(np.int64)
            w = g.w.cpu().numpy()
            idx = np.repeat(np.arange(e.n), rl)
            pos = (np.repeat(rs[:-1], rl) + (np.arange(rl.sum()) - np.repeat(np.cumsum(rl) - rl, rl))).astype(np.int64)
            np.add.at(deg, idx, w[pos].astype(np.int64))
            assert np.array_equal(K, deg)
            assert np.array_equal(S, np.bincount(C, weights=K, minlength=e.n).astype(np.int64))
            assert np.array_equal(size, np.bincount(C, minlength=e.n).astype(size.dtype))
            big = S >= int(g.two_m_t.item()) // 1024
            assert big.sum() >= 1  # the deferred path had large communities to defer
    finally:
        lib.set_tuning()
