"""The hand-worked DF update of tests/golden/df_six_vertex_step.txt (its
comments carry the derivation): the oracle on the CPU, and the HIP library
in both modes on the GPU, must reproduce every value."""
from fractions import Fraction

import numpy as np
import pytest

from tests import golden as G

FX = "df_six_vertex_step.txt"


def test_oracle_reproduces_the_hand_worked_step(orc):
    fx = G.load(FX)
    e, b = G.edges(fx), G.batch(fx)
    g = orc.Graph.from_edges(e)
    C0 = np.array(fx["prev_C"], np.int32)
    K0 = np.array(fx["prev_K"], np.int64)
    S0 = np.array(fx["prev_Sigma"], np.int64)
    assert g.two_m == fx["prev_two_m"]
    assert np.array_equal(g.degrees(), K0)
    assert np.array_equal(np.bincount(C0, weights=K0, minlength=fx["n"]).astype(np.int64), S0)
    f, _ = g.mark("df", b, C0, K0, S0)
    assert np.nonzero(f)[0].tolist() == fx["marked"]
    K1, S1 = orc.update_weights(fx["n"], b, C0, K0, S0)
    assert K1.tolist() == fx["K"] and S1.tolist() == fx["Sigma"]
    assert g.apply_batch(b) == 0
    assert g.two_m == fx["two_m"]
    assert g.degrees().tolist() == fx["K"]
    assert abs(g.modularity(C0) - float(fx["modularity_prev"])) < 1e-15
    for approach, mode in (("df", "sync"), ("df", "async"), ("nd", "sync"), ("nd", "async")):
        C, K, S, st = g.louvain(approach, batch=b, state=(C0, K0, S0), mode=mode)
        assert G.partition(C) == fx["partition"], mode
        assert K.tolist() == fx["K"]
        assert [[int(S[C[grp[0]]])] for grp in G.partition(C)] == fx["community_Sigma"]
        assert st["passes"] == fx["passes"] and st["iterations"] == fx["iterations"], (mode, st)
        assert st["iter_moves"] == fx["iter_moves"] and st["iter_gain"] == fx["iter_gain"], (mode, st)
        assert abs(g.modularity(C) - float(fx["modularity"])) < 1e-15


def test_fixture_modularities_follow_eq1():
    # the two fractions of the fixture, recomputed from its edge list with
    # exact rationals (Eq. 1: sum over communities of sigma/2m - (Sigma/2m)^2)
    fx = G.load(FX)
    w = {}
    for u, v, x in fx["edge"]:
        w[(min(u, v), max(u, v))] = x
    for u, v, x in fx["del"]:
        w[(min(u, v), max(u, v))] -= x
    for u, v, x in fx["ins"]:
        w[(min(u, v), max(u, v))] = w.get((min(u, v), max(u, v)), 0) + x

    def q(groups):
        two_m = 2 * sum(w.values())
        of = {v: k for k, grp in enumerate(groups) for v in grp}
        inside = [0] * len(groups)
        tot = [0] * len(groups)
        for (u, v), x in w.items():
            tot[of[u]] += x
            tot[of[v]] += x
            if of[u] == of[v]:
                inside[of[u]] += 2 * x
        return sum(Fraction(inside[k], two_m) - Fraction(tot[k], two_m) ** 2 for k in range(len(groups)))

    assert 2 * sum(w.values()) == fx["two_m"]
    assert q(fx["partition"]) == fx["modularity"]
    assert q([[0, 1, 2], [3, 4, 5]]) == fx["modularity_prev"]
    # the summed gain of iteration 1, over 2m^2, is the change of Eq. 1
    two_m = fx["two_m"]
    assert Fraction(fx["iter_gain"][0][0] * 2, two_m * two_m) == fx["modularity"] - fx["modularity_prev"]


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["sync", "async"])
def test_hip_path_reproduces_the_hand_worked_step(mode):
    from paper_2404_19634_amd import lib
    lib.load()
    lib.set_tuning()
    fx = G.load(FX)
    e, b = G.edges(fx), G.batch(fx)
    g = lib.Graph.from_edges(e)
    assert g.two_m == fx["prev_two_m"]
    st = lib.State.from_host(fx["prev_C"], fx["prev_K"], fx["prev_Sigma"])
    db = lib.Batch.from_host(b)
    lib.apply_batch(g, db)
    assert g.two_m == fx["two_m"]
    st, s = lib.louvain_df(g, db, st, mode=mode)
    C, K, S = st.host()
    assert G.partition(C) == fx["partition"]
    assert K.tolist() == fx["K"]
    assert [[int(S[C[grp[0]]])] for grp in G.partition(C)] == fx["community_Sigma"]
    assert s["passes"] == fx["passes"] and s["iterations"] == fx["iterations"], dict(s)
    assert s["iter_moves"] == fx["iter_moves"] and s["iter_gain"] == fx["iter_gain"], dict(s)
    assert abs(lib.modularity(g, st.C) - float(fx["modularity"])) < 1e-15
