"""The bound the GPU scan uses to skip candidates before reading their
totals (Eq. 2 scaled by 2m^2 to integers, in the local-moving phase of
Alg. 5): for a vertex i in community d and a neighbouring community
c != d,

    gain(c) = 2m (K_ic - K_id) - K_i (Sigma_c - Sigma_d + K_i)
           <= K_ic (2m - K_i) - t,   t = 2m K_id - K_i (Sigma_d - K_i),

because every member j of c counts the arc j -> i in K_j, so
Sigma_c >= K_ic.  Checked exhaustively on random weighted graphs with
self-loops (aggregated levels have them) and random memberships; a
candidate the bound rejects never has a positive gain."""
import numpy as np
import pytest


def _graph(rng, n, m, loops):
    u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    w = rng.integers(1, 9, m)
    keep = (u != v) | loops
    A = np.zeros((n, n), dtype=np.int64)
    for a, b, x in zip(u[keep], v[keep], w[keep]):
        A[a, b] += x
        if a != b:
            A[b, a] += x
    return A


@pytest.mark.parametrize("seed", range(12))
def test_bound_holds_and_rejected_candidates_cannot_gain(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 40))
    A = _graph(rng, n, int(rng.integers(n, 6 * n)), loops=bool(seed % 2))
    K = A.sum(axis=1)
    two_m = int(K.sum())
    if two_m == 0:
        return
    k = int(rng.integers(1, n + 1))
    C = rng.integers(0, k, n)
    S = np.bincount(C, weights=K, minlength=k).astype(np.int64)
    checked = 0
    for i in range(n):
        d = C[i]
        Ki = int(K[i])
        # weights from i to each community, the self-loop excluded
        row = A[i].copy()
        row[i] = 0
        Kc = np.bincount(C, weights=row, minlength=k).astype(np.int64)
        Kid = int(Kc[d])
        t = two_m * Kid - Ki * (int(S[d]) - Ki)
        for c in np.nonzero(Kc)[0]:
            if c == d:
                continue
            Kic = int(Kc[c])
            gain = two_m * (Kic - Kid) - Ki * (int(S[c]) - int(S[d]) + Ki)
            bound = Kic * (two_m - Ki) - t
            assert int(S[c]) >= Kic
            assert gain <= bound, (i, c, gain, bound)
            if bound <= 0:
                assert gain <= 0
            checked += 1
    assert checked > 0
