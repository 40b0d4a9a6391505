"""Independent exact-arithmetic checks used to pin the oracle.

These are written from the definitions (Newman's pairwise modularity,
exhaustive partition search), not from the oracle's code paths.
"""
from fractions import Fraction

import numpy as np


def arcs_of(e):
    """Both arc directions of an undirected edge list."""
    src = np.concatenate([e.u, e.v]).astype(np.int64)
    dst = np.concatenate([e.v, e.u]).astype(np.int64)
    w = np.concatenate([e.w, e.w]).astype(np.int64)
    return src, dst, w


def degrees(n, src, w):
    return np.bincount(src, weights=w, minlength=n).astype(np.int64)


def modularity_pairwise(n, src, dst, w, C) -> Fraction:
    """Q = (1/2m) Σ_{i,j} [A_ij - K_i K_j / 2m] δ(C_i, C_j), summed over all
    ordered vertex pairs, as an exact rational."""
    C = np.asarray(C)
    A = {}
    for s, d, x in zip(src.tolist(), dst.tolist(), w.tolist()):
        A[(s, d)] = A.get((s, d), 0) + x
    K = [0] * n
    for (s, d), x in A.items():
        K[s] += x
    two_m = sum(K)
    tot = Fraction(0)
    for i in range(n):
        for j in range(n):
            if C[i] != C[j]:
                continue
            tot += Fraction(A.get((i, j), 0)) - Fraction(K[i] * K[j], two_m)
    return tot / two_m


def set_partitions(n):
    """All set partitions of n items as restricted-growth label arrays."""
    out = []
    a = [0] * n

    def rec(i, mx):
        if i == n:
            out.append(list(a))
            return
        for l in range(mx + 2):
            a[i] = l
            rec(i + 1, max(mx, l))

    if n == 0:
        return np.zeros((1, 0), dtype=np.int64)
    a[0] = 0
    rec(1, 0)
    return np.asarray(out, dtype=np.int64)


def max_modularity_bruteforce(n, src, dst, w):
    """Exact maximum of Q over every partition (returns numerator, 2m^2 form
    as a Fraction, and one maximising labelling)."""
    P = set_partitions(n)
    K = degrees(n, src, w)
    two_m = int(K.sum())
    same = P[:, src] == P[:, dst]
    sig_in = same.astype(np.int64) @ w
    sig_tot_sq = np.zeros(P.shape[0], dtype=np.int64)
    for lab in range(n):
        s = (P == lab).astype(np.int64) @ K
        sig_tot_sq += s * s
    qnum = two_m * sig_in - sig_tot_sq
    k = int(np.argmax(qnum))
    return Fraction(int(qnum[k]), two_m * two_m), P[k]


def qnum(n, src, dst, w, C):
    """Integer numerator of Q scaled by (2m)^2: 2m Σσ_c - Σ Σ_c^2."""
    C = np.asarray(C, dtype=np.int64)
    K = degrees(n, src, w)
    two_m = int(K.sum())
    sig_in = int(w[C[src] == C[dst]].sum())
    tot = np.bincount(C, weights=K, minlength=n).astype(np.int64)
    return two_m * sig_in - int((tot.astype(object) ** 2).sum())
