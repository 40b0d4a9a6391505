"""Loader of the hand-worked fixtures in this folder (plain text, one key
per line; `|` separates groups)."""
import os
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name: str) -> dict:
    out = {"edge": [], "del": [], "ins": []}
    for line in open(os.path.join(HERE, name)):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, _, rest = line.partition(" ")
        if key in ("edge", "del", "ins"):
            out[key].append(tuple(int(x) for x in rest.split()))
        elif "|" in rest:
            out[key] = [[int(x) for x in g.split()] for g in rest.split("|")]
        elif "/" in rest:
            out[key] = Fraction(rest.strip())
        else:
            vals = [int(x) for x in rest.split()]
            out[key] = vals[0] if len(vals) == 1 and key in ("n", "two_m", "prev_two_m", "passes") else vals
    return out


def edges(fx):
    from paper_2404_19634_amd import workloads as W
    a = np.array(fx["edge"], dtype=np.int32)
    return W.Edges(fx["n"], a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy())


def batch(fx):
    from paper_2404_19634_amd import workloads as W
    d = np.array(fx["del"], dtype=np.int32).reshape(-1, 3)
    i = np.array(fx["ins"], dtype=np.int32).reshape(-1, 3)
    return W.Batch(d[:, 0].copy(), d[:, 1].copy(), d[:, 2].copy(), i[:, 0].copy(), i[:, 1].copy(), i[:, 2].copy())


def partition(C) -> list:
    """Memberships as sorted member lists, ordered by smallest member."""
    groups = {}
    for v, c in enumerate(np.asarray(C).tolist()):
        groups.setdefault(c, []).append(v)
    return sorted(groups.values())
