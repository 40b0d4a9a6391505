"""Seeded synthetic graphs and batch updates.

This module only draws random numbers and builds edge lists; it holds none of
the community-detection arithmetic.  Both the HIP path and the sequential
oracle take their inputs from here, so the two never feed each other.

Conventions shared by every generator:

* an undirected graph is returned as ``Edges(n, u, v, w)`` with every edge
  listed once, ``u < v``, no self-loops and no duplicate pairs; ``u``, ``v``
  and ``w`` are ``int32`` numpy arrays and weights are positive integers
  (unit weights unless merging duplicates makes them larger);
* a batch update is ``Batch(del_*, ins_*)``: deletions are existing edges,
  removed whole (their current weight), insertions are absent pairs with
  weight 1.  This follows the paper's random-batch recipe (Section 5.1.4:
  80% insertions of uniformly chosen vertex pairs, 20% deletions of
  uniformly chosen existing edges, unit weights, undirected, no new
  vertices).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Edges", "Batch", "sbm", "config1_sbm", "rmat", "config2_rmat",
    "random_batch", "batch_size", "batch_sequence", "real_weights", "real_batch", "two_cliques_bridge", "ring_of_cliques",
    "random_small_graph", "apply_batch_np", "chung_lu", "config3_chung_lu", "pa_temporal_stream",
    "temporal_workload", "config4_temporal", "multi_sbm_specs",
]


@dataclass
class Edges:
    n: int
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray

    @property
    def m(self) -> int:
        return int(self.u.shape[0])


@dataclass
class Batch:
    del_u: np.ndarray
    del_v: np.ndarray
    del_w: np.ndarray
    ins_u: np.ndarray
    ins_v: np.ndarray
    ins_w: np.ndarray

    @property
    def size(self) -> int:
        return int(self.del_u.shape[0] + self.ins_u.shape[0])


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _canon(u: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    a = np.minimum(u, v).astype(np.int64)
    b = np.maximum(u, v).astype(np.int64)
    return a * np.int64(n) + b


def _from_keys(keys: np.ndarray, n: int, w=None) -> Edges:
    keys = np.asarray(keys, dtype=np.int64)
    u = keys // n
    v = keys % n
    if w is None:
        w = np.ones(keys.shape[0], dtype=np.int32)
    return Edges(int(n), _i32(u), _i32(v), _i32(w))


def _distinct_pairs(sample, k: int, rng, exclude=None) -> np.ndarray:
    """Draw ``k`` distinct canonical pair keys from ``sample(count, rng)``.

    ``sample`` returns candidate keys (possibly repeated, ``-1`` for rejects).
    Candidates are kept in the order drawn, so the first ``k`` distinct ones
    are a uniform ``k``-subset of the pairs ``sample`` draws uniformly.
    """
    if k <= 0:
        return np.zeros(0, dtype=np.int64)
    got = np.zeros(0, dtype=np.int64)
    want = k
    while True:
        cand = sample(max(64, int(want * 1.3) + 16), rng)
        cand = cand[cand >= 0]
        if exclude is not None and exclude.shape[0] > 0:
            pos = np.searchsorted(exclude, cand)
            pos = np.minimum(pos, exclude.shape[0] - 1)
            cand = cand[exclude[pos] != cand]
        allc = np.concatenate([got, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        got = allc[first]
        if got.shape[0] >= k:
            return got[:k]
        want = k - got.shape[0]


# ---------------------------------------------------------------------------
# Stochastic block model (planted partition)
# ---------------------------------------------------------------------------

def sbm(block_sizes, p_in, p_out, seed: int) -> Edges:
    """Planted-partition SBM: pairs inside a block appear with probability
    ``p_in`` (a scalar or one value per block), pairs across blocks with
    ``p_out``.  Edge counts are Binomial and the edges a uniform subset of the
    eligible pairs, which is the same distribution as independent
    Bernoulli draws per pair."""
    rng = np.random.default_rng(seed)
    bs = np.asarray(block_sizes, dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(bs)[:-1]])
    n = int(bs.sum())
    pin = np.broadcast_to(np.asarray(p_in, dtype=np.float64), bs.shape)
    pairs_in = bs * (bs - 1) // 2
    k_in = rng.binomial(pairs_in, np.clip(pin, 0.0, 1.0))
    total_in = int(k_in.sum())
    # intra-block: per block, its own count, pairs uniform inside the block
    keys_in = []
    blk_of_edge = np.repeat(np.arange(bs.shape[0]), k_in)
    if total_in:
        # draw per block with rejection, vectorised over all blocks at once
        need = k_in.copy()
        acc = [np.zeros(0, dtype=np.int64) for _ in range(bs.shape[0])]
        have = np.zeros(bs.shape[0], dtype=np.int64)
        active = np.nonzero(need > 0)[0]
        while active.shape[0]:
            reps = np.maximum((need[active] - have[active]) * 13 // 10 + 4, 4)
            blk = np.repeat(active, reps)
            a = starts[blk] + (rng.random(blk.shape[0]) * bs[blk]).astype(np.int64)
            b = starts[blk] + (rng.random(blk.shape[0]) * bs[blk]).astype(np.int64)
            ok = a != b
            blk, a, b = blk[ok], a[ok], b[ok]
            key = np.minimum(a, b) * n + np.maximum(a, b)
            order = np.argsort(blk, kind="stable")
            blk, key = blk[order], key[order]
            bounds = np.searchsorted(blk, active)
            ends = np.searchsorted(blk, active, side="right")
            nxt = []
            for t, bidx in enumerate(active):
                allk = np.concatenate([acc[bidx], key[bounds[t]:ends[t]]])
                _, first = np.unique(allk, return_index=True)
                first.sort()
                acc[bidx] = allk[first][: need[bidx]]
                have[bidx] = acc[bidx].shape[0]
                if have[bidx] < need[bidx]:
                    nxt.append(bidx)
            active = np.asarray(nxt, dtype=np.int64)
        keys_in = np.concatenate(acc) if acc else np.zeros(0, dtype=np.int64)
    else:
        keys_in = np.zeros(0, dtype=np.int64)
    del blk_of_edge
    # inter-block: one Binomial over all cross pairs, uniform cross pairs
    pairs_all = n * (n - 1) // 2
    pairs_out = pairs_all - int(pairs_in.sum())
    k_out = int(rng.binomial(pairs_out, min(max(float(p_out), 0.0), 1.0))) if pairs_out > 0 else 0
    block_id = np.repeat(np.arange(bs.shape[0]), bs)

    def sample_out(cnt, r):
        a = r.integers(0, n, cnt, dtype=np.int64)
        b = r.integers(0, n, cnt, dtype=np.int64)
        key = np.minimum(a, b) * n + np.maximum(a, b)
        key[block_id[a] == block_id[b]] = -1
        return key

    keys_out = _distinct_pairs(sample_out, k_out, rng)
    keys = np.sort(np.concatenate([keys_in, keys_out]))
    return _from_keys(keys, n)


def config1_sbm(seed: int = 1235) -> Edges:
    """10,000 vertices in 50 blocks of 200; expected intra-degree 16 and
    inter-degree 4; unit weights."""
    b, nb = 200, 50
    n = b * nb
    return sbm([b] * nb, 16.0 / (b - 1), 4.0 / (n - b), seed)


# ---------------------------------------------------------------------------
# R-MAT
# ---------------------------------------------------------------------------

def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         chunk: int = 1 << 23) -> Edges:
    """R-MAT: ``edge_factor * 2**scale`` sampled arcs, each descending
    ``scale`` quadrant choices with probabilities (a, b, c, 1-a-b-c).  Self
    pairs are dropped, the rest symmetrised and duplicates merged into
    integer weights; isolated vertices are kept."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    total = edge_factor * n
    keys = []
    ab, abc = a + b, a + b + c
    for lo in range(0, total, chunk):
        cnt = min(chunk, total - lo)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(cnt)
            bu = (r >= ab).astype(np.int64)            # quadrants c, d: lower half
            bv = ((r >= a) & (r < ab)) | (r >= abc)    # quadrants b, d: right half
            u = (u << 1) | bu
            v = (v << 1) | bv.astype(np.int64)
        ok = u != v
        keys.append(np.minimum(u[ok], v[ok]) * n + np.maximum(u[ok], v[ok]))
    allk = np.concatenate(keys)
    del keys
    uk, cnts = np.unique(allk, return_counts=True)
    return _from_keys(uk, n, cnts)


def _cache_dir():
    d = os.environ.get("LV_WORKLOAD_CACHE", "/tmp/lv_workloads")
    return d or None


def _cached(name: str, make):
    d = _cache_dir()
    if d:
        path = os.path.join(d, name + ".npz")
        if os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            return Edges(int(z["n"]), z["u"], z["v"], z["w"])
    e = make()
    if d:
        os.makedirs(d, exist_ok=True)
        tmp = os.path.join(d, name + f".tmp{os.getpid()}.npz")
        np.savez(tmp, n=np.int64(e.n), u=e.u, v=e.v, w=e.w)
        os.replace(tmp, path)
    return e


def config2_rmat(scale: int = 22, seed: int = 1236) -> Edges:
    """R-MAT, edge factor 16, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05)."""
    return _cached(f"rmat_s{scale}_ef16_seed{seed}",
                   lambda: rmat(scale, 16, 0.57, 0.19, 0.19, seed))


# ---------------------------------------------------------------------------
# Random batch updates (Section 5.1.4)
# ---------------------------------------------------------------------------

def batch_size(fraction: float, m: int) -> int:
    """Number of undirected updates for a batch of ``fraction * |E|``."""
    return max(1, int(round(fraction * m)))


def random_batch(g: Edges, size: int, seed: int, ins_frac: float = 0.8) -> Batch:
    """``size`` undirected updates: ``round(ins_frac*size)`` insertions of
    uniformly drawn absent vertex pairs (weight 1) and the rest deletions of
    uniformly drawn existing edges (whole weight)."""
    rng = np.random.default_rng(seed)
    n_ins = int(round(ins_frac * size))
    n_del = size - n_ins
    n_del = min(n_del, g.m)
    pick = rng.choice(g.m, n_del, replace=False) if n_del else np.zeros(0, dtype=np.int64)
    pick = np.sort(pick)
    existing = np.sort(_canon(g.u, g.v, g.n))
    n = g.n

    def sample_ins(cnt, r):
        a = r.integers(0, n, cnt, dtype=np.int64)
        b = r.integers(0, n, cnt, dtype=np.int64)
        key = np.minimum(a, b) * n + np.maximum(a, b)
        key[a == b] = -1
        return key

    ins = _distinct_pairs(sample_ins, n_ins, rng, exclude=existing)
    # random orientation so both endpoint orders appear in the batch
    flip = rng.random(ins.shape[0]) < 0.5
    iu, iv = ins // n, ins % n
    iu, iv = np.where(flip, iv, iu), np.where(flip, iu, iv)
    return Batch(_i32(g.u[pick]), _i32(g.v[pick]), _i32(g.w[pick]),
                 _i32(iu), _i32(iv), np.ones(ins.shape[0], dtype=np.int32))


def real_weights(e: Edges, seed: int, lo: float = 0.25, hi: float = 4.0) -> Edges:
    """The same edges with float32 weights drawn uniformly from [lo, hi)
    (seeded): the weighted graphs of the paper's precision (Section 5.1.2
    keeps edge weights in 32-bit floats)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(lo, hi, e.m).astype(np.float32)
    return Edges(e.n, e.u, e.v, w)


def real_batch(b: Batch, g: Edges, seed: int, lo: float = 0.25, hi: float = 4.0) -> Batch:
    """A batch for a real-weighted graph `g`: deletions remove the whole
    current weight of their edge (looked up in g), insertions get float32
    weights drawn uniformly from [lo, hi) (seeded)."""
    keys = _canon(g.u, g.v, g.n)
    order = np.argsort(keys)
    pos = order[np.searchsorted(keys[order], _canon(b.del_u, b.del_v, g.n))]
    rng = np.random.default_rng(seed)
    return Batch(b.del_u, b.del_v, np.asarray(g.w, dtype=np.float32)[pos], b.ins_u, b.ins_v,
                 rng.uniform(lo, hi, b.ins_u.shape[0]).astype(np.float32))


def batch_sequence(g: Edges, sizes, count: int, seed: int) -> list:
    """``count`` batches cycling through ``sizes`` (undirected updates), each
    80% insertions of absent uniform pairs and 20% deletions of uniform
    existing edges.  All are drawn at once from disjoint pools, so applying
    them in sequence is always valid (a deletion's edge still exists, an
    insertion's pair is still absent)."""
    plan = [sizes[k % len(sizes)] for k in range(count)]
    n_ins = [int(round(0.8 * s)) for s in plan]
    n_del = [s - i for s, i in zip(plan, n_ins)]
    pool = random_batch(g, sum(n_ins) + sum(n_del), seed, ins_frac=sum(n_ins) / max(1, sum(plan)))
    out, pi, pd = [], 0, 0
    for a, d in zip(n_ins, n_del):
        out.append(Batch(pool.del_u[pd:pd + d], pool.del_v[pd:pd + d], pool.del_w[pd:pd + d],
                         pool.ins_u[pi:pi + a], pool.ins_v[pi:pi + a], pool.ins_w[pi:pi + a]))
        pi += a
        pd += d
    return out


def apply_batch_np(g: Edges, b: Batch) -> Edges:
    """Edge list after the batch (deletions subtract, then insertions add);
    used by generators that chain batches, not by either implementation."""
    n = g.n
    real = np.issubdtype(np.asarray(g.w).dtype, np.floating)
    acc = np.float32 if real else np.int64   # float32 weights stay float32, as the implementations keep them
    keys = _canon(g.u, g.v, n)
    w = g.w.astype(acc).copy()
    order = np.argsort(keys)
    keys, w = keys[order], w[order]
    dk = _canon(b.del_u, b.del_v, n)
    pos = np.searchsorted(keys, dk)
    w[pos] -= np.asarray(b.del_w).astype(acc)
    ik = _canon(b.ins_u, b.ins_v, n)
    allk = np.concatenate([keys, ik])
    allw = np.concatenate([w, np.asarray(b.ins_w).astype(acc)])
    uk, inv = np.unique(allk, return_inverse=True)
    ww = np.zeros(uk.shape[0], dtype=acc)
    np.add.at(ww, inv, allw)
    keep = ww > 0
    if real:
        return Edges(int(n), _i32(uk[keep] // n), _i32(uk[keep] % n), ww[keep].astype(np.float32))
    return _from_keys(uk[keep], n, ww[keep])


# ---------------------------------------------------------------------------
# Small structured graphs with known optimal partitions
# ---------------------------------------------------------------------------

def _clique_keys(base: int, k: int, n: int):
    a, b = np.triu_indices(k, 1)
    return (a + base).astype(np.int64) * n + (b + base)


def two_cliques_bridge(k: int) -> Edges:
    """Two K_k cliques (vertices 0..k-1 and k..2k-1) joined by the edge
    (k-1, k)."""
    n = 2 * k
    keys = np.concatenate([_clique_keys(0, k, n), _clique_keys(k, k, n),
                           np.array([(k - 1) * n + k], dtype=np.int64)])
    return _from_keys(np.sort(keys), n)


def ring_of_cliques(r: int, k: int) -> Edges:
    """``r`` K_k cliques; clique t holds vertices t*k..t*k+k-1 and its last
    vertex links to the first vertex of clique t+1 (mod r)."""
    n = r * k
    parts = [_clique_keys(t * k, k, n) for t in range(r)]
    for t in range(r):
        a = t * k + k - 1
        b = ((t + 1) % r) * k
        parts.append(np.array([min(a, b) * n + max(a, b)], dtype=np.int64))
    return _from_keys(np.unique(np.concatenate(parts)), n)


def random_small_graph(n: int, m: int, seed: int, max_w: int = 1) -> Edges:
    """Uniform random simple graph with ``m`` edges and weights in
    [1, max_w]."""
    rng = np.random.default_rng(seed)
    m = min(m, n * (n - 1) // 2)

    def sample(cnt, r):
        a = r.integers(0, n, cnt, dtype=np.int64)
        b = r.integers(0, n, cnt, dtype=np.int64)
        key = np.minimum(a, b) * n + np.maximum(a, b)
        key[a == b] = -1
        return key

    keys = np.sort(_distinct_pairs(sample, m, rng))
    w = rng.integers(1, max_w + 1, keys.shape[0]) if max_w > 1 else None
    return _from_keys(keys, n, w)


# ---------------------------------------------------------------------------
# Larger configurations (power-law, temporal, many graphs)
# ---------------------------------------------------------------------------

def _splitmix64(x):
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) of int64 torch
    counters: one independent 64-bit draw per counter.  Plain integer
    arithmetic (wrapping products, logical shifts), so CPU and GPU give the
    same bits."""
    import torch

    def shr(z, k):  # logical right shift of int64
        return (z >> k) & ((1 << (64 - k)) - 1)

    def c64(v):  # unsigned 64-bit constant as a wrapped int64
        return v - (1 << 64) if v >= (1 << 63) else v

    z = x + c64(0x9E3779B97F4A7C15)
    z = (z ^ shr(z, 30)) * c64(0xBF58476D1CE4E5B9)
    z = (z ^ shr(z, 27)) * c64(0x94D049BB133111EB)
    return z ^ shr(z, 31)


def _uniform01(counters):
    """Doubles in [0, 1) from the top 53 bits of SplitMix64 draws."""
    import torch
    h = _splitmix64(counters)
    return ((h >> 11) & ((1 << 53) - 1)).to(torch.float64) * (1.0 / (1 << 53))


def chung_lu(n: int, gamma: float, mean_degree: float, seed: int, m_target: int | None = None,
             device: str = "cpu", chunk: int = 1 << 26) -> Edges:
    """Chung-Lu power-law graph: weights w_i ~ (i+1)^(-1/(gamma-1)) times a
    scale s, capped at sqrt(s * sum_i (i+1)^(-1/(gamma-1))); endpoints drawn
    proportional to w, self pairs and repeats dropped until ``m_target``
    distinct edges (default n*mean_degree/2); unit weights.

    The scale is searched in [1e-6, 1e6] for a mean capped weight of
    ``mean_degree``.  The mean degree itself is fixed by ``m_target``; the
    search only places the cap.  For the 20M-vertex configuration (gamma
    2.1, mean 50) the search ends at its upper bound, where the cap binds on
    the 261 heaviest vertices only (realised maximum degree 144,862).

    The draws are counter-based (SplitMix64 of the draw index and the seed)
    and run in torch on ``device``: the hundreds of millions of draws of
    the 20M-vertex configuration take seconds on a GPU, and any device
    yields the same edge list.  When more than ``m_target`` distinct pairs
    come up, the ones with the smallest SplitMix64 hash of (pair, seed) are
    kept."""
    import torch
    expo = -1.0 / (gamma - 1.0)
    base = np.power(np.arange(1, n + 1, dtype=np.float64), expo)
    total = base.sum()

    def mean_at(scale):
        return np.minimum(base * scale, math.sqrt(total * scale)).mean()

    lo, hi = 1e-6, 1e6
    for _ in range(80):   # bisection on the scale so that mean(w) hits the target
        mid = math.sqrt(lo * hi)
        if mean_at(mid) < mean_degree:
            lo = mid
        else:
            hi = mid
    wv = np.minimum(base * hi, math.sqrt(total * hi))
    cdf = np.cumsum(wv)
    cdf /= cdf[-1]
    dev = torch.device(device)
    tcdf = torch.from_numpy(cdf).to(dev)
    m_target = int(m_target if m_target is not None else round(n * mean_degree / 2))
    stream = (int(seed) & 0xFFFFF) << 42   # draw counters of this seed: 2^42 per seed
    drawn = 0
    keys = torch.zeros(0, dtype=torch.int64, device=dev)
    while keys.numel() < m_target:
        need = m_target - keys.numel()
        cnt = int(need * 1.15) + 1024
        parts = [keys]
        for off in range(0, cnt, chunk):
            c = min(chunk, cnt - off)
            ctr = torch.arange(drawn, drawn + c, dtype=torch.int64, device=dev) * 2 + stream
            drawn += c
            a = torch.searchsorted(tcdf, _uniform01(ctr), right=True)
            b = torch.searchsorted(tcdf, _uniform01(ctr + 1), right=True)
            del ctr
            a.clamp_(max=n - 1)
            b.clamp_(max=n - 1)
            ok = a != b
            a, b = a[ok], b[ok]
            parts.append(torch.minimum(a, b) * n + torch.maximum(a, b))
            del a, b, ok
        keys = torch.unique(torch.cat(parts))
        del parts
    if keys.numel() > m_target:
        h = _splitmix64(keys ^ (int(seed) * 0x2545F4914F6CDD1D % (1 << 62)))
        order = torch.sort(h, stable=True).indices[:m_target]
        keys = torch.sort(keys[order]).values
        del h, order
    u = (keys // n).to(torch.int32).cpu().numpy()
    v = (keys % n).to(torch.int32).cpu().numpy()
    return Edges(int(n), u, v, np.ones(u.shape[0], dtype=np.int32))


def config3_chung_lu(device: str = "cpu") -> Edges:
    """Chung-Lu, 20M vertices, degree exponent 2.1, mean degree 50."""
    return chung_lu(20_000_000, 2.1, 50.0, 1237, device=device)


def pa_temporal_stream(n: int, targets: int, seed: int, block: int = 1024):
    """Preferential-attachment growth: every vertex t >= targets+1 links to
    ``targets`` distinct earlier vertices, drawn with probability
    proportional to degree + 1.  Vertices join in blocks of up to ``block``
    (a quarter of the vertices so far while the graph is small); a block's
    vertices draw from the degrees as they stood when the block began, and
    each takes a uniform choice of ``targets`` among its distinct draws.
    Returns (u, v) int32 arrays in creation order (the temporal order)."""
    rng = np.random.default_rng(seed)
    k = targets
    seed_n = k + 1
    a, b = np.triu_indices(seed_n, 1)
    us, vs = [b.astype(np.int64)], [a.astype(np.int64)]
    # endpoint pool: a uniform draw from it is degree-proportional; the +1
    # smoothing is a uniform draw over the existing vertices
    pool = np.zeros(2 * k * n + 2 * a.shape[0], dtype=np.int64)
    pool[: 2 * a.shape[0]] = np.concatenate([a, b])
    plen = 2 * a.shape[0]
    t = seed_n
    R = 3 * k + 8
    while t < n:
        B = min(block, max(1, t // 4), n - t)
        chosen = np.zeros((B, k), dtype=np.int64)
        todo = np.arange(B)
        while todo.shape[0]:
            x = rng.integers(0, plen + t, (todo.shape[0], R))
            cand = np.where(x < plen, pool[np.minimum(x, plen - 1)], x - plen)
            srt = np.sort(cand, axis=1)
            dup = np.zeros_like(srt, dtype=bool)
            dup[:, 1:] = srt[:, 1:] == srt[:, :-1]
            ok = (~dup).sum(axis=1) >= k
            prio = rng.random(srt.shape)
            prio[dup] = 2.0
            pick = np.argsort(prio, axis=1)[:, :k]
            rows = todo[ok]
            chosen[rows] = np.take_along_axis(srt[ok], pick[ok], axis=1)
            todo = todo[~ok]
        src = np.repeat(np.arange(t, t + B, dtype=np.int64), k)
        dst = chosen.reshape(-1)
        us.append(src)
        vs.append(dst)
        pool[plen:plen + B * k] = src
        pool[plen + B * k:plen + 2 * B * k] = dst
        plen += 2 * B * k
        t += B
    return _i32(np.concatenate(us)), _i32(np.concatenate(vs))


def temporal_workload(n: int, targets: int, seed: int, initial_frac: float = 0.9, batches: int = 100,
                      window: int | None = None):
    """A temporal stream cut into an initial graph and consecutive batches.

    The stream's first ``initial_frac`` of edges (in creation order) are the
    prefix; the graph holds the ``window`` most recent edges of it (all of
    it when ``window`` is None).  Batch j inserts the next slice of the
    remaining edges and deletes the edges that drop out of the window.
    Returns (initial Edges, list of Batch)."""
    u, v = pa_temporal_stream(n, targets, seed)
    E = u.shape[0]
    t0 = int(round(initial_frac * E))
    window = E if window is None else int(window)
    lo = max(0, t0 - window)
    a = np.minimum(u[lo:t0], v[lo:t0]).astype(np.int64)
    b = np.maximum(u[lo:t0], v[lo:t0]).astype(np.int64)
    order = np.argsort(a * n + b)
    g = Edges(int(n), _i32(a[order]), _i32(b[order]), np.ones(t0 - lo, dtype=np.int32))
    cuts = np.linspace(t0, E, batches + 1).round().astype(np.int64)
    out = []
    for j in range(batches):
        s, e = int(cuts[j]), int(cuts[j + 1])
        d0, d1 = max(0, s - window), max(0, e - window)
        one = np.ones(e - s, dtype=np.int32)
        out.append(Batch(_i32(u[d0:d1]), _i32(v[d0:d1]), np.ones(d1 - d0, dtype=np.int32),
                         _i32(u[s:e]), _i32(v[s:e]), one))
    return g, out


def config4_temporal(scale: float = 1.0):
    """Preferential-attachment stream grown to 2M vertices and 30M edges
    (15 per new vertex); the first 90% form the initial graph, the rest
    arrive as 100 batches under a sliding window of the 20M newest edges.
    ``scale`` shrinks vertices and window together for small test cases."""
    n = max(64, int(round(2_000_000 * scale)))
    return temporal_workload(n, 15, 1238, window=int(round(20_000_000 * scale)))


def multi_sbm_specs(count: int, seed: int, n_lo=1000, n_hi=200000, b_lo=20, b_hi=2000):
    """Per-graph (n, block size, seed) for the many-graph workload: vertex
    counts and block sizes log-uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count)).astype(np.int64)
    bs = np.exp(rng.uniform(math.log(b_lo), math.log(b_hi), count)).astype(np.int64)
    bs = np.minimum(bs, ns)
    seeds = rng.integers(0, 2**31 - 1, count)
    return [(int(a), int(b), int(s)) for a, b, s in zip(ns, bs, seeds)]


def multi_sbm_graph(n: int, b: int, seed: int, deg_in=12.0, deg_out=3.0) -> Edges:
    nb = max(1, n // b)
    sizes = [b] * nb
    sizes[-1] += n - b * nb
    p_in = [deg_in / max(1, s - 1) for s in sizes]
    p_out = deg_out / max(1, n - b)
    return sbm(sizes, p_in, p_out, seed)
