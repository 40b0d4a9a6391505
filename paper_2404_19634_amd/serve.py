"""Serving loop: streaming batch updates on device-resident graphs.

Requests name a graph and a batch of edge updates (Section 3.4).  Graphs
and their community state (C, K, Sigma, member counts) stay resident in
HBM between requests; each request is apply_batch + DF Louvain on its
graph (Alg. 1).  The loop batches continuously: worker threads each own a
HIP stream and repeatedly take up to `slots` waiting requests on distinct
graphs, admit their graphs into HBM (evicting idle graphs to host memory
when the byte budget would be exceeded), and run them in one persistent
launch (`louvain_df_many`).  Requests that arrive while a launch is on the
GPU are picked up by the next free worker, so launches overlap on the
device.  Latency is arrival to completion; the summary reports p50/p99
and requests per second.

Only argument marshalling and bookkeeping happen here; every step of the
update runs in the HIP library.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import lib


@dataclass
class Request:
    gid: int
    batch: object          # workloads.Batch (host arrays)
    t_arrival: float
    rid: int = 0
    t_start: float = 0.0
    t_done: float = 0.0
    status: int = 1        # 1 pending, else the library status
    src: tuple = ()        # (per-launch statistics list, index): read on demand
    refreshed: bool = False  # static Louvain replaced the state after this update
    approach: str = "df"     # "df" (batched DF launch) or "ds" (DS fallback after a modularity drop)
    modularity: float = float("nan")  # Q after this update (measured when the DS fallback is on)

    @property
    def stats(self) -> dict:
        return self.src[0][self.src[1]] if self.src else {}


class Resident:
    """A graph, its state and its batched-kernel scratch on the device."""

    def __init__(self, graph: lib.Graph, state: lib.State, scratch: torch.Tensor):
        self.graph, self.state, self.scratch = graph, state, scratch
        self.busy = False
        self.last_used = 0.0
        self.since_refresh = 0  # updates since the state came from static Louvain
        self.q_ref = None       # Q right after the last static run (DS fallback reference)
        self.use_ds = False     # DS fallback in force: Q fell more than ds_drop below q_ref

    @property
    def nbytes(self) -> int:
        g, s = self.graph, self.state
        t = [g.row_start, g.row_len, g.col, g.w, g.two_m_t, s.C, s.K, s.Sigma, s.size, self.scratch]
        return sum(x.numel() * x.element_size() for x in t)


class GraphStore:
    """Graphs by id; at most `budget_bytes` of them resident in HBM.

    A graph enters HBM when a request needs it (built from its edge list
    and given a static Louvain state the first time, copied back from the
    host after an eviction) and leaves, least recently used first, when an
    admission would exceed the budget."""

    def __init__(self, budget_bytes: int, max_updates: int, device="cuda", mode="async", slack_frac=0.5,
                 slack_min=16, init_mode=None, refresh_every=0, ds_drop=None):
        self.budget = int(budget_bytes)
        self.max_updates = int(max_updates)
        self.device = torch.device(device)
        self.mode = mode
        # mode of the static Louvain run that gives an admitted graph its
        # first state (SYNC makes it reproducible run to run)
        self.init_mode = init_mode or mode
        # quality policy (the remedy of the paper's appendix on DF's
        # correctness: communities that a run of deletions splits, and
        # outliers the frontier misses, are repaired by running static
        # Louvain every so many batches): after every `refresh_every`
        # updates of a graph, static Louvain (in init_mode) replaces its
        # state; 0 turns this off
        self.refresh_every = int(refresh_every)
        self.refreshes = 0
        # DS fallback (the paper's advice where DF's modularity falls behind:
        # Delta-screening marks more vertices, Section 5.2.1 and the
        # conclusion): after each update the graph's modularity Q is
        # measured; while it is more than `ds_drop` below Q after the last
        # static run, the graph's updates run apply_batch + DS Louvain
        # instead of the batched DF launch.  None turns this off.
        self.ds_drop = None if ds_drop is None else float(ds_drop)
        self.ds_updates = 0
        self.slack = (slack_frac, slack_min)
        self.edges = {}        # gid -> workloads.Edges (never-admitted graphs)
        self.host = {}         # gid -> evicted device arrays, on the host
        self.res = {}          # gid -> Resident
        self.moving = set()    # gids being evicted or admitted (outside the lock)
        self.lock = threading.Lock()
        self.resident_bytes = 0
        self.evictions = 0
        self.admissions = 0

    def add(self, gid: int, edges) -> None:
        self.edges[gid] = edges

    def _footprint(self, gid) -> int:
        """Device bytes graph `gid` takes once resident (graph, state, scratch)."""
        L = lib.load()
        h = self.host.get(gid)
        if h is not None:
            n, cap = h["n"], h["cap"]
        else:
            e = self.edges[gid]
            n = e.n
            cap = max(int(L.lv_graph_capacity_bound(n, e.m, self.slack[0], self.slack[1])), 1)
        graph = 8 * (n + 1) + 4 * n + 8 * cap + 8
        state = (4 + 8 + 8 + 4) * n
        return graph + state + int(L.lv_many_scratch_bytes(n, self.max_updates))

    def _build(self, gid, h=None) -> Resident:
        """Makes graph `gid` resident: from its evicted arrays `h`, or built
        from its edge list with a static Louvain state.  Runs without the
        store lock."""
        if h is not None:
            g = lib.Graph(h["n"], h["cap"], self.device)
            for name in ("row_start", "row_len", "col", "w", "two_m_t"):
                getattr(g, name).copy_(h[name], non_blocking=False)
            st = lib.State(h["C"].to(self.device), h["K"].to(self.device), h["Sigma"].to(self.device),
                           h["size"].to(self.device))
            since = h["since_refresh"]
            q_ref, use_ds = h["q_ref"], h["use_ds"]
        else:
            e = self.edges[gid]
            g = lib.Graph.from_edges(e, slack_frac=self.slack[0], slack_min=self.slack[1], device=self.device)
            st, _ = lib.louvain_static(g, mode=self.init_mode)
            q_ref = lib.modularity(g, st.C) if self.ds_drop is not None else None
            g._ws = None  # the build workspace is not kept; louvain_df_many needs none per graph
            since, use_ds = 0, False
        scratch = lib.many_scratch(g.n, self.max_updates, self.device)
        r = Resident(g, st, scratch)
        r.since_refresh, r.q_ref, r.use_ds = since, q_ref, use_ds
        return r

    @staticmethod
    def _to_host(r: Resident) -> dict:
        g, s = r.graph, r.state
        return {"n": g.n, "cap": g.cap, "row_start": g.row_start.cpu(), "row_len": g.row_len.cpu(),
                "col": g.col.cpu(), "w": g.w.cpu(), "two_m_t": g.two_m_t.cpu(), "C": s.C.cpu(),
                "K": s.K.cpu(), "Sigma": s.Sigma.cpu(), "size": s.size.cpu(), "since_refresh": r.since_refresh,
                "q_ref": r.q_ref, "use_ds": r.use_ds}

    def _reserve(self, gids):
        """Marks resident graphs busy; for the others reserves their bytes,
        choosing least recently used idle graphs to evict, and marks both
        as moving (no worker takes a moving graph).  Store lock held; only
        bookkeeping happens here."""
        plan, victims = [], []
        for gid in gids:
            r = self.res.get(gid)
            if r is not None:
                r.busy = True
                plan.append((gid, r, 0))
                continue
            nb = self._footprint(gid)
            while self.resident_bytes + nb > self.budget:
                idle = [(x.last_used, g) for g, x in self.res.items() if not x.busy]
                if not idle:
                    break
                _, v = min(idle)
                x = self.res.pop(v)
                self.resident_bytes -= x.nbytes
                self.moving.add(v)
                victims.append((v, x))
                self.evictions += 1
            self.resident_bytes += nb
            self.moving.add(gid)
            plan.append((gid, None, nb))
        return plan, victims

    def acquire(self, gids) -> list:
        """Marks the graphs busy and makes them resident (call without the
        store lock).  Bookkeeping happens under the lock; copies of evicted
        graphs to the host and builds or restores of admitted ones happen
        outside it, so other workers keep scheduling and finishing."""
        with self.lock:
            plan, victims = self._reserve(gids)
        return self._admit(plan, victims)

    def _admit(self, plan, victims) -> list:
        """The device work of an admission planned by _reserve (store lock
        not held): evicted graphs go to the host, planned ones are built or
        restored and published."""
        for v, x in victims:
            h = self._to_host(x)
            with self.lock:
                self.host[v] = h
                self.moving.discard(v)
        out = []
        for gid, r, nb in plan:
            if r is None:
                with self.lock:
                    h = self.host.pop(gid, None)
                r = self._build(gid, h)
                r.busy = True
                with self.lock:
                    self.resident_bytes += r.nbytes - nb
                    self.res[gid] = r
                    self.moving.discard(gid)
                    self.admissions += 1
            out.append(r)
        return out

    def refresh(self, r: Resident, ws: torch.Tensor, stream) -> None:
        """Static Louvain on a resident graph, in place of its state (ws:
        a workspace of at least lv_workspace_bytes for the graph)."""
        r.graph._ws = ws
        try:
            lib.louvain_static(r.graph, lib.params(mode=self.init_mode), r.state, stream=stream)
            if self.ds_drop is not None:
                r.q_ref = lib.modularity(r.graph, r.state.C, stream=stream)
                r.use_ds = False
        finally:
            r.graph._ws = None
        r.since_refresh = 0
        with self.lock:
            self.refreshes += 1

    def tune(self, gids, batches) -> dict:
        """One update per listed graph through lv_autotune_many: the updates
        are applied (results as louvain_df_many's) while the batched launch
        is tuned for their size class.  Call with no worker running.
        Returns the class and the tuning chosen."""
        residents = self.acquire(gids)
        try:
            big = max(residents, key=lambda x: x.graph.n * 4 + x.graph.cap)
            ws = torch.empty(int(lib.load().lv_workspace_bytes(big.graph.n, big.graph.cap)), dtype=torch.uint8,
                             device=self.device)
            dev = [lib.Batch.from_host(b, self.device) for b in batches]
            status, _, best = lib.autotune_many([r.graph for r in residents], dev, [r.state for r in residents],
                                                [r.scratch for r in residents], self.max_updates,
                                                prm=lib.params(mode=self.mode), ws=ws)
            if any(s != 0 for s in status):
                raise RuntimeError(f"tuning pass: statuses {sorted(set(status))}")
        finally:
            self.release(gids)
        return {"size_class": lib.many_size_class([r.graph for r in residents]), "tuning": best}

    @staticmethod
    def save_tuning(path: str) -> None:
        """Writes the batched launch's tuning table (one entry per size
        class) to a JSON file."""
        import json
        with open(path, "w") as f:
            json.dump(lib.get_many_tuning(), f)

    @staticmethod
    def load_tuning(path: str) -> None:
        """Restores a tuning table written by save_tuning."""
        import json
        with open(path) as f:
            lib.set_many_tuning(json.load(f))

    def measure(self, r: Resident, ws: torch.Tensor, stream) -> float:
        """Q of a resident graph's state (Eq. 1); sets or clears its DS
        fallback against the reference of its last static run."""
        r.graph._ws = ws
        try:
            q = lib.modularity(r.graph, r.state.C, stream=stream)
        finally:
            r.graph._ws = None
        r.use_ds = q < r.q_ref - self.ds_drop
        return q

    def ds_update(self, r: Resident, batch: lib.Batch, prm, ws: torch.Tensor, stream) -> int:
        """apply_batch + DS Louvain (Alg. 3) on one resident graph; returns
        the status (LV_ENOSLACK leaves the graph unchanged)."""
        r.graph._ws = ws
        try:
            lib.apply_batch(r.graph, batch, stream=stream)
            lib.louvain_ds(r.graph, batch, r.state, prm, stream=stream)
        except lib.LouvainError as ex:
            return ex.code
        finally:
            r.graph._ws = None
        with self.lock:
            self.ds_updates += 1
        return 0

    def grow(self, r: Resident, slack_frac: float, slack_min: int) -> None:
        """Lays a resident graph out again with more slack per row."""
        before = r.nbytes
        r.graph = r.graph.relayout(slack_frac=slack_frac, slack_min=slack_min)
        r.graph._ws = None  # the relayout workspace is not kept
        with self.lock:
            self.resident_bytes += r.nbytes - before

    def release(self, gids) -> None:
        now = time.perf_counter()
        for gid in gids:
            r = self.res[gid]
            r.busy = False
            r.last_used = now


class Server:
    """Continuous batching over a GraphStore (see the module docstring)."""

    def __init__(self, store: GraphStore, slots=1024, workers=2, **params):
        self.store = store
        self.slots = int(slots)
        self.workers = int(workers)
        self.params = lib.params(mode=store.mode, **params)
        self.queue = collections.deque()
        self.done = []
        self.cv = threading.Condition(store.lock)
        self.closed = False
        self.launches = 0
        self._next_rid = 0
        self._threads = []

    def submit(self, gid: int, batch, t_arrival=None) -> Request:
        with self.cv:
            r = Request(gid, batch, time.perf_counter() if t_arrival is None else t_arrival, self._next_rid)
            self._next_rid += 1
            self.queue.append(r)
            self.cv.notify()
        return r

    def start(self):
        for k in range(self.workers):
            t = threading.Thread(target=self._worker, args=(k,), daemon=True)
            t.start()
            self._threads.append(t)

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self._threads:
            t.join()

    def _take(self):
        """Up to `slots` waiting requests on distinct idle graphs, oldest
        first (a graph's requests stay in arrival order)."""
        picked, seen, keep = [], set(), collections.deque()
        while self.queue and len(picked) < self.slots:
            r = self.queue.popleft()
            res = self.store.res.get(r.gid)
            if r.gid in seen or r.gid in self.store.moving or (res is not None and res.busy):
                keep.append(r)
                seen.add(r.gid)
                continue
            seen.add(r.gid)
            picked.append(r)
        keep.extend(self.queue)
        self.queue.clear()
        self.queue.extend(keep)
        return picked

    def _worker(self, k):
        stream = torch.cuda.Stream(device=self.store.device)
        desc = torch.empty(int(lib.load().lv_many_desc_bytes(self.slots)), dtype=torch.uint8,
                           device=self.store.device)
        ws = None
        staging = None  # pinned host buffer of the batches' transfer
        while True:
            with self.cv:
                while not self.queue and not self.closed:
                    self.cv.wait()
                if not self.queue and self.closed:
                    return
                picked = self._take()
                if not picked:
                    self.cv.wait(0.001)
                    continue
                # bookkeeping only under the lock; the copies and builds of
                # the admission run outside it
                plan, victims = self.store._reserve([r.gid for r in picked])
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                residents = self.store._admit(plan, victims)
                need_i32 = sum(r.batch.size * 3 for r in picked)
                if staging is None or staging.numel() < need_i32:
                    staging = torch.empty(max(need_i32, 1 << 16) * 2, dtype=torch.int32, pin_memory=True)
                batches = lib.Batch.many_from_host([r.batch for r in picked], self.store.device, staging)
                big = max(residents, key=lambda x: x.graph.n * 4 + x.graph.cap)
                need = int(lib.load().lv_workspace_bytes(big.graph.n, big.graph.cap))
                if ws is None or ws.numel() < need:
                    ws = torch.empty(need, dtype=torch.uint8, device=self.store.device)
                fallback = self.store.ds_drop is not None
                dsj = [j for j, x in enumerate(residents) if fallback and x.use_ds]
                dfj = [j for j in range(len(picked)) if not (fallback and residents[j].use_ds)]
                status, src = [0] * len(picked), [()] * len(picked)
                approach = ["ds" if j in dsj else "df" for j in range(len(picked))]
                redo = dfj
                # the batched DF launch; a batch that does not fit its rows'
                # slack left the graph as it was: lay the graph out again with
                # more slack and rerun
                for attempt in range(4):
                    if not redo:
                        break
                    if attempt:
                        for j in redo:
                            self.store.grow(residents[j], 0.5 * 2 ** (attempt - 1), 16 << (attempt - 1))
                        big = max((residents[j] for j in redo), key=lambda x: x.graph.n * 4 + x.graph.cap)
                        need = int(lib.load().lv_workspace_bytes(big.graph.n, big.graph.cap))
                        if ws.numel() < need:
                            ws = torch.empty(need, dtype=torch.uint8, device=self.store.device)
                    st2, sts2 = lib.louvain_df_many([residents[j].graph for j in redo], [batches[j] for j in redo],
                                                    [residents[j].state for j in redo],
                                                    [residents[j].scratch for j in redo], self.store.max_updates,
                                                    prm=self.params, ws=ws, desc=desc, stream=stream)
                    for q, (j, a) in enumerate(zip(redo, st2)):
                        status[j], src[j] = a, (sts2, q)
                    redo = [j for j in redo if status[j] == lib.LV_ENOSLACK]
                # graphs under the DS fallback: apply_batch + DS Louvain each
                for j in dsj:
                    x = residents[j]
                    for attempt in range(4):
                        if attempt:
                            self.store.grow(x, 0.5 * 2 ** (attempt - 1), 16 << (attempt - 1))
                        need = int(lib.load().lv_workspace_bytes(x.graph.n, x.graph.cap))
                        if ws.numel() < need:
                            ws = torch.empty(need, dtype=torch.uint8, device=self.store.device)
                        status[j] = self.store.ds_update(x, batches[j], self.params, ws, stream)
                        if status[j] != lib.LV_ENOSLACK:
                            break
                quality = [float("nan")] * len(picked)
                if fallback:
                    for j, x in enumerate(residents):
                        if status[j] == 0:
                            quality[j] = self.store.measure(x, ws, stream)
                refreshed = [False] * len(picked)
                if self.store.refresh_every:
                    for j, (x, st) in enumerate(zip(residents, status)):
                        if st != 0:
                            continue
                        x.since_refresh += 1
                        if x.since_refresh >= self.store.refresh_every:
                            need = int(lib.load().lv_workspace_bytes(x.graph.n, x.graph.cap))
                            if ws.numel() < need:
                                ws = torch.empty(need, dtype=torch.uint8, device=self.store.device)
                            self.store.refresh(x, ws, stream)
                            refreshed[j] = True
            t1 = time.perf_counter()
            with self.cv:
                self.launches += 1
                for r, s, sr, rf, ap, q in zip(picked, status, src, refreshed, approach, quality):
                    r.t_start, r.t_done, r.status, r.src, r.refreshed = t0, t1, s, sr, rf
                    r.approach, r.modularity = ap, q
                    self.done.append(r)
                self.store.release([r.gid for r in picked])
                self.cv.notify_all()

    def wait(self, count: int, timeout: float = 600.0) -> None:
        """Blocks until `count` requests are done."""
        end = time.perf_counter() + timeout
        with self.cv:
            while len(self.done) < count:
                left = end - time.perf_counter()
                if left <= 0:
                    raise TimeoutError(f"{len(self.done)} of {count} requests done")
                self.cv.wait(left)

    def summary(self) -> dict:
        lat = np.array([r.t_done - r.t_arrival for r in self.done]) * 1e3
        if not len(lat):
            return {}
        t0 = min(r.t_arrival for r in self.done)
        t1 = max(r.t_done for r in self.done)
        return {"requests": len(self.done), "latency_ms_p50": float(np.percentile(lat, 50)),
                "latency_ms_p99": float(np.percentile(lat, 99)), "requests_per_s": len(self.done) / (t1 - t0),
                "launches": self.launches, "admissions": self.store.admissions,
                "evictions": self.store.evictions, "refreshes": self.store.refreshes,
                "ds_updates": self.store.ds_updates,
                "failed": sum(1 for r in self.done if r.status != 0)}
