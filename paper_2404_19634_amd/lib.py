"""Python binding of the HIP library (argument marshalling only).

Every operation runs in ``liblouvain_hip.so``; this module passes device
pointers of torch tensors and the current HIP stream through the C
interface declared in ``include/louvain.h``.  Importing it without the built
library raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
from collections.abc import Mapping
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblouvain_hip.so")

LV_OK = 0
STATUS = {0: "LV_OK", -1: "LV_EINVAL", -2: "LV_ENOEDGE", -3: "LV_ENOSLACK", -4: "LV_EOVERFLOW",
          -5: "LV_EEMPTY", -6: "LV_EHIP", -7: "LV_EWORKSPACE", -8: "LV_ETOOLARGE"}
LV_EINVAL, LV_ENOEDGE, LV_ENOSLACK, LV_EOVERFLOW, LV_EEMPTY, LV_EHIP, LV_EWORKSPACE = -1, -2, -3, -4, -5, -6, -7
LV_ETOOLARGE = -8
SYNC, ASYNC = 0, 1
MAX_PASSES, MAX_ITERS = 16, 32
# degree bins of the local-moving scan (LV_BIN_*) and the timing selector
BINS = ("g4", "g8", "g16", "g32", "wave", "block", "hub")
NBINS = len(BINS)
# kernels the timing hook can bracket (LV_TIME_*)
TIMED = ("scan", "binning", "hub_clear", "hub_decide")
TIME_SCAN, TIME_BINNING, TIME_HUB_CLEAR, TIME_HUB_DECIDE = range(4)
NTIMED = len(TIMED)

EXPORTS = ["lv_default_params", "lv_workspace_bytes", "lv_graph_capacity_bound", "lv_graph_build",
           "lv_graph_relayout", "apply_batch", "louvain_static", "louvain_nd", "louvain_ds", "louvain_df",
           "modularity", "louvain_df_apply", "lv_set_tuning", "lv_get_tuning", "lv_set_timing", "lv_last_error",
           "lv_many_scratch_bytes", "lv_many_desc_bytes", "louvain_df_many", "lv_autotune",
           "lv_noalloc_scratch_bytes", "louvain_df_noalloc", "lv_get_many_tuning", "lv_set_many_tuning",
           "lv_many_size_class", "lv_autotune_many", "lv_workspace_bytes_f", "lv_graph_build_f", "apply_batch_f",
           "louvain_static_f", "louvain_df_f", "modularity_f"]


class LouvainError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CGraph(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("cap", ct.c_int64), ("row_start", ct.c_void_p), ("row_len", ct.c_void_p),
                ("col", ct.c_void_p), ("w", ct.c_void_p), ("two_m", ct.c_void_p)]


class CEdges(ct.Structure):
    _fields_ = [("u", ct.c_void_p), ("v", ct.c_void_p), ("w", ct.c_void_p), ("count", ct.c_int64)]


class CState(ct.Structure):
    _fields_ = [("C", ct.c_void_p), ("K", ct.c_void_p), ("Sigma", ct.c_void_p), ("size", ct.c_void_p)]


class Params(ct.Structure):
    _fields_ = [("tolerance", ct.c_double), ("tolerance_drop", ct.c_double),
                ("aggregation_tolerance", ct.c_double), ("max_iterations", ct.c_int32),
                ("max_passes", ct.c_int32), ("mode", ct.c_int32), ("swap_guard", ct.c_int32),
                ("recompute_weights", ct.c_int32), ("reserved", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("passes", ct.c_int32), ("iterations", ct.c_int32 * MAX_PASSES),
                ("communities", ct.c_int64 * MAX_PASSES), ("moves", ct.c_int64), ("arcs_scanned", ct.c_int64),
                ("vertices_affected", ct.c_int64), ("iter_moves", (ct.c_int64 * MAX_ITERS) * MAX_PASSES),
                ("iter_gain", (ct.c_int64 * MAX_ITERS) * MAX_PASSES), ("seconds", ct.c_double),
                ("ms_mark", ct.c_float), ("ms_move", ct.c_float), ("ms_aggregate", ct.c_float),
                ("ms_other", ct.c_float), ("arcs_aggregated", ct.c_int64),
                ("bin_vertices", ct.c_int64 * NBINS), ("bin_arcs", ct.c_int64 * NBINS),
                ("bin_launches", ct.c_int32 * NBINS), ("timed_launches", ct.c_int32 * NTIMED),
                ("timed_ms", ct.c_double * NTIMED)]

    def as_dict(self) -> dict:
        p = self.passes
        its = [self.iterations[k] for k in range(p)]
        return {
            "passes": p, "iterations": its,
            "communities": [int(self.communities[k]) for k in range(p)],
            "moves": int(self.moves), "arcs_scanned": int(self.arcs_scanned),
            "vertices_affected": int(self.vertices_affected),
            "iter_moves": [[int(self.iter_moves[k][t]) for t in range(its[k])] for k in range(p)],
            "iter_gain": [[int(self.iter_gain[k][t]) for t in range(its[k])] for k in range(p)],
            "seconds": float(self.seconds), "ms_mark": float(self.ms_mark), "ms_move": float(self.ms_move),
            "ms_aggregate": float(self.ms_aggregate), "ms_other": float(self.ms_other),
            "arcs_aggregated": int(self.arcs_aggregated),
            "bin_vertices": [int(x) for x in self.bin_vertices], "bin_arcs": [int(x) for x in self.bin_arcs],
            "bin_launches": [int(x) for x in self.bin_launches],
            "timed_launches": [int(x) for x in self.timed_launches], "timed_ms": [float(x) for x in self.timed_ms],
        }


class CItem(ct.Structure):
    _fields_ = [("g", CGraph), ("state", CState), ("dels", CEdges), ("ins", CEdges), ("scratch", ct.c_void_p),
                ("max_updates", ct.c_int32)]


class Tuning(ct.Structure):
    _fields_ = [("wave_max_degree", ct.c_int32), ("blocks_small", ct.c_int32), ("blocks_wave", ct.c_int32),
                ("blocks_hub", ct.c_int32), ("async_rounds_log2", ct.c_int32),
                ("async_rounds_min_frontier", ct.c_int32), ("async_round_order", ct.c_int32),
                ("fuse_max_frontier", ct.c_int32), ("defer_totals", ct.c_int32),
                ("revisit_min_degree", ct.c_int32)]


_lib = None


def load():
    """Loads the library (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback")
    L = ct.CDLL(LIB_PATH, mode=ct.RTLD_GLOBAL)
    P, I32, I64, SZ = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
    GP, EP, SP, PP, STP = (ct.POINTER(CGraph), ct.POINTER(CEdges), ct.POINTER(CState), ct.POINTER(Params),
                           ct.POINTER(Stats))
    L.lv_default_params.argtypes = [PP]
    L.lv_workspace_bytes.restype = SZ
    L.lv_workspace_bytes.argtypes = [I32, I64]
    L.lv_graph_capacity_bound.restype = I64
    L.lv_graph_capacity_bound.argtypes = [I32, I64, ct.c_float, I32]
    L.lv_graph_build.restype = I32
    L.lv_graph_build.argtypes = [GP, EP, ct.c_float, I32, P, SZ, P]
    L.lv_graph_relayout.restype = I32
    L.lv_graph_relayout.argtypes = [GP, GP, ct.c_float, I32, P, SZ, P]
    L.apply_batch.restype = I32
    L.apply_batch.argtypes = [GP, EP, EP, P, SZ, P]
    L.louvain_static.restype = I32
    L.louvain_static.argtypes = [GP, PP, SP, P, SZ, STP, P]
    for name in ("louvain_nd", "louvain_ds", "louvain_df", "louvain_df_apply"):
        f = getattr(L, name)
        f.restype = I32
        f.argtypes = [GP, EP, EP, PP, SP, P, SZ, STP, P]
    L.modularity.restype = I32
    L.modularity.argtypes = [GP, P, ct.POINTER(ct.c_double), P, SZ, P]
    L.lv_set_tuning.argtypes = [ct.POINTER(Tuning)]
    L.lv_get_tuning.argtypes = [ct.POINTER(Tuning)]
    L.lv_many_scratch_bytes.restype = SZ
    L.lv_many_scratch_bytes.argtypes = [I32, I32]
    L.lv_many_desc_bytes.restype = SZ
    L.lv_many_desc_bytes.argtypes = [I32]
    L.louvain_df_many.restype = I32
    L.louvain_df_many.argtypes = [ct.POINTER(CItem), I32, PP, P, SZ, P, SZ, ct.POINTER(I32), STP, P]
    L.lv_get_many_tuning.argtypes = [I32, P]
    L.lv_set_many_tuning.argtypes = [I32, P]
    L.lv_many_size_class.restype = I32
    L.lv_many_size_class.argtypes = [P, I32]
    L.lv_autotune_many.restype = I32
    L.lv_autotune_many.argtypes = [ct.POINTER(CItem), I32, PP, P, SZ, P, SZ, ct.POINTER(I32), STP, P, P]
    L.lv_autotune.restype = I32
    L.lv_autotune.argtypes = [GP, SP, P, SZ, I32, ct.POINTER(Tuning), P]
    L.lv_noalloc_scratch_bytes.restype = SZ
    L.lv_noalloc_scratch_bytes.argtypes = []
    L.louvain_df_noalloc.restype = I32
    L.louvain_df_noalloc.argtypes = [GP, EP, EP, PP, SP, STP, P]
    L.lv_set_timing.restype = I32
    L.lv_set_timing.argtypes = [ct.c_uint32]
    L.lv_workspace_bytes_f.restype = SZ
    L.lv_workspace_bytes_f.argtypes = [I32, I64]
    L.lv_graph_build_f.restype = I32
    L.lv_graph_build_f.argtypes = [GP, EP, ct.c_float, I32, P, SZ, P]
    L.apply_batch_f.restype = I32
    L.apply_batch_f.argtypes = [GP, EP, EP, P, SZ, P]
    L.louvain_static_f.restype = I32
    L.louvain_static_f.argtypes = [GP, PP, SP, P, SZ, STP, P]
    L.louvain_df_f.restype = I32
    L.louvain_df_f.argtypes = [GP, EP, EP, PP, SP, P, SZ, STP, P]
    L.modularity_f.restype = I32
    L.modularity_f.argtypes = [GP, P, ct.POINTER(ct.c_double), P, SZ, P]
    L.lv_last_error.restype = ct.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != LV_OK:
        raise LouvainError(code, load().lv_last_error().decode())


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream=None):
    """The HIP stream handle of `stream`, else of the current stream (read
    without building a Stream object when torch offers that)."""
    if stream is not None:
        return ct.c_void_p(stream.cuda_stream)
    if _raw_stream is not None:
        return ct.c_void_p(_raw_stream(torch.cuda.current_device()))
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ct.c_void_p(t.data_ptr())


def params(tolerance=1e-2, tolerance_drop=10.0, aggregation_tolerance=0.8, max_iterations=20, max_passes=10,
           mode="async", swap_guard=1, recompute_weights=0) -> Params:
    """Defaults are the paper's (Section 5.1.2).  recompute_weights=1: the
    dynamic calls recompute K and Sigma from scratch (Section 4.2's variant
    without auxiliary information)."""
    m = {"sync": SYNC, "async": ASYNC}[mode] if isinstance(mode, str) else int(mode)
    return Params(float(tolerance), float(tolerance_drop), float(aggregation_tolerance), int(max_iterations),
                  int(max_passes), m, int(swap_guard), int(recompute_weights), 0)


DEFAULT_ASYNC_ROUNDS_LOG2 = 7


DEFAULT_FUSE_MAX_FRONTIER = 1 << 20
DEFAULT_ASYNC_ROUNDS_MIN_FRONTIER = 256
DEFAULT_REVISIT_MIN_DEGREE = 128


def set_timing(kernels=()):
    """Time every launch of the given kernels (indices into TIMED) with HIP
    events stamped by the launch itself; the louvain_* calls then report
    timed_launches and timed_ms per kernel.  () turns timing off."""
    mask = 0
    for k in kernels:
        mask |= 1 << int(k)
    _check(load().lv_set_timing(mask))


def set_tuning(wave_max_degree=0, blocks_small=0, blocks_wave=0, blocks_hub=0,
               async_rounds_log2=DEFAULT_ASYNC_ROUNDS_LOG2,
               async_rounds_min_frontier=DEFAULT_ASYNC_ROUNDS_MIN_FRONTIER, async_round_order=2,
               fuse_max_frontier=DEFAULT_FUSE_MAX_FRONTIER, defer_totals=1,
               revisit_min_degree=DEFAULT_REVISIT_MIN_DEGREE):
    load().lv_set_tuning(ct.byref(Tuning(wave_max_degree, blocks_small, blocks_wave, blocks_hub,
                                         async_rounds_log2, async_rounds_min_frontier, async_round_order,
                                         fuse_max_frontier, defer_totals, revisit_min_degree)))


def autotune(g: "Graph", repeats: int = 2, stream=None) -> dict:
    """Picks the wavefront / workgroup degree threshold for graph g by
    timing full SYNC sweeps (lv_autotune); the choice becomes the
    process-wide tuning.  Returns the tuning now in force."""
    L = load()
    st = State.empty(g.n, g.device, with_size=False)
    cs, cg = st.c(), g.c()
    ws, nb = g.ws_args()
    out = Tuning()
    _check(L.lv_autotune(ct.byref(cg), ct.byref(cs), ws, nb, int(repeats), ct.byref(out), _stream(stream)))
    return {f: getattr(out, f) for f, _ in Tuning._fields_}


def get_tuning() -> dict:
    t = Tuning()
    load().lv_get_tuning(ct.byref(t))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def _dev_i32(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.int32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.int32))).to(device)


class Edges:
    """Undirected edge or update list on the device (each pair once)."""

    def __init__(self, u, v, w, device="cuda"):
        self.u = _dev_i32(u, device)
        self.v = _dev_i32(v, device)
        self.w = _dev_i32(w, device)

    @property
    def count(self) -> int:
        return int(self.u.shape[0])

    def c(self) -> CEdges:
        return CEdges(*self.cvals())

    def cvals(self) -> tuple:
        """The lv_edges fields in order (null pointers as 0)."""
        n = self.count
        if n == 0:
            return 0, 0, 0, 0
        return self.u.data_ptr(), self.v.data_ptr(), self.w.data_ptr(), n


@dataclass
class Batch:
    dels: Edges
    ins: Edges

    @classmethod
    def from_host(cls, b, device="cuda"):
        return cls(Edges(b.del_u, b.del_v, b.del_w, device), Edges(b.ins_u, b.ins_v, b.ins_w, device))

    @classmethod
    def empty(cls, device="cuda"):
        z = np.zeros(0, np.int32)
        return cls(Edges(z, z, z, device), Edges(z, z, z, device))

    @classmethod
    def many_from_host(cls, batches, device="cuda", staging: Optional[torch.Tensor] = None):
        """Device copies of many host batches through one transfer: every
        array lands in one device buffer and each batch refers to its part
        by address.  `staging`, a pinned int32 host tensor, is reused for
        the transfer when large enough (the caller must not refill it
        before the copy has completed, e.g. before the stream's next
        synchronisation)."""
        parts = []
        for b in batches:
            parts += [b.del_u, b.del_v, b.del_w, b.ins_u, b.ins_v, b.ins_w]
        sizes = np.array([len(x) for x in parts], dtype=np.int64)
        total = int(sizes.sum())
        if staging is None or staging.numel() < total:
            staging = torch.empty(max(total, 1), dtype=torch.int32, pin_memory=True)
        host = staging.numpy()[:total]
        if parts:
            np.concatenate([np.asarray(x, np.int32) for x in parts], out=host)
        dev = torch.empty(max(total, 1), dtype=torch.int32, device=device)
        dev[:total].copy_(staging[:total], non_blocking=True)
        a = (dev.data_ptr() + 4 * (np.cumsum(sizes) - sizes)).tolist()
        n = sizes.tolist()
        E = _EdgesAt
        return [cls(E(dev, a[k], a[k + 1], a[k + 2], n[k]), E(dev, a[k + 3], a[k + 4], a[k + 5], n[k + 3]))
                for k in range(0, 6 * len(batches), 6)]


class _EdgesAt:
    """An update list inside a shared device buffer (addresses only; the
    buffer is kept alive by reference)."""
    __slots__ = ("buf", "pu", "pv", "pw", "count")

    def __init__(self, buf, pu, pv, pw, count):
        self.buf, self.pu, self.pv, self.pw, self.count = buf, pu, pv, pw, count

    def c(self) -> CEdges:
        return CEdges(*self.cvals())

    def cvals(self) -> tuple:
        if self.count == 0:
            return 0, 0, 0, 0
        return self.pu, self.pv, self.pw, self.count


class Graph:
    """Slack-padded CSR on the device plus its workspace."""

    def __init__(self, n: int, cap: int, device="cuda"):
        self.device = torch.device(device)
        self.n = int(n)
        self.cap = int(cap)
        self.row_start = torch.zeros(self.n + 1, dtype=torch.int64, device=self.device)
        self.row_len = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.col = torch.zeros(max(self.cap, 1), dtype=torch.int32, device=self.device)
        self.w = torch.zeros(max(self.cap, 1), dtype=torch.int32, device=self.device)
        self.two_m_t = torch.zeros(1, dtype=torch.int64, device=self.device)
        self._ws = None

    def c(self) -> CGraph:
        return CGraph(*self.cvals())

    def cvals(self) -> tuple:
        """The lv_graph fields in order (kept while the arrays are the same
        objects: a batched call marshals thousands of graphs)."""
        key = (self.n, self.cap, id(self.row_start), id(self.row_len), id(self.col), id(self.w), id(self.two_m_t))
        c = self.__dict__.get("_cv")
        if c is None or c[0] != key:
            c = (key, (self.n, self.cap, self.row_start.data_ptr(), self.row_len.data_ptr(), self.col.data_ptr(),
                       self.w.data_ptr(), self.two_m_t.data_ptr()))
            self.__dict__["_cv"] = c
        return c[1]

    @property
    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            nbytes = int(load().lv_workspace_bytes(self.n, self.cap))
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def ws_args(self):
        ws = self.workspace
        return ct.c_void_p(ws.data_ptr()), ws.numel()

    @property
    def two_m(self) -> int:
        return int(self.two_m_t.item())

    @classmethod
    def build(cls, n, u, v, w, slack_frac=0.1, slack_min=4, device="cuda", stream=None) -> "Graph":
        L = load()
        e = Edges(u, v, w, device)
        cap = int(L.lv_graph_capacity_bound(int(n), e.count, float(slack_frac), int(slack_min)))
        g = cls(n, cap, device)
        ce = e.c()
        cg = g.c()
        ws, nb = g.ws_args()
        _check(L.lv_graph_build(ct.byref(cg), ct.byref(ce), float(slack_frac), int(slack_min), ws, nb,
                                _stream(stream)))
        return g

    @classmethod
    def from_edges(cls, e, **kw) -> "Graph":
        return cls.build(e.n, e.u, e.v, e.w, **kw)

    def relayout(self, slack_frac=0.5, slack_min=8, stream=None) -> "Graph":
        """A copy of this graph with more free capacity per row."""
        L = load()
        arcs = int(self.row_len.sum().item())
        cap = int(L.lv_graph_capacity_bound(self.n, (arcs + 1) // 2, float(slack_frac), int(slack_min)))
        g = Graph(self.n, cap, self.device)
        src, dst = self.c(), g.c()
        ws, nb = g.ws_args()
        _check(L.lv_graph_relayout(ct.byref(src), ct.byref(dst), float(slack_frac), int(slack_min), ws, nb,
                                   _stream(stream)))
        return g

    def csr_host(self):
        """(offsets, col, w) on the host with every row sorted by neighbour."""
        rs = self.row_start.cpu().numpy()
        rl = self.row_len.cpu().numpy().astype(np.int64)
        col = self.col.cpu().numpy()
        w = self.w.cpu().numpy()
        off = np.zeros(self.n + 1, dtype=np.int64)
        off[1:] = np.cumsum(rl)
        idx = np.concatenate([np.arange(rs[i], rs[i] + rl[i]) for i in range(self.n)]) if self.n else np.zeros(0, np.int64)
        idx = idx.astype(np.int64)
        rows = np.repeat(np.arange(self.n), rl)
        c2, w2 = col[idx], w[idx].astype(np.int64)
        order = np.lexsort((c2, rows))
        return off, c2[order], w2[order]


@dataclass
class State:
    """C, K, Sigma on the device, plus the optional member count per
    community (`size`).  A state returned by louvain_static carries `size`,
    and the dynamic calls keep it exact; a state built from host arrays has
    none, and the library then counts member sizes itself on every call."""
    C: torch.Tensor
    K: torch.Tensor
    Sigma: torch.Tensor
    size: Optional[torch.Tensor] = None

    @classmethod
    def empty(cls, n, device="cuda", with_size=True):
        """Output buffers for louvain_static (which fills all four)."""
        return cls(torch.zeros(n, dtype=torch.int32, device=device), torch.zeros(n, dtype=torch.int64, device=device),
                   torch.zeros(n, dtype=torch.int64, device=device),
                   torch.zeros(n, dtype=torch.int32, device=device) if with_size else None)

    @classmethod
    def from_host(cls, C, K, S, device="cuda"):
        return cls(torch.from_numpy(np.asarray(C, np.int32).copy()).to(device),
                   torch.from_numpy(np.asarray(K, np.int64).copy()).to(device),
                   torch.from_numpy(np.asarray(S, np.int64).copy()).to(device))

    def clone(self) -> "State":
        return State(self.C.clone(), self.K.clone(), self.Sigma.clone(),
                     None if self.size is None else self.size.clone())

    def host(self):
        return self.C.cpu().numpy(), self.K.cpu().numpy(), self.Sigma.cpu().numpy()

    def c(self) -> CState:
        return CState(*self.cvals())

    def cvals(self) -> tuple:
        """The lv_state fields in order (no member counts: 0); kept while
        the arrays are the same objects."""
        key = (id(self.C), id(self.K), id(self.Sigma), id(self.size))
        c = self.__dict__.get("_cv")
        if c is None or c[0] != key:
            c = (key, (self.C.data_ptr(), self.K.data_ptr(), self.Sigma.data_ptr(),
                       0 if self.size is None else self.size.data_ptr()))
            self.__dict__["_cv"] = c
        return c[1]


def apply_batch(g: Graph, b: Batch, stream=None):
    L = load()
    cg, cd, ci = g.c(), b.dels.c(), b.ins.c()
    ws, nb = g.ws_args()
    _check(L.apply_batch(ct.byref(cg), ct.byref(cd), ct.byref(ci), ws, nb, _stream(stream)))


def louvain_static(g: Graph, prm: Params = None, state: State = None, stream=None, **kw):
    L = load()
    prm = prm if prm is not None else params(**kw)
    state = state if state is not None else State.empty(g.n, g.device)
    st = Stats()
    cg, cs = g.c(), state.c()
    ws, nb = g.ws_args()
    _check(L.louvain_static(ct.byref(cg), ct.byref(prm), ct.byref(cs), ws, nb, ct.byref(st), _stream(stream)))
    return state, StatsView(st)


def _dynamic(fn, g, b, state, prm, stream, kw):
    L = load()
    prm = prm if prm is not None else params(**kw)
    st = Stats()
    cg, cd, ci, cs = g.c(), b.dels.c(), b.ins.c(), state.c()
    ws, nb = g.ws_args()
    _check(getattr(L, fn)(ct.byref(cg), ct.byref(cd), ct.byref(ci), ct.byref(prm), ct.byref(cs), ws, nb,
                          ct.byref(st), _stream(stream)))
    return state, StatsView(st)


def louvain_nd(g, b, state, prm=None, stream=None, **kw):
    return _dynamic("louvain_nd", g, b, state, prm, stream, kw)


def louvain_ds(g, b, state, prm=None, stream=None, **kw):
    return _dynamic("louvain_ds", g, b, state, prm, stream, kw)


def louvain_df(g, b, state, prm=None, stream=None, **kw):
    return _dynamic("louvain_df", g, b, state, prm, stream, kw)


def louvain_df_apply(g, b, state, prm=None, stream=None, **kw):
    """apply_batch(g, b) and louvain_df(g, b, state) in one call (one host
    wait).  On LV_EINVAL / LV_ENOEDGE / LV_ENOSLACK / LV_EOVERFLOW the
    batch was refused and graph and state are unchanged."""
    return _dynamic("louvain_df_apply", g, b, state, prm, stream, kw)


def louvain_df_noalloc(g, b, state, prm=None, stream=None, **kw):
    """louvain_df through the entry point that allocates nothing: its
    scratch is the library's own device array (lv_noalloc_scratch_bytes()),
    so the graph's workspace is neither used nor created."""
    L = load()
    prm = prm if prm is not None else params(**kw)
    st = Stats()
    cg, cd, ci, cs = g.c(), b.dels.c(), b.ins.c(), state.c()
    _check(L.louvain_df_noalloc(ct.byref(cg), ct.byref(cd), ct.byref(ci), ct.byref(prm), ct.byref(cs),
                                ct.byref(st), _stream(stream)))
    return state, StatsView(st)


def many_scratch(n: int, max_updates: int, device="cuda") -> torch.Tensor:
    """Zeroed scratch for one graph of louvain_df_many (kept per graph; each
    call leaves it ready for the next)."""
    nbytes = int(load().lv_many_scratch_bytes(int(n), int(max_updates)))
    return torch.zeros(nbytes, dtype=torch.uint8, device=device)


def louvain_df_many(graphs, batches, states, scratches, max_updates, prm=None, ws=None, desc=None, stream=None,
                    **kw):
    """apply_batch + louvain_df on every (graph, batch, state) in one
    persistent launch.  `max_updates` is the capacity each scratch was sized
    for (an int, or one per graph); `ws` is a workspace tensor for graphs
    that continue on the single-graph path (None: they report
    LV_EWORKSPACE).  Returns (status list, stats list)."""
    return _many("louvain_df_many", graphs, batches, states, scratches, max_updates, prm, ws, desc, stream, kw)


def autotune_many(graphs, batches, states, scratches, max_updates, prm=None, ws=None, desc=None, stream=None,
                  **kw):
    """louvain_df_many that also tunes the batched launch for the items'
    size class (lv_autotune_many).  Returns (status list, stats list,
    the chosen tuning as a dict)."""
    best = ManyTuning()
    status, stats = _many("lv_autotune_many", graphs, batches, states, scratches, max_updates, prm, ws, desc,
                          stream, kw, best)
    return status, stats, {f: getattr(best, f) for f, _ in ManyTuning._fields_}


class ManyTuning(ct.Structure):
    _fields_ = [("wave_max_degree", ct.c_int32), ("grid", ct.c_int32)]


MANY_CLASSES = 12


def get_many_tuning() -> list:
    """The batched launch's tuning table, one dict per size class."""
    L = load()
    out = []
    for k in range(MANY_CLASSES):
        t = ManyTuning()
        L.lv_get_many_tuning(k, ct.byref(t))
        out.append({f: getattr(t, f) for f, _ in ManyTuning._fields_})
    return out


def set_many_tuning(table) -> None:
    """Restores a table from get_many_tuning (e.g. one saved to a file)."""
    L = load()
    for k, row in enumerate(table[:MANY_CLASSES]):
        L.lv_set_many_tuning(k, ct.byref(ManyTuning(int(row["wave_max_degree"]), int(row["grid"]))))


def many_size_class(graphs) -> int:
    """The size class of a batched call on these graphs."""
    items = (CItem * max(len(graphs), 1))()
    for k, g in enumerate(graphs):
        items[k].g.n = g.n
    return int(load().lv_many_size_class(items, len(graphs)))


def _many(fn, graphs, batches, states, scratches, max_updates, prm, ws, desc, stream, kw, best=None):
    L = load()
    count = len(graphs)
    prm = prm if prm is not None else params(**kw)
    caps = list(max_updates) if hasattr(max_updates, "__len__") else [int(max_updates)] * count
    items = np.zeros(max(count, 1), dtype=_item_dtype())
    if count:
        # one record per item, fields in lv_item order
        items[:count] = [g.cvals() + s.cvals() + b.dels.cvals() + b.ins.cvals() + (x.data_ptr(), cap)
                         for g, s, b, x, cap in zip(graphs, states, batches, scratches, caps)]
    need = int(L.lv_many_desc_bytes(count))
    if desc is None or desc.numel() < need:
        desc = torch.empty(need, dtype=torch.uint8, device=graphs[0].device if count else "cuda")
    status = np.zeros(max(count, 1), dtype=np.int32)
    # uninitialised records (the call writes every one it returns): a
    # zero-filled ctypes array of 8.6 KB per item costs more than the launch
    stats = np.empty(max(count, 1) * ct.sizeof(Stats), dtype=np.uint8)
    wp, wb = (ct.c_void_p(ws.data_ptr()), ws.numel()) if ws is not None else (None, 0)
    args = [items.ctypes.data_as(ct.POINTER(CItem)), count, ct.byref(prm), ct.c_void_p(desc.data_ptr()),
            desc.numel(), wp, wb, status.ctypes.data_as(ct.POINTER(ct.c_int32)),
            stats.ctypes.data_as(ct.POINTER(Stats))]
    if best is not None:
        args.append(ct.byref(best))
    _check(getattr(L, fn)(*args, _stream(stream)))
    return status[:count].tolist(), StatsList(stats, count)


class StatsView(Mapping):
    """One call's lv_stats as a read-only mapping, converted on first read
    (the conversion is not part of the call)."""

    def __init__(self, st: Stats):
        self._st, self._d = st, None

    def _dict(self) -> dict:
        if self._d is None:
            self._d = self._st.as_dict()
        return self._d

    def __getitem__(self, k):
        return self._dict()[k]

    def __iter__(self):
        return iter(self._dict())

    def __len__(self):
        return len(self._dict())

    def __repr__(self):
        return repr(self._dict())


class StatsList:
    """Per-item statistics of louvain_df_many (records in a byte array),
    converted to dicts when read."""

    def __init__(self, arr, count):
        self._a, self._n, self._d = arr, count, {}

    def __len__(self):
        return self._n

    def __getitem__(self, k):
        if isinstance(k, slice):
            return [self[j] for j in range(*k.indices(self._n))]
        if k < 0:
            k += self._n
        if not 0 <= k < self._n:
            raise IndexError(k)
        if k not in self._d:
            self._d[k] = StatsView(Stats.from_buffer(self._a, k * ct.sizeof(Stats)))
        return self._d[k]

    def __iter__(self):
        return (self[k] for k in range(self._n))


_ITEM_DTYPE = None


def _item_dtype() -> np.dtype:
    """numpy layout of lv_item (field offsets taken from the ctypes
    declaration, so the two cannot drift apart)."""
    global _ITEM_DTYPE
    if _ITEM_DTYPE is None:
        kinds = {ct.c_int32: np.int32, ct.c_int64: np.int64, ct.c_void_p: np.uint64}
        names, fmts, offs = [], [], []

        def walk(t, base, prefix):
            for f, ft in t._fields_:
                off = base + getattr(t, f).offset
                if isinstance(ft, type) and issubclass(ft, ct.Structure):
                    walk(ft, off, prefix + f + ".")
                else:
                    names.append(prefix + f)
                    fmts.append(kinds[ft])
                    offs.append(off)

        walk(CItem, 0, "")
        _ITEM_DTYPE = np.dtype({"names": names, "formats": fmts, "offsets": offs, "itemsize": ct.sizeof(CItem)})
    return _ITEM_DTYPE


def modularity(g: Graph, C: torch.Tensor, stream=None) -> float:
    L = load()
    q = ct.c_double(0.0)
    cg = g.c()
    ws, nb = g.ws_args()
    _check(L.modularity(ct.byref(cg), _ptr(C), ct.byref(q), ws, nb, _stream(stream)))
    return float(q.value)


RUN = {"static": None, "nd": louvain_nd, "ds": louvain_ds, "df": louvain_df}


# ---------------------------------------------------------------------------
# Paper precision (float32 edge weights, FP64 sums; Section 5.1.2).  The C
# structs have the integer ones' layout, so CGraph / CEdges / CState carry
# the pointers; only the element types differ.
# ---------------------------------------------------------------------------
class EdgesF(Edges):
    """Undirected edge or update list with float32 weights on the device."""

    def __init__(self, u, v, w, device="cuda"):
        self.u = _dev_i32(u, device)
        self.v = _dev_i32(v, device)
        if isinstance(w, torch.Tensor):
            self.w = w.to(device=device, dtype=torch.float32).contiguous()
        else:
            self.w = torch.from_numpy(np.ascontiguousarray(np.asarray(w, dtype=np.float32))).to(device)


@dataclass
class BatchF:
    dels: EdgesF
    ins: EdgesF

    @classmethod
    def from_host(cls, b, device="cuda"):
        return cls(EdgesF(b.del_u, b.del_v, b.del_w, device), EdgesF(b.ins_u, b.ins_v, b.ins_w, device))


class GraphF(Graph):
    """Slack-padded CSR with float32 weights and an FP64 total."""

    def __init__(self, n: int, cap: int, device="cuda"):
        self.device = torch.device(device)
        self.n = int(n)
        self.cap = int(cap)
        self.row_start = torch.zeros(self.n + 1, dtype=torch.int64, device=self.device)
        self.row_len = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.col = torch.zeros(max(self.cap, 1), dtype=torch.int32, device=self.device)
        self.w = torch.zeros(max(self.cap, 1), dtype=torch.float32, device=self.device)
        self.two_m_t = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._ws = None

    @property
    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            nbytes = int(load().lv_workspace_bytes_f(self.n, self.cap))
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    @property
    def two_m(self) -> float:
        return float(self.two_m_t.item())

    @classmethod
    def build(cls, n, u, v, w, slack_frac=0.1, slack_min=4, device="cuda", stream=None) -> "GraphF":
        L = load()
        e = EdgesF(u, v, w, device)
        cap = int(L.lv_graph_capacity_bound(int(n), e.count, float(slack_frac), int(slack_min)))
        g = cls(n, cap, device)
        ce, cg = e.c(), g.c()
        ws, nb = g.ws_args()
        _check(L.lv_graph_build_f(ct.byref(cg), ct.byref(ce), float(slack_frac), int(slack_min), ws, nb,
                                  _stream(stream)))
        return g

    def relayout(self, *a, **kw):
        raise NotImplementedError("relayout is offered for the integer graph only")

    def csr_host(self):
        """(offsets, col, w) on the host with every row sorted by neighbour."""
        rs = self.row_start.cpu().numpy()
        rl = self.row_len.cpu().numpy().astype(np.int64)
        col, w = self.col.cpu().numpy(), self.w.cpu().numpy()
        off = np.zeros(self.n + 1, dtype=np.int64)
        off[1:] = np.cumsum(rl)
        idx = (np.concatenate([np.arange(rs[i], rs[i] + rl[i]) for i in range(self.n)]) if self.n
               else np.zeros(0, np.int64)).astype(np.int64)
        rows = np.repeat(np.arange(self.n), rl)
        c2, w2 = col[idx], w[idx]
        order = np.lexsort((c2, rows))
        return off, c2[order], w2[order]


@dataclass
class StateF(State):
    """C (int32), K and Sigma (FP64), optional member counts."""

    @classmethod
    def empty(cls, n, device="cuda", with_size=True):
        return cls(torch.zeros(n, dtype=torch.int32, device=device),
                   torch.zeros(n, dtype=torch.float64, device=device),
                   torch.zeros(n, dtype=torch.float64, device=device),
                   torch.zeros(n, dtype=torch.int32, device=device) if with_size else None)

    @classmethod
    def from_host(cls, C, K, S, device="cuda"):
        return cls(torch.from_numpy(np.asarray(C, np.int32).copy()).to(device),
                   torch.from_numpy(np.asarray(K, np.float64).copy()).to(device),
                   torch.from_numpy(np.asarray(S, np.float64).copy()).to(device))

    def clone(self) -> "StateF":
        return StateF(self.C.clone(), self.K.clone(), self.Sigma.clone(),
                      None if self.size is None else self.size.clone())


def apply_batch_f(g: GraphF, b: BatchF, stream=None):
    L = load()
    cg, cd, ci = g.c(), b.dels.c(), b.ins.c()
    ws, nb = g.ws_args()
    _check(L.apply_batch_f(ct.byref(cg), ct.byref(cd), ct.byref(ci), ws, nb, _stream(stream)))


def louvain_static_f(g: GraphF, prm: Params = None, state: StateF = None, stream=None, **kw):
    L = load()
    prm = prm if prm is not None else params(**kw)
    state = state if state is not None else StateF.empty(g.n, g.device)
    st = Stats()
    cg, cs = g.c(), state.c()
    ws, nb = g.ws_args()
    _check(L.louvain_static_f(ct.byref(cg), ct.byref(prm), ct.byref(cs), ws, nb, ct.byref(st), _stream(stream)))
    return state, StatsView(st)


def louvain_df_f(g: GraphF, b: BatchF, state: StateF, prm: Params = None, stream=None, **kw):
    return _dynamic("louvain_df_f", g, b, state, prm, stream, kw)


def modularity_f(g: GraphF, C: torch.Tensor, stream=None) -> float:
    L = load()
    q = ct.c_double(0.0)
    cg = g.c()
    ws, nb = g.ws_args()
    _check(L.modularity_f(ct.byref(cg), _ptr(C), ct.byref(q), ws, nb, _stream(stream)))
    return float(q.value)
