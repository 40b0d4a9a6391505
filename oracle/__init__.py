"""Sequential CPU oracle for the DF Louvain hot path (test infrastructure).

Only the test suite, the package smoke check and the benchmark's CPU
baseline use this package.  The product library never imports it, and it
imports nothing from the product: the two share only the seeded workload
generators, which hold none of the method's arithmetic.

The arithmetic lives in ``louvain_oracle.cpp`` (plain sequential C++,
compiled by :func:`build`); this module is argument marshalling over
ctypes, with numpy arrays on the host.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "louvain_oracle.cpp")
SRC_FP = os.path.join(HERE, "louvain_oracle_fp.cpp")  # the paper's precision: float32 weights, FP64 sums
LIB = os.path.join(HERE, "liboracle.so")

STATIC, ND, DS, DF = 0, 1, 2, 3
SYNC, ASYNC = 0, 1
APPROACH = {"static": STATIC, "nd": ND, "ds": DS, "df": DF}
MODE = {"sync": SYNC, "async": ASYNC}

OK, E_INVAL, E_NOEDGE, E_OVERFLOW, E_EMPTY = 0, -1, -2, -4, -5

MAX_PASSES = 16
MAX_ITERS = 32


def build(force: bool = True) -> str:
    """Compile the oracle into ``liboracle.so`` with the host compiler."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                         os.path.getmtime(SRC_FP)):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, SRC, SRC_FP])
        os.replace(tmp, LIB)
    return LIB


class Params(ct.Structure):
    _fields_ = [
        ("tolerance", ct.c_double),
        ("tolerance_drop", ct.c_double),
        ("aggregation_tolerance", ct.c_double),
        ("max_iterations", ct.c_int32),
        ("max_passes", ct.c_int32),
        ("mode", ct.c_int32),
        ("swap_guard", ct.c_int32),
    ]


class Stats(ct.Structure):
    _fields_ = [
        ("passes", ct.c_int32),
        ("iterations", ct.c_int32 * MAX_PASSES),
        ("communities", ct.c_int64 * MAX_PASSES),
        ("moves", ct.c_int64),
        ("arcs_scanned", ct.c_int64),
        ("vertices_affected", ct.c_int64),
        ("iter_moves", (ct.c_int64 * MAX_ITERS) * MAX_PASSES),
        ("iter_gain", (ct.c_int64 * MAX_ITERS) * MAX_PASSES),
        ("seconds", ct.c_double),
    ]

    def as_dict(self) -> dict:
        p = self.passes
        its = [self.iterations[k] for k in range(p)]
        return {
            "passes": p,
            "iterations": its,
            "communities": [int(self.communities[k]) for k in range(p)],
            "moves": int(self.moves),
            "arcs_scanned": int(self.arcs_scanned),
            "vertices_affected": int(self.vertices_affected),
            "iter_moves": [[int(self.iter_moves[k][t]) for t in range(its[k])] for k in range(p)],
            "iter_gain": [[int(self.iter_gain[k][t]) for t in range(its[k])] for k in range(p)],
            "seconds": float(self.seconds),
        }


class StatsF(ct.Structure):
    """Statistics of the paper-precision oracle (ΔQ sums in FP64)."""
    _fields_ = [
        ("passes", ct.c_int32),
        ("iterations", ct.c_int32 * MAX_PASSES),
        ("communities", ct.c_int64 * MAX_PASSES),
        ("moves", ct.c_int64),
        ("arcs_scanned", ct.c_int64),
        ("iter_moves", (ct.c_int64 * MAX_ITERS) * MAX_PASSES),
        ("iter_dq", (ct.c_double * MAX_ITERS) * MAX_PASSES),
        ("seconds", ct.c_double),
    ]

    def as_dict(self) -> dict:
        p = self.passes
        its = [self.iterations[k] for k in range(p)]
        return {"passes": p, "iterations": its, "communities": [int(self.communities[k]) for k in range(p)],
                "moves": int(self.moves), "arcs_scanned": int(self.arcs_scanned),
                "iter_moves": [[int(self.iter_moves[k][t]) for t in range(its[k])] for k in range(p)],
                "iter_dq": [[float(self.iter_dq[k][t]) for t in range(its[k])] for k in range(p)],
                "seconds": float(self.seconds)}


def params(tolerance=1e-2, tolerance_drop=10.0, aggregation_tolerance=0.8,
           max_iterations=20, max_passes=10, mode="sync", swap_guard=1) -> Params:
    """Defaults are the paper's (Section 5.1.2)."""
    return Params(float(tolerance), float(tolerance_drop), float(aggregation_tolerance),
                  int(max_iterations), int(max_passes), MODE[mode] if isinstance(mode, str) else int(mode),
                  int(swap_guard))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(SRC_FP)):
            build(force=True)
        L = ct.CDLL(LIB)
        P = ct.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.orc_graph_new.restype = P
        L.orc_graph_new.argtypes = [ct.c_int32, ct.c_int64, i32p, i32p, i32p, ct.POINTER(ct.c_int32)]
        L.orc_graph_free.argtypes = [P]
        L.orc_graph_n.restype = ct.c_int32
        L.orc_graph_n.argtypes = [P]
        L.orc_two_m.restype = ct.c_int64
        L.orc_two_m.argtypes = [P]
        L.orc_arc_count.restype = ct.c_int64
        L.orc_arc_count.argtypes = [P]
        L.orc_export.argtypes = [P, i64p, i32p, i64p]
        L.orc_apply_batch.restype = ct.c_int32
        L.orc_apply_batch.argtypes = [P, ct.c_int64, i32p, i32p, i32p, ct.c_int64, i32p, i32p, i32p]
        L.orc_weighted_degrees.argtypes = [P, i64p]
        L.orc_modularity.restype = ct.c_double
        L.orc_modularity.argtypes = [P, i32p]
        L.orc_mark.restype = ct.c_int32
        L.orc_mark.argtypes = [P, ct.c_int32, ct.c_int64, i32p, i32p, i32p, ct.c_int64, i32p, i32p,
                               i32p, i32p, i64p, i64p, u8p, u8p]
        L.orc_update_weights.argtypes = [ct.c_int32, ct.c_int64, i32p, i32p, i32p, ct.c_int64, i32p,
                                         i32p, i32p, i32p, i64p, i64p]
        L.orc_louvain.restype = ct.c_int32
        L.orc_louvain.argtypes = [P, ct.c_int32, ct.POINTER(Params), ct.c_int64, i32p, i32p, i32p,
                                  ct.c_int64, i32p, i32p, i32p, i32p, i64p, i64p, ct.POINTER(Stats)]
        L.orc_decide.restype = ct.c_int32
        L.orc_decide.argtypes = [P, i32p, i64p, i64p, i32p, ct.c_int32, ct.c_int64, i32p, i32p, i64p, u8p]
        L.orc_aggregate.restype = P
        L.orc_aggregate.argtypes = [P, i32p, ct.c_int32]
        L.orc_graph_from_arcs.restype = P
        L.orc_graph_from_arcs.argtypes = [ct.c_int32, ct.c_int64, i32p, i32p, i64p]
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.orcf_graph_new.restype = P
        L.orcf_graph_new.argtypes = [ct.c_int32, ct.c_int64, i32p, i32p, f32p, ct.POINTER(ct.c_int32)]
        L.orcf_graph_free.argtypes = [P]
        L.orcf_two_m.restype = ct.c_double
        L.orcf_two_m.argtypes = [P]
        L.orcf_apply_batch.restype = ct.c_int32
        L.orcf_apply_batch.argtypes = [P, ct.c_int64, i32p, i32p, f32p, ct.c_int64, i32p, i32p, f32p]
        L.orcf_degrees.argtypes = [P, f64p]
        L.orcf_modularity.restype = ct.c_double
        L.orcf_modularity.argtypes = [P, i32p]
        L.orcf_decide.argtypes = [P, i32p, f64p, f64p, i32p, ct.c_int32, ct.c_int64, i32p, i32p, f64p, u8p]
        L.orcf_louvain.restype = ct.c_int32
        L.orcf_louvain.argtypes = [P, ct.c_int32, ct.POINTER(Params), ct.c_int64, i32p, i32p, f32p, ct.c_int64,
                                   i32p, i32p, f32p, i32p, f64p, f64p, ct.POINTER(StatsF)]
        L.orcf_arc_count.restype = ct.c_int64
        L.orcf_arc_count.argtypes = [P]
        L.orcf_export.argtypes = [P, i64p, i32p, f32p]
        L.orcf_stats_size.restype = ct.c_int32
        assert L.orcf_stats_size() == ct.sizeof(StatsF)
        L.orc_stats_size.restype = ct.c_int32
        L.orc_params_size.restype = ct.c_int32
        assert L.orc_stats_size() == ct.sizeof(Stats)
        assert L.orc_params_size() == ct.sizeof(Params)
        _lib = L
    return _lib


def _a32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _a64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


_EMPTY32 = np.zeros(0, dtype=np.int32)


def _batch_args(batch):
    if batch is None:
        return (0, _EMPTY32, _EMPTY32, _EMPTY32, 0, _EMPTY32, _EMPTY32, _EMPTY32)
    du, dv, dw = _a32(batch.del_u), _a32(batch.del_v), _a32(batch.del_w)
    iu, iv, iw = _a32(batch.ins_u), _a32(batch.ins_v), _a32(batch.ins_w)
    return (du.shape[0], du, dv, dw, iu.shape[0], iu, iv, iw)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class Graph:
    """Adjacency-list graph held by the C++ oracle."""

    def __init__(self, n=None, u=None, v=None, w=None, *, handle=None):
        L = lib()
        if handle is not None:
            self._h = handle
        else:
            st = ct.c_int32(0)
            u, v, w = _a32(u), _a32(v), _a32(w)
            h = L.orc_graph_new(int(n), int(u.shape[0]), u, v, w, ct.byref(st))
            if not h:
                raise OracleError(st.value, "graph build")
            self._h = h

    @classmethod
    def from_edges(cls, e):
        return cls(e.n, e.u, e.v, e.w)

    @classmethod
    def from_arcs(cls, n, src, dst, w):
        src, dst, w = _a32(src), _a32(dst), _a64(w)
        return cls(handle=lib().orc_graph_from_arcs(int(n), int(src.shape[0]), src, dst, w))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_graph_free(h)
            self._h = None

    @property
    def n(self) -> int:
        return lib().orc_graph_n(self._h)

    @property
    def two_m(self) -> int:
        return lib().orc_two_m(self._h)

    def arcs(self) -> int:
        return lib().orc_arc_count(self._h)

    def csr(self):
        """(offsets int64[n+1], col int32[arcs], w int64[arcs]), rows sorted."""
        n, a = self.n, self.arcs()
        off = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(a, dtype=np.int32)
        w = np.zeros(a, dtype=np.int64)
        lib().orc_export(self._h, off, col, w)
        return off, col, w

    def apply_batch(self, batch) -> int:
        return lib().orc_apply_batch(self._h, *_batch_args(batch))

    def degrees(self) -> np.ndarray:
        K = np.zeros(self.n, dtype=np.int64)
        lib().orc_weighted_degrees(self._h, K)
        return K

    def modularity(self, C) -> float:
        return float(lib().orc_modularity(self._h, _a32(C)))

    def mark(self, approach, batch, C, K, Sig):
        n = self.n
        f = np.zeros(n, dtype=np.uint8)
        r = np.zeros(n, dtype=np.uint8)
        lib().orc_mark(self._h, APPROACH[approach] if isinstance(approach, str) else approach,
                       *_batch_args(batch), _a32(C), _a64(K), _a64(Sig), f, r)
        return f, r

    def decide(self, C, K, Sig, size, verts, guard=1):
        verts = _a32(verts)
        oc = np.zeros(verts.shape[0], dtype=np.int32)
        og = np.zeros(verts.shape[0], dtype=np.int64)
        om = np.zeros(verts.shape[0], dtype=np.uint8)
        lib().orc_decide(self._h, _a32(C), _a64(K), _a64(Sig), _a32(size), int(guard),
                         verts.shape[0], verts, oc, og, om)
        return oc, og, om.astype(bool)

    def aggregate(self, C, nc) -> "Graph":
        return Graph(handle=lib().orc_aggregate(self._h, _a32(C), int(nc)))

    def louvain(self, approach="static", batch=None, state=None, prm=None, **kw):
        """Run Static/ND/DS/DF Louvain.  ``state`` = (C, K, Sigma) before the
        batch (ignored for static).  Returns (C, K, Sigma, stats dict)."""
        n = self.n
        if prm is None:
            prm = params(**kw)
        if state is None:
            C = np.zeros(n, dtype=np.int32)
            K = np.zeros(n, dtype=np.int64)
            S = np.zeros(n, dtype=np.int64)
        else:
            C, K, S = (np.array(state[0], dtype=np.int32), np.array(state[1], dtype=np.int64),
                       np.array(state[2], dtype=np.int64))
        st = Stats()
        code = lib().orc_louvain(self._h, APPROACH[approach], ct.byref(prm), *_batch_args(batch),
                                 C, K, S, ct.byref(st))
        if code != OK:
            raise OracleError(code, "louvain")
        return C, K, S, st.as_dict()


def update_weights(n, batch, C, K, Sig):
    K = np.array(K, dtype=np.int64)
    S = np.array(Sig, dtype=np.int64)
    lib().orc_update_weights(int(n), *_batch_args(batch), _a32(C), K, S)
    return K, S


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


_EMPTYF = np.zeros(0, dtype=np.float32)


def _batch_args_f(batch):
    if batch is None:
        return (0, _EMPTY32, _EMPTY32, _EMPTYF, 0, _EMPTY32, _EMPTY32, _EMPTYF)
    du, dv, dw = _a32(batch.del_u), _a32(batch.del_v), _f32(batch.del_w)
    iu, iv, iw = _a32(batch.ins_u), _a32(batch.ins_v), _f32(batch.ins_w)
    return (du.shape[0], du, dv, dw, iu.shape[0], iu, iv, iw)


class GraphF:
    """The paper-precision oracle's graph: float32 weights, FP64 sums
    (louvain_oracle_fp.cpp)."""

    def __init__(self, n, u, v, w):
        st = ct.c_int32(0)
        u, v, w = _a32(u), _a32(v), _f32(w)
        h = lib().orcf_graph_new(int(n), int(u.shape[0]), u, v, w, ct.byref(st))
        if not h:
            raise OracleError(st.value, "graph build")
        self._h = h
        self.n = int(n)

    @classmethod
    def from_edges(cls, e):
        return cls(e.n, e.u, e.v, e.w)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orcf_graph_free(h)
            self._h = None

    @property
    def two_m(self) -> float:
        return float(lib().orcf_two_m(self._h))

    def apply_batch(self, batch) -> int:
        return lib().orcf_apply_batch(self._h, *_batch_args_f(batch))

    def csr(self):
        """(offsets int64[n+1], col int32[arcs], w float32[arcs]), rows sorted."""
        a = int(lib().orcf_arc_count(self._h))
        off = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(a, dtype=np.int32)
        w = np.zeros(a, dtype=np.float32)
        lib().orcf_export(self._h, off, col, w)
        return off, col, w

    def degrees(self) -> np.ndarray:
        K = np.zeros(self.n, dtype=np.float64)
        lib().orcf_degrees(self._h, K)
        return K

    def modularity(self, C) -> float:
        return float(lib().orcf_modularity(self._h, _a32(C)))

    def decide(self, C, K, Sig, size, verts, guard=1):
        verts = _a32(verts)
        oc = np.zeros(verts.shape[0], dtype=np.int32)
        odq = np.zeros(verts.shape[0], dtype=np.float64)
        om = np.zeros(verts.shape[0], dtype=np.uint8)
        lib().orcf_decide(self._h, _a32(C), np.ascontiguousarray(K, dtype=np.float64),
                          np.ascontiguousarray(Sig, dtype=np.float64), _a32(size), int(guard), verts.shape[0],
                          verts, oc, odq, om)
        return oc, odq, om.astype(bool)

    def louvain(self, approach="static", batch=None, state=None, prm=None, **kw):
        """Static or DF Louvain in the paper's precision.  ``state`` =
        (C, K, Sigma) before the batch (FP64 K and Sigma).  Returns (C, K,
        Sigma, stats dict)."""
        n = self.n
        if prm is None:
            prm = params(**kw)
        if state is None:
            C, K, S = np.zeros(n, np.int32), np.zeros(n, np.float64), np.zeros(n, np.float64)
        else:
            C, K, S = (np.array(state[0], dtype=np.int32), np.array(state[1], dtype=np.float64),
                       np.array(state[2], dtype=np.float64))
        st = StatsF()
        code = lib().orcf_louvain(self._h, APPROACH[approach], ct.byref(prm), *_batch_args_f(batch), C, K, S,
                                  ct.byref(st))
        if code != OK:
            raise OracleError(code, "louvain (paper precision)")
        return C, K, S, st.as_dict()
