"""Multi-core CPU DF Louvain (the paper's OpenMP design) for the
benchmark's CPU comparison.

Measurement infrastructure: only the test suite and the benchmark's CPU
leg use this package; the product library never imports it.  The C++ code
(``louvain_omp.cpp``, compiled by :func:`build`) shares nothing with the
oracle or the GPU library; this module marshals numpy arrays over ctypes.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "louvain_omp.cpp")
LIB = os.path.join(HERE, "liblouvain_omp.so")

STATIC, ND, DF = 0, 1, 3
APPROACH = {"static": STATIC, "nd": ND, "df": DF}
MODE = {"sync": 0, "async": 1}
MAX_PASSES, MAX_ITERS = 16, 32


def build(force: bool = True) -> str:
    """Compile ``liblouvain_omp.so`` with the host compiler and OpenMP."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class Params(ct.Structure):
    _fields_ = [("tolerance", ct.c_double), ("tolerance_drop", ct.c_double),
                ("aggregation_tolerance", ct.c_double), ("max_iterations", ct.c_int32),
                ("max_passes", ct.c_int32), ("mode", ct.c_int32), ("swap_guard", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("passes", ct.c_int32), ("iterations", ct.c_int32 * MAX_PASSES),
                ("communities", ct.c_int64 * MAX_PASSES), ("moves", ct.c_int64), ("arcs_scanned", ct.c_int64),
                ("vertices_affected", ct.c_int64), ("iter_moves", (ct.c_int64 * MAX_ITERS) * MAX_PASSES),
                ("iter_gain", (ct.c_int64 * MAX_ITERS) * MAX_PASSES), ("seconds", ct.c_double),
                ("threads", ct.c_int32)]

    def as_dict(self) -> dict:
        p = self.passes
        its = [self.iterations[k] for k in range(p)]
        return {"passes": p, "iterations": its, "communities": [int(self.communities[k]) for k in range(p)],
                "moves": int(self.moves), "arcs_scanned": int(self.arcs_scanned),
                "vertices_affected": int(self.vertices_affected),
                "iter_moves": [[int(self.iter_moves[k][t]) for t in range(its[k])] for k in range(p)],
                "iter_gain": [[int(self.iter_gain[k][t]) for t in range(its[k])] for k in range(p)],
                "seconds": float(self.seconds), "threads": int(self.threads)}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ct.CDLL(LIB)
        P = ct.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        L.omp_threads.restype = ct.c_int32
        L.omp_graph_new.restype = P
        L.omp_graph_new.argtypes = [ct.c_int32, ct.c_int64, i32p, i32p, i32p, ct.POINTER(ct.c_int32)]
        L.omp_graph_free.argtypes = [P]
        L.omp_apply_batch.restype = ct.c_int32
        L.omp_apply_batch.argtypes = [P, ct.c_int64, i32p, i32p, i32p, ct.c_int64, i32p, i32p, i32p]
        L.omp_modularity.restype = ct.c_double
        L.omp_modularity.argtypes = [P, i32p]
        L.omp_louvain.restype = ct.c_int32
        L.omp_louvain.argtypes = [P, ct.c_int32, ct.POINTER(Params), ct.c_int64, i32p, i32p, i32p, ct.c_int64, i32p,
                                  i32p, i32p, i32p, i64p, i64p, ct.POINTER(Stats)]
        L.omp_stats_size.restype = ct.c_int32
        L.omp_params_size.restype = ct.c_int32
        assert L.omp_stats_size() == ct.sizeof(Stats)
        assert L.omp_params_size() == ct.sizeof(Params)
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().omp_threads())


def params(tolerance=1e-2, tolerance_drop=10.0, aggregation_tolerance=0.8, max_iterations=20, max_passes=10,
           mode="async", swap_guard=1) -> Params:
    """Defaults are the paper's (Section 5.1.2)."""
    return Params(float(tolerance), float(tolerance_drop), float(aggregation_tolerance), int(max_iterations),
                  int(max_passes), MODE[mode] if isinstance(mode, str) else int(mode), int(swap_guard))


def _a32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


_EMPTY = np.zeros(0, dtype=np.int32)


def _batch_args(b):
    if b is None:
        return (0, _EMPTY, _EMPTY, _EMPTY, 0, _EMPTY, _EMPTY, _EMPTY)
    d = (_a32(b.del_u), _a32(b.del_v), _a32(b.del_w))
    i = (_a32(b.ins_u), _a32(b.ins_v), _a32(b.ins_w))
    return (d[0].shape[0], *d, i[0].shape[0], *i)


class Graph:
    """Adjacency rows held by the multi-core CPU implementation."""

    def __init__(self, e):
        st = ct.c_int32(0)
        self._h = lib().omp_graph_new(int(e.n), int(e.m), _a32(e.u), _a32(e.v), _a32(e.w), ct.byref(st))
        if not self._h:
            raise RuntimeError(f"graph build failed with status {st.value}")
        self.n = int(e.n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.omp_graph_free(h)
            self._h = None

    def apply_batch(self, b) -> int:
        return int(lib().omp_apply_batch(self._h, *_batch_args(b)))

    def modularity(self, C) -> float:
        return float(lib().omp_modularity(self._h, _a32(C)))

    def louvain(self, approach="static", batch=None, state=None, prm=None, **kw):
        """Static, ND or DF Louvain.  ``state`` = (C, K, Sigma) before the
        batch (ignored for static).  Returns (C, K, Sigma, stats dict)."""
        n = self.n
        prm = prm if prm is not None else params(**kw)
        if state is None:
            C, K, S = np.zeros(n, np.int32), np.zeros(n, np.int64), np.zeros(n, np.int64)
        else:
            C, K, S = (np.array(state[0], dtype=np.int32), np.array(state[1], dtype=np.int64),
                       np.array(state[2], dtype=np.int64))
        st = Stats()
        code = lib().omp_louvain(self._h, APPROACH[approach], ct.byref(prm), *_batch_args(batch), C, K, S,
                                 ct.byref(st))
        if code != 0:
            raise RuntimeError(f"louvain failed with status {code}")
        return C, K, S, st.as_dict()
