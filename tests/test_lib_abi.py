"""The C-ABI library loads and exports every entry point the header declares
(no device work: these run without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "louvain.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("louvain_static", "louvain_nd", "louvain_ds", "louvain_df", "apply_batch", "modularity",
                 "lv_workspace_bytes", "lv_graph_build", "lv_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2404_19634_amd import lib
    L = lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(lib.EXPORTS) <= set(declared_functions())


def test_struct_layouts_match_header():
    from paper_2404_19634_amd import lib
    # lv_params: 3 doubles + 6 int32
    assert ct.sizeof(lib.Params) == 3 * 8 + 6 * 4
    # lv_stats starts with the oracle's layout
    import oracle
    prefix = ct.sizeof(oracle.Stats)
    assert lib.Stats.ms_mark.offset == prefix
    assert ct.sizeof(lib.CGraph) == 56


def test_workspace_size_is_monotone_and_host_only():
    from paper_2404_19634_amd import lib
    L = lib.load()
    a = L.lv_workspace_bytes(1000, 10000)
    b = L.lv_workspace_bytes(2000, 10000)
    c = L.lv_workspace_bytes(2000, 40000)
    assert 0 < a < b < c
    assert L.lv_graph_capacity_bound(10, 5, 0.0, 0) >= 10


def test_default_params_are_the_papers():
    from paper_2404_19634_amd import lib
    p = lib.Params()
    lib.load().lv_default_params(ct.byref(p))
    assert (p.tolerance, p.tolerance_drop, p.aggregation_tolerance) == (1e-2, 10.0, 0.8)
    assert (p.max_iterations, p.max_passes) == (20, 10)
    assert (p.recompute_weights, p.reserved) == (0, 0)


def test_bad_parameters_rejected_before_device_work():
    # host-side checks only: the graph's pointers are never dereferenced
    from paper_2404_19634_amd import lib
    L = lib.load()
    g = lib.CGraph(10, 40, 8, 8, 8, 8, 8)
    e = lib.CEdges(None, None, None, 0)
    s = lib.CState(8, 8, 8, None)
    st = lib.Stats()
    for kw in ({"recompute_weights": 2}, {"max_iterations": 0}, {"mode": 7}):
        p = lib.params(**kw)
        code = L.louvain_df(ct.byref(g), ct.byref(e), ct.byref(e), ct.byref(p), ct.byref(s), None, 0,
                            ct.byref(st), None)
        assert code == lib.LV_EINVAL, kw
        assert b"parameters" in L.lv_last_error(), kw
    p = lib.params()
    p.reserved = 1
    code = L.louvain_df(ct.byref(g), ct.byref(e), ct.byref(e), ct.byref(p), ct.byref(s), None, 0, ct.byref(st), None)
    assert code == lib.LV_EINVAL


def test_null_arguments_rejected_without_device_work():
    from paper_2404_19634_amd import lib
    L = lib.load()
    st = lib.Stats()
    p = lib.params()
    code = L.louvain_static(None, ct.byref(p), None, None, 0, ct.byref(st), None)
    assert code == lib.LV_EINVAL
    assert b"invalid" in L.lv_last_error()
