"""Benchmark: DF Louvain update latency (p50/p99) and edges scanned per
second against GPU static Louvain.

The headline line runs the largest single-GPU workload: a Chung-Lu
power-law graph of 20,000,000 vertices (degree exponent 2.1, mean degree 50,
500M undirected edges) with random 80/20 batch updates of 1e-5|E| and
1e-4|E|.  R-MAT scale 22 (4,194,304 vertices, edge factor 16, batches of
1e-7..1e-3 |E|) follows as extra keys, with the ND / DS / DF x SYNC /
ASYNC comparison.

A step is one batch through the whole hot path: apply_batch (in-place CSR
edit) then louvain_df (marking, weight update, local-moving, aggregation).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DF Louvain update latency p50/p99 & edges scanned/s vs GPU Static Louvain"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published peak
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes of the local-moving scan (Alg. 5): per scanned arc the
# neighbour id, the weight and the neighbour's community (4 + 4 + 4 B); per
# processed vertex its row start and length, K_i and C_i (8 + 4 + 8 + 4 B).
# The frontier binning kernel reads one 4 B frontier word per 32 vertices
# and, per active vertex, its row length and one list entry (4 + 4 B).  A
# hub row's decision units read at most one 8 B (community, weight) pair
# per arc; the clear kernel resets per-hub sums (and the global tables of
# rows above 2^18 arcs, not priced here).
SCAN_BYTES_PER_ARC = 12
SCAN_BYTES_PER_VERTEX = 24
BIN_BYTES_PER_WORD = 4
BIN_BYTES_PER_VERTEX = 8
HUB_PAIR_BYTES_PER_ARC = 8
KERNELS = ("k_move_all", "k_bin_frontier", "k_hub_clear", "k_hub_decide")   # index = LV_TIME_*
SHORT = ("move_all", "bin_frontier", "hub_clear", "hub_decide")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class ProfilerRegion:
    """Marks the timed region with a ROCTx range named "timed_region" so a
    profile taken with `rocprofv3 --marker-trace --kernel-trace` can be cut
    to the kernels dispatched inside it; a no-op when the marker library is
    absent."""

    def __init__(self):
        import ctypes
        self.lib = None
        for path in ("/opt/rocm/lib/librocprofiler-sdk-roctx.so", "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(path)
                self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except OSError:
                self.lib = None

    def resume(self):
        if self.lib is not None:
            self.lib.roctxRangePushA(b"timed_region")

    def pause(self):
        if self.lib is not None:
            self.lib.roctxRangePop()


class KernelMeter:
    """Per-kernel launches, event time and algorithmic bytes (index
    LV_TIME_*), summed over the louvain_* calls it is fed (their lv_stats)."""

    def __init__(self, lib, n):
        self.lib, self.n = lib, n
        self.launches = [0] * lib.NTIMED
        self.ms = [0.0] * lib.NTIMED
        self.bytes = [0] * lib.NTIMED

    def add(self, s):
        L = self.lib
        for k in range(L.NTIMED):
            self.launches[k] += s["timed_launches"][k]
            self.ms[k] += s["timed_ms"][k]
        arcs, verts = s["bin_arcs"], s["bin_vertices"]
        self.bytes[L.TIME_SCAN] += SCAN_BYTES_PER_ARC * sum(arcs) + SCAN_BYTES_PER_VERTEX * sum(verts)
        # binning runs once per sub-round; its launches are known when timed
        words = (self.n + 31) // 32
        nbin = s["timed_launches"][L.TIME_BINNING]
        self.bytes[L.TIME_BINNING] += BIN_BYTES_PER_WORD * words * nbin + BIN_BYTES_PER_VERTEX * sum(verts)
        hub_arcs = arcs[L.BINS.index("hub")]
        self.bytes[L.TIME_HUB_DECIDE] += HUB_PAIR_BYTES_PER_ARC * hub_arcs

    def dominant(self):
        return max(range(self.lib.NTIMED), key=lambda k: self.ms[k])


def move_instance(tuning):
    """Name of the fused scan instantiation a DF step launches: its
    wavefront tables hold twice the degree threshold."""
    return f"k_move_all<{2 * int(tuning['wave_max_degree'])}, 7>"


def traffic_for(kernel_name, instance, workload):
    """HBM bytes per launch of `instance` (a template instantiation of
    `kernel_name`) in the DF steps of `workload`, from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there
    is none for that instantiation or the kernel sources changed since the
    counters were taken."""
    import hashlib
    import re
    tag = "_".join(re.findall(r"\d+", instance))
    path = os.path.join(PROFILES, f"traffic_{kernel_name}_{tag}_{workload}_df.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != instance:
        return None
    src = os.path.join(ROOT, "paper_2404_19634_amd", "csrc", "move.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv.get("move_hip_sha256_16"):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _kname(name):
    import re
    name = name.replace("(anonymous namespace)::", "").replace("lv::", "").replace("void ", "")
    return re.sub(r"\(.*$", "", name)


def summarize(db_path, kernel, launches):
    """Text summary of a rocprofv3 database written by this script.

    A kernel-trace database with the ROCTx range of the timed region gives
    the per-kernel table of that region.  A counter database (one --pmc
    counter) gives, for `kernel`, the counter per dispatch averaged over its
    last `launches` dispatches (the timed region, when the final static run
    is skipped), and the same counter for the largest device copy (the 1 GiB
    calibration copy), with the scale factor the copy implies."""
    import sqlite3
    db = sqlite3.connect(db_path)
    tabs = {r[0] for r in db.execute("select name from sqlite_master where type in ('table','view')")}
    out = []
    rows = []
    if "counters_collection" in tabs:
        rows = db.execute("select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
                          "group by dispatch_id, counter_name order by dispatch_id").fetchall()
    if rows and kernel == "all":
        counters = sorted({r[2] for r in rows})
        names = sorted({_kname(k) for d, k, c, v in rows})
        out.append(f"{'kernel (avg per dispatch, last ' + str(launches or 'all') + ')':40s} " +
                   " ".join(f"{c:>24s}" for c in counters))
        for nm in names:
            cells = []
            for cn in counters:
                vals = [v for d, k, c, v in rows if c == cn and _kname(k) == nm]
                tail = vals[-launches:] if launches else vals
                cells.append(f"{sum(tail) / len(tail):24.1f}" if tail else f"{'-':>24s}")
            out.append(f"{nm[:40]:40s} " + " ".join(cells))
        return "\n".join(out)
    if rows:
        counters = sorted({r[2] for r in rows})
        for cn in counters:
            mine = [v for d, k, c, v in rows if c == cn and _kname(k) == kernel]
            copies = [v for d, k, c, v in rows if c == cn and "copyBuffer" in k]
            tail = mine[-launches:] if launches else mine
            avg = sum(tail) / len(tail) if tail else float("nan")
            # the calibration copy (1 GiB device to device) is the run's last copy
            big = copies[-1] if copies else float("nan")
            scale = (1 << 20) / big if copies and big > 0 else float("nan")
            out.append(f"{cn}: {kernel} dispatches {len(mine)}, last {len(tail)} average {avg:.1f} KiB")
            out.append(f"{cn}: last copy (the 1 GiB calibration copy) reads {big:.1f} KiB -> scale {scale:.4f}")
            out.append(f"{cn}_bytes_per_launch: {avg * scale * 1024:.0f}")
        return "\n".join(out)
    t0 = t1 = None
    if "regions" in tabs:
        r = db.execute("select start, end from regions where category like 'MARKER%'").fetchall()
        if len(r) == 1:
            t0, t1 = r[0]
    q = "select name, duration from kernels" + (" where start >= ? and end <= ?" if t0 is not None else "")
    rows = db.execute(q, (t0, t1) if t0 is not None else ()).fetchall()
    agg = {}
    for name, d in rows:
        a = agg.setdefault(_kname(name), [0, 0.0, float("inf"), 0.0])
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
    tot = sum(a[1] for a in agg.values())
    if t0 is not None:
        out.append(f"timed region {(t1 - t0) / 1e6:.3f} ms, {len(rows)} dispatches, kernel time {tot / 1e6:.3f} ms")
    out.append(f"{'kernel':34s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}")
    for k, a in sorted(agg.items(), key=lambda x: -x[1][1]):
        out.append(f"{k[:34]:34s} {a[0]:6d} {a[1] / 1e6:9.3f} {a[1] / a[0] / 1e3:8.2f} {a[2] / 1e3:8.2f} "
                   f"{a[3] / 1e3:8.2f} {100 * a[1] / tot:6.2f}")
    return "\n".join(out)


def pct(x, q):
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else None


def host_cpu():
    """The host's CPU model, the logical CPUs it has and those this process
    may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(e, batch, budget_s=60.0):
    """The sequential oracle (one thread) on a bounded sample of the same
    workload: one full local-moving sweep of static Louvain (every vertex
    scanned once), then DF Louvain on one batch starting from that sweep's
    partition."""
    import oracle
    t0 = time.perf_counter()
    G = oracle.Graph.from_edges(e)
    build_s = time.perf_counter() - t0
    C, K, S, st = G.louvain("static", mode="async", max_passes=1, max_iterations=1)
    sweep_s, sweep_arcs = st["seconds"], st["arcs_scanned"]
    res = {"value": sweep_arcs / sweep_s, "unit": "edges scanned/s", "cores": 1, "kind": "oracle",
           "sample": (f"one static local-moving sweep over all {sweep_arcs} arcs "
                      f"({sweep_s:.2f} s) then DF Louvain on one batch of {batch.size} updates"),
           "static_sweep_edges_per_s": sweep_arcs / sweep_s, "graph_build_s": build_s, **host_cpu()}
    if sweep_s < budget_s:
        assert G.apply_batch(batch) == 0
        C2, K2, S2, st2 = G.louvain("df", batch=batch, state=(C, K, S), mode="async")
        res["df_latency_ms"] = st2["seconds"] * 1e3
        res["df_edges_scanned"] = st2["arcs_scanned"]
        res["df_edges_per_s"] = st2["arcs_scanned"] / st2["seconds"] if st2["seconds"] > 0 else None
    del G
    return res


def cpu_multicore(e, batches, count=4):
    """The multi-core CPU implementation (baseline_cpu: the paper's OpenMP
    design, all host threads) on the same workload: static Louvain in ASYNC
    mode, then DF Louvain on the first `count` batches of the sequence
    (apply_batch untimed, as the paper times the algorithm only)."""
    import baseline_cpu
    t0 = time.perf_counter()
    P = baseline_cpu.Graph(e)
    build_s = time.perf_counter() - t0
    C, K, S, st = P.louvain("static", mode="async")
    q = P.modularity(C)
    lat, arcs = [], []
    state = (C, K, S)
    for b in batches[:count]:
        assert P.apply_batch(b) == 0
        C, K, S, sd = P.louvain("df", batch=b, state=state, mode="async")
        state = (C, K, S)
        lat.append(sd["seconds"] * 1e3)
        arcs.append(sd["arcs_scanned"])
    del P
    return {"kind": "multicore (OpenMP, the paper's parallel design)", "threads": st["threads"],
            "graph_build_s": build_s, "static_latency_ms": st["seconds"] * 1e3,
            "static_edges_scanned_per_s": st["arcs_scanned"] / st["seconds"], "static_modularity": q,
            "static_passes": st["passes"], "static_iterations": st["iterations"],
            "df_latency_ms": lat, "df_batch_sizes": [b.size for b in batches[:count]],
            "df_latency_ms_p50": pct(lat, 50), "df_edges_scanned_per_s": float(np.sum(arcs)) / (np.sum(lat) * 1e-3),
            **host_cpu()}


def sweep(g, e, runs):
    """One SYNC local-moving iteration over every vertex from singletons,
    `runs` times (the kernels a full sweep launches, for rocprofv3), then a
    plain 1 GiB device-to-device copy whose counters calibrate FETCH_SIZE
    and WRITE_SIZE."""
    import torch
    from paper_2404_19634_amd import lib
    prm = lib.params(mode="sync", max_iterations=1, max_passes=1)
    st = lib.State.empty(e.n, g.device)
    for r in range(runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, s = lib.louvain_static(g, prm, st)
        torch.cuda.synchronize()
        log(f"sweep {r}: {1e3 * (time.perf_counter() - t):.3f} ms, arcs {s['arcs_scanned']}, "
            f"moves {s['moves']}, ms_move {s['ms_move']:.3f}")
    x = torch.empty(1 << 28, dtype=torch.int32, device=g.device).fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    log("copy: 1 GiB read + 1 GiB written")


def full_sweep_roofline(lib, g, runs=3):
    """Roofline of the scan on a full sweep: one SYNC local-moving iteration
    over every vertex from singletons (static Louvain's first iteration),
    the scan kernel's launches timed with HIP events.  Bytes are the
    algorithmic ones (12 B per arc, 24 B per vertex).  The best of `runs`."""
    import torch
    prm = lib.params(mode="sync", max_iterations=1, max_passes=1)
    best = None
    lib.set_timing([lib.TIME_SCAN])
    try:
        for _ in range(runs):
            st = lib.State.empty(g.n, g.device)
            torch.cuda.synchronize()
            st, s = lib.louvain_static(g, prm, st)
            torch.cuda.synchronize()
            ms = s["timed_ms"][lib.TIME_SCAN]
            if best is None or ms < best[0]:
                best = (ms, s)
    finally:
        lib.set_timing(())
    ms, s = best
    arcs, verts = sum(s["bin_arcs"]), sum(s["bin_vertices"])
    nbytes = SCAN_BYTES_PER_ARC * arcs + SCAN_BYTES_PER_VERTEX * verts
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": "k_move_all (all roles, hub insert units included)",
            "launches": s["timed_launches"][lib.TIME_SCAN], "scan_ms": ms, "bytes": nbytes,
            "arcs": arcs, "vertices": verts, "local_moving_ms": s["ms_move"],
            "local_moving_edges_per_s": arcs / (s["ms_move"] * 1e-3) if s["ms_move"] > 0 else None,
            "workload": "one SYNC local-moving iteration from singletons over every vertex"}


def approaches(lib, e, sizes, reps=2, seed=777):
    """Update latency of ND, DS and DF Louvain in SYNC and ASYNC mode, and
    static Louvain in both modes, on the same graph: per (approach, mode) a
    fresh copy of the graph, its static state, then `reps` rounds of the
    batch sizes, each apply_batch followed by the approach (timed).  In
    ASYNC mode each approach also runs without auxiliary information (K and
    Sigma recomputed from scratch per batch, "async_no_aux"), and
    "aux_speedup" is that variant's p50 over the incremental one's."""
    import torch
    from paper_2404_19634_amd import workloads as W
    dev = torch.device("cuda:0")
    batches = W.batch_sequence(e, sizes, reps * len(sizes), seed=seed)
    out = {"static": {}}
    for mode in ("sync", "async"):
        prm = lib.params(mode=mode)
        g = lib.Graph.from_edges(e, slack_frac=0.1, slack_min=8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st0, s0 = lib.louvain_static(g, prm, lib.State.empty(e.n, dev))
        torch.cuda.synchronize()
        out["static"][mode] = {"latency_ms": (time.perf_counter() - t) * 1e3, "edges_scanned": s0["arcs_scanned"],
                               "modularity": lib.modularity(g, st0.C)}
        del g
        runs = [(name, 0) for name in ("nd", "ds", "df")]
        if mode == "async":
            runs += [(name, 1) for name in ("nd", "ds", "df")]
        for name, no_aux in runs:
            fn = getattr(lib, "louvain_" + name)
            prm_run = lib.params(mode=mode, recompute_weights=no_aux)
            g = lib.Graph.from_edges(e, slack_frac=0.1, slack_min=8)
            st = st0.clone()
            lat, arcs, by = [], [], {}
            for b in batches:
                db = lib.Batch.from_host(b, dev)
                try:
                    lib.apply_batch(g, db)
                except lib.LouvainError as ex:
                    if ex.code != lib.LV_ENOSLACK:
                        raise
                    g = g.relayout(slack_frac=0.5, slack_min=16)
                    lib.apply_batch(g, db)
                torch.cuda.synchronize()
                t = time.perf_counter()
                st, s = fn(g, db, st, prm_run)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t) * 1e3
                lat.append(ms)
                arcs.append(s["arcs_scanned"])
                by.setdefault(str(b.size), []).append(ms)
            rec = {
                "latency_ms_p50": pct(lat, 50), "latency_ms_p99": pct(lat, 99),
                "by_batch_size": {k: float(np.median(v)) for k, v in by.items()},
                "edges_scanned_per_s": float(np.sum(arcs)) / (np.sum(lat) * 1e-3),
                "speedup_vs_static": out["static"][mode]["latency_ms"] / pct(lat, 50),
                "modularity": lib.modularity(g, st.C)}
            if no_aux:
                rec["aux_speedup"] = pct(lat, 50) / out[name][mode]["latency_ms_p50"]
                out[name][mode + "_no_aux"] = rec
            else:
                out.setdefault(name, {})[mode] = rec
            del g, st
            torch.cuda.empty_cache()
    return out


def _gen_graph(spec):
    """One graph of the many-graph workload and three consecutive 1e-3|E|
    batches: the tuning pass, the burst and the Poisson phase."""
    from paper_2404_19634_amd import workloads as W
    n, b, seed = spec
    e = W.multi_sbm_graph(int(n), int(b), int(seed))
    out = [e]
    cur = e
    for k in range(3):
        bk = W.random_batch(cur, W.batch_size(1e-3, cur.m), (int(seed) + k) % (1 << 30))
        out.append(bk)
        cur = W.apply_batch_np(cur, bk)
    return tuple(out)


def serve_bench(args):
    """Many independent SBM graphs (vertex counts log-uniform in [1e3, 2e5],
    block sizes log-uniform in [20, 2000], expected intra/inter degree
    12/3), each with 1e-3|E| 80/20 batches, served from HBM.  Phase 1 sends
    every graph's first batch at once (the batched persistent launch at
    saturation); phase 2 sends the second batches with Poisson arrivals at
    a fraction of that rate and reports latency percentiles."""
    import multiprocessing as mp
    import torch
    from paper_2404_19634_amd import lib, serve
    from paper_2404_19634_amd import workloads as W
    lib.load()
    specs = W.multi_sbm_specs(args.serve_graphs, 1244)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
        data = pool.map(_gen_graph, specs, chunksize=4)
    sum_n = sum(d[0].n for d in data)
    sum_m = sum(d[0].m for d in data)
    log(f"{len(data)} graphs, {sum_n} vertices, {sum_m} edges generated in {time.perf_counter() - t0:.1f} s")
    cap = max(max(b.size for b in d[1:]) for d in data)
    free, _ = torch.cuda.mem_get_info()
    store = serve.GraphStore(int(free * 0.8), max_updates=cap, mode=args.mode)
    for gid, d in enumerate(data):
        store.add(gid, d[0])
    t0 = time.perf_counter()
    store.acquire(list(range(len(data))))
    store.release(list(range(len(data))))
    torch.cuda.synchronize()
    log(f"resident: {store.resident_bytes / 1e9:.2f} GB after {time.perf_counter() - t0:.1f} s "
        f"(build + static Louvain per graph)")
    # tuning pass: every graph's first batch in one lv_autotune_many call,
    # whose items are dealt to the candidate mappings of the batched launch
    t0 = time.perf_counter()
    gids = list(range(len(data)))
    tuned = store.tune(gids, [d[1] for d in data])
    tune_s = time.perf_counter() - t0
    log(f"tuning pass: {len(data)} updates in {tune_s * 1e3:.1f} ms, class {tuned['size_class']}: {tuned['tuning']}")
    srv = serve.Server(store, slots=args.serve_slots, workers=2)
    srv.start()
    t0 = time.perf_counter()
    for gid, d in enumerate(data):
        srv.submit(gid, d[2], t_arrival=t0)
    srv.wait(len(data))
    burst_s = time.perf_counter() - t0
    burst = srv.summary()
    # the burst's scan work, from the per-graph statistics of its launches
    # (the k_many_df roofline divides its algorithmic bytes by the launch's
    # duration in a kernel trace)
    arcs = verts = 0
    for r in srv.done:
        if r.src:
            sts, q = r.src
            arcs += int(sts[q]["arcs_scanned"])
            verts += int(sts[q]["vertices_affected"])
    burst["arcs_scanned"] = arcs
    burst["vertices_affected"] = verts
    burst["scan_algorithmic_bytes"] = SCAN_BYTES_PER_ARC * arcs + SCAN_BYTES_PER_VERTEX * verts
    sat = len(data) / burst_s
    log(f"burst: {len(data)} updates in {burst_s * 1e3:.1f} ms ({sat:.0f} graphs/s), {burst}")
    srv.done.clear()
    srv.launches = 0
    rate = args.serve_load * sat
    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / rate, len(data))
    order = rng.permutation(len(data))
    # arrivals at their scheduled times: whatever is due is submitted (with
    # its scheduled time as arrival), then the submitter sleeps, so that it
    # does not hold the interpreter lock the workers need
    due = time.perf_counter() + np.cumsum(gaps)
    k = 0
    while k < len(order):
        now = time.perf_counter()
        while k < len(order) and due[k] <= now:
            srv.submit(int(order[k]), data[int(order[k])][3], t_arrival=float(due[k]))
            k += 1
        time.sleep(2e-4)
    srv.wait(len(data))
    srv.close()
    poisson = srv.summary()
    out = {"metric": "batched DF update latency p50/p99 and graphs/s, many-graph serving", "unit": "graphs/s",
           "value": sat, "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "int64",
           "config": {"workload": f"{len(data)} SBM graphs (n log-uniform 1e3..2e5, blocks log-uniform 20..2000, "
                                  f"degree 12/3), 1e-3|E| 80/20 batches", "graphs": len(data),
                      "vertices": sum_n, "undirected_edges": sum_m, "mode": args.mode, "slots": args.serve_slots},
           "tuning": {"ms": tune_s * 1e3, **tuned},
           "burst": {"graphs_per_s": sat, "ms": burst_s * 1e3, **burst},
           "poisson": {"offered_rate_per_s": rate, "load": args.serve_load, **poisson},
           "resident_gb": store.resident_bytes / 1e9}
    print(json.dumps(out), flush=True)


# Workloads of the DF line: the batch sizes (fractions of |E|) and the seed
# of the batch pools.  The sequences match the ones the oracle's ASYNC
# fixtures were computed on (tests/golden/async_quality_<name>.json) when
# warmup + steps equals their batch count.
WORKLOADS = {
    "chunglu20m": {"desc": "Chung-Lu power-law graph, 20,000,000 vertices, degree exponent 2.1, mean degree 50 "
                           "(500M undirected edges, unit weights), random 80/20 batches of 1e-5 and 1e-4 |E|",
                   "fracs": [1e-5, 1e-4], "seed": 4343},
    "rmat22": {"desc": "R-MAT scale 22 (edge factor 16, a=0.57 b=0.19 c=0.19), random 80/20 batches of "
                       "1e-7..1e-3 |E|",
               "fracs": [1e-7, 1e-6, 1e-5, 1e-4, 1e-3], "seed": 4242},
}


def load_workload(name):
    from paper_2404_19634_amd import workloads as W
    if name == "chunglu20m":
        return W.config3_chung_lu(device="cuda")
    if name == "rmat22":
        return W.config2_rmat()
    raise SystemExit(f"unknown workload {name}")


def oracle_fixture(name, batches):
    """The oracle's ASYNC modularity values for this workload's batch
    sequence, when the sequence is the one they were computed on."""
    path = os.path.join(ROOT, "tests", "golden", f"async_quality_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        gold = json.load(f)
    from tests.golden import make_async_golden as MG
    if len(batches) != gold["batch_count"] or MG.batches_fingerprint(batches) != gold["batches_sha256_32"]:
        return None
    return gold


def df_line(args, lib, name, e, region=None):
    """Static Louvain and the DF steps on workload `name` (graph `e`):
    returns the line's fields and the GPU graph after the steps."""
    import torch
    from paper_2404_19634_amd import workloads as W
    dev = torch.device("cuda:0")
    spec = WORKLOADS[name]
    sizes = [W.batch_size(f, e.m) for f in spec["fracs"]]
    total = args.warmup + args.steps
    t0 = time.perf_counter()
    batches = W.batch_sequence(e, sizes, total, seed=spec["seed"])
    dbatches = [lib.Batch.from_host(b, dev) for b in batches]
    g = lib.Graph.from_edges(e, slack_frac=0.1, slack_min=8)
    prm = lib.params(mode=args.mode)
    torch.cuda.synchronize()
    log(f"{name}: {len(batches)} batches of {sizes}, graph on the device ({time.perf_counter() - t0:.1f} s)")
    if args.sweep:
        sweep(g, e, args.sweep)
        return None, g, None
    lib.set_tuning(**args.tuning_kv)
    autotune_ms = None
    if not args.no_autotune and "wave_max_degree" not in args.tuning_kv:
        t = time.perf_counter()
        lib.autotune(g, repeats=2)
        autotune_ms = (time.perf_counter() - t) * 1e3
        log(f"autotune: {lib.get_tuning()} ({autotune_ms:.0f} ms)")

    # GPU static Louvain on the initial graph (comparison baseline)
    static_ms, static_arcs, static_stats = [], [], None
    state0 = None
    for r in range(args.static_runs):
        st = lib.State.empty(e.n, dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, s = lib.louvain_static(g, prm, st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if r > 0 or args.static_runs == 1:
            static_ms.append(dt * 1e3)
            static_arcs.append(s["arcs_scanned"])
        static_stats, state0 = s, st
    q_static = lib.modularity(g, state0.C)
    log(f"static: {np.median(static_ms):.2f} ms, arcs scanned {static_arcs[-1]}, Q={q_static:.6f}, "
        f"passes {static_stats['passes']} iters {static_stats['iterations']}")

    # DF steps.  The warmup times every scan kernel (HIP events) to find the
    # one that dominates; the timed region brackets only that kernel.
    state = state0.clone()
    lat, arcs, per_size, stats = [], [], {}, []
    relayouts = 0
    warm = KernelMeter(lib, e.n)
    meter = KernelMeter(lib, e.n)
    lib.set_timing(range(lib.NTIMED))
    torch.cuda.synchronize()
    dom = None
    t_region = time.perf_counter()
    for k in range(total):
        if k == args.warmup:
            dom = warm.dominant() if args.warmup else lib.TIME_BINNING
            lib.set_timing([dom])
            torch.cuda.synchronize()
            if region is not None:
                region.resume()
            t_region = time.perf_counter()
        b = dbatches[k]
        t = time.perf_counter()
        # one update: the batch edit and DF Louvain in one call (one host wait)
        try:
            state, s = lib.louvain_df_apply(g, b, state, prm)
        except lib.LouvainError as ex:  # a row ran out of slack (nothing changed): re-lay out, retry
            if ex.code != lib.LV_ENOSLACK:
                raise
            g = g.relayout(slack_frac=0.5, slack_min=16)
            relayouts += 1
            state, s = lib.louvain_df_apply(g, b, state, prm)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k < args.warmup:
            warm.add(s)
        else:
            # statistics are read after the timed region
            stats.append(s)
            lat.append((t2 - t) * 1e3)
            per_size.setdefault(batches[k].size, []).append((t2 - t) * 1e3)
    torch.cuda.synchronize()
    region_s = time.perf_counter() - t_region
    if region is not None:
        region.pause()
    for s in stats:
        meter.add(s)
        arcs.append(s["arcs_scanned"])
    lib.set_timing(())
    q_df = lib.modularity(g, state.C)

    # static Louvain on the final graph, same mode (quality and time reference)
    static_final_ms = q_static_final = None
    if not args.no_final_static:
        st = lib.State.empty(e.n, dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, s_final = lib.louvain_static(g, prm, st)
        torch.cuda.synchronize()
        static_final_ms = (time.perf_counter() - t) * 1e3
        q_static_final = lib.modularity(g, st.C)
        del st
    del state, state0
    if args.calibrate_copy:
        x = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    df_arcs = int(np.sum(arcs))
    static_eps = float(np.median([a / (m / 1e3) for a, m in zip(static_arcs, static_ms)]))
    out = {
        "value": df_arcs / region_s,
        "ms_per_step": region_s * 1e3 / args.steps,
        "config": {"workload": spec["desc"], "vertices": e.n, "undirected_edges": e.m, "batch_sizes": sizes,
                   "mode": args.mode, "tuning": lib.get_tuning(), "autotuned": autotune_ms is not None,
                   "autotune_ms": autotune_ms},
        "df_latency_ms_p50": pct(lat, 50),
        "df_latency_ms_p99": pct(lat, 99),
        "df_latency_ms_by_batch_size": {str(k): float(np.median(v)) for k, v in sorted(per_size.items())},
        "latency_includes_batch_edit": True,
        "relayouts": relayouts,
        "df_edges_scanned_per_s": df_arcs / (np.sum(lat) / 1e3),
        "static_latency_ms": float(np.median(static_ms)),
        "static_edges_scanned_per_s": static_eps,
        "static_passes": static_stats["passes"], "static_iterations": static_stats["iterations"],
        "df_speedup_vs_static": float(np.median(static_ms)) / pct(lat, 50),
        "modularity": {"static_initial": q_static, "df_final": q_df, "static_final": q_static_final},
        "static_final_ms": static_final_ms,
    }
    gold = oracle_fixture(name, batches)
    if gold is not None:
        out["modularity"]["oracle"] = {"static_initial": gold["static_async"]["modularity"],
                                       "df_final": gold["df_chain_async"]["modularity"],
                                       "static_final": gold["static_async_final_graph"]["modularity"],
                                       "source": f"tests/golden/async_quality_{name}.json"}
    nl = meter.launches[dom]
    if nl and meter.ms[dom] > 0:
        per_launch = meter.bytes[dom] / nl
        achieved = per_launch / (meter.ms[dom] / nl * 1e-3) / 1e9
        inst = move_instance(lib.get_tuning()) if dom == lib.TIME_SCAN else KERNELS[dom]
        tr = traffic_for(SHORT[dom], inst, name)
        out["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "kernel": inst,
            "launches": nl, "avg_launch_us": meter.ms[dom] / nl * 1e3, "bytes_per_launch": per_launch,
            "warmup_kernel_ms": {lib.TIMED[k]: round(warm.ms[k], 4) for k in range(lib.NTIMED)},
        }
    if not args.no_approaches:
        log("full-sweep roofline ...")
        out["roofline_full_sweep"] = full_sweep_roofline(lib, g)
    return out, g, batches


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="chunglu20m", choices=sorted(WORKLOADS),
                    help="workload of the headline line (the other one follows as extra keys)")
    ap.add_argument("--mode", default="async", choices=["async", "sync"])
    ap.add_argument("--static-runs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tuning instead of lv_autotune's choice for the graph")
    ap.add_argument("--no-approaches", action="store_true",
                    help="skip the ND/DS/DF x SYNC/ASYNC comparison and the full-sweep rooflines")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only (no R-MAT keys)")
    ap.add_argument("--tuning", default="", help="lv_tuning overrides, e.g. fuse_max_frontier=1024,defer_totals=1")
    ap.add_argument("--no-final-static", action="store_true",
                    help="skip the static run on the final graph (counter runs: the timed region's dispatches "
                         "are then the last ones of each kernel)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain 1 GiB device copy whose counters calibrate FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--summarize", metavar="DB", help="print a summary of a rocprofv3 database and exit")
    ap.add_argument("--kernel", default="k_move_all<512, 7>",
                    help="kernel of --summarize for counter databases ('all': a table of every kernel)")
    ap.add_argument("--launches", type=int, default=0, help="last dispatches of --kernel to average")
    ap.add_argument("--serve", action="store_true", help="many-graph serving benchmark instead of the DF line")
    ap.add_argument("--serve-graphs", type=int, default=4096)
    ap.add_argument("--serve-slots", type=int, default=4096)
    ap.add_argument("--serve-load", type=float, default=0.5, help="Poisson rate as a fraction of the burst rate")
    ap.add_argument("--sweep", type=int, default=0,
                    help="profiling mode: run this many single full local-moving sweeps (SYNC, all vertices "
                         "from singletons) of the workload and one 1 GiB device copy for counter "
                         "calibration, then exit")
    args = ap.parse_args()
    if args.summarize:
        print(summarize(args.summarize, args.kernel, args.launches))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the single-GPU line is the result",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_19634_amd import lib

    if args.serve:
        serve_bench(args)
        return
    args.tuning_kv = {k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(",") if kv)}
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    e = load_workload(args.workload)
    torch.cuda.synchronize()
    log(f"{args.workload}: n={e.n} undirected edges={e.m} ({time.perf_counter() - t0:.1f} s)")
    head, g, batches = df_line(args, lib, args.workload, e, region=ProfilerRegion())
    if head is None:   # --sweep
        return
    out = {"metric": METRIC, "value": head.pop("value"), "unit": "edges scanned/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic", "config": head.pop("config")}
    out.update(head)
    if args.workload == "rmat22" and not args.no_approaches:
        log("approaches (ND / DS / DF x SYNC / ASYNC) ...")
        out["approaches"] = approaches(lib, e, out["config"]["batch_sizes"])
    del g
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(e, batches[0])
        log("cpu baseline (multi-core) ...")
        out["cpu_baseline"]["multicore"] = cpu_multicore(e, batches)
    del e
    if not args.no_extras and args.workload != "rmat22":
        log("rmat22 ...")
        e2 = load_workload("rmat22")
        extra, g2, b2 = df_line(args, lib, "rmat22", e2)
        del g2
        torch.cuda.empty_cache()
        if not args.no_approaches:
            log("approaches (ND / DS / DF x SYNC / ASYNC) ...")
            extra["approaches"] = approaches(lib, e2, extra["config"]["batch_sizes"])
        out["rmat22"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
