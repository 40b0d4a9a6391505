"""Writes the ASYNC quality fixtures ``async_quality_<workload>.json``.

Every value is computed by the sequential oracle (``oracle/``) from the
seeded generators (``paper_2404_19634_amd/workloads.py``); nothing comes
from the HIP path.  For one large workload it records:

* the oracle's static Louvain in ASYNC mode (Alg. 4 with every vertex
  affected, local-moving by Alg. 5 in ascending id order): modularity
  (Eq. 1), passes and iterations per pass;
* the oracle's DF Louvain chain (Alg. 1) from that static result over the
  workload's batch sequence (Section 5.1.4 random batches), modularity at
  the end;
* the oracle's static Louvain on the final graph (the reference the
  paper's "DF reaches static's modularity" statement compares with,
  Section 5.2.2).

The GPU tests hold the HIP path's ASYNC results to within 1e-3 of these
(the stated quality bar for the asynchronous mode).  A fingerprint of the
edge list and of the batches is stored too, so the tests can check that
they regenerate the same inputs.

    python tests/golden/make_async_golden.py rmat22
    python tests/golden/make_async_golden.py chunglu20m

The Chung-Lu workload needs about 35 GB of host memory and tens of minutes.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# The batch sequences the GPU side runs (the benchmark's DF steps): sizes
# as fractions of |E|, number of batches, seed of the pools.
WORKLOADS = {
    "rmat22": {"fracs": [1e-7, 1e-6, 1e-5, 1e-4, 1e-3], "count": 25, "seed": 4242},
    "chunglu20m": {"fracs": [1e-5, 1e-4], "count": 24, "seed": 4343},
}


def edges_of(name):
    from paper_2404_19634_amd import workloads as W
    if name == "rmat22":
        return W.config2_rmat()
    if name == "chunglu20m":
        return W.config3_chung_lu(device="cpu")
    raise KeyError(name)


def batches_of(name, e):
    from paper_2404_19634_amd import workloads as W
    spec = WORKLOADS[name]
    sizes = [W.batch_size(f, e.m) for f in spec["fracs"]]
    return sizes, W.batch_sequence(e, sizes, spec["count"], spec["seed"])


def fingerprint(arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:32]


def edges_fingerprint(e) -> str:
    return fingerprint([np.array([e.n], dtype=np.int64), e.u, e.v, e.w])


def batches_fingerprint(batches) -> str:
    return fingerprint([a for b in batches for a in (b.del_u, b.del_v, b.del_w, b.ins_u, b.ins_v, b.ins_w)])


def path_of(name) -> str:
    return os.path.join(HERE, f"async_quality_{name}.json")


def load(name) -> dict:
    with open(path_of(name)) as f:
        return json.load(f)


def main(name):
    import oracle
    t0 = time.time()
    e = edges_of(name)
    sizes, batches = batches_of(name, e)
    print(f"{name}: n={e.n} m={e.m} batches {len(batches)} ({time.time() - t0:.0f} s)", flush=True)
    G = oracle.Graph.from_edges(e)
    C, K, S, st = G.louvain("static", mode="async")
    q0 = G.modularity(C)
    print(f"static ASYNC Q={q0:.9f} passes {st['passes']} iterations {st['iterations']} "
          f"({time.time() - t0:.0f} s)", flush=True)
    state = (C, K, S)
    for k, b in enumerate(batches):
        assert G.apply_batch(b) == 0
        C, K, S, _ = G.louvain("df", batch=b, state=state, mode="async")
        state = (C, K, S)
    q_df = G.modularity(state[0])
    print(f"DF chain Q={q_df:.9f} ({time.time() - t0:.0f} s)", flush=True)
    Cf, _, _, stf = G.louvain("static", mode="async")
    q_final = G.modularity(Cf)
    print(f"static on the final graph Q={q_final:.9f} ({time.time() - t0:.0f} s)", flush=True)
    out = {
        "workload": name,
        "how": "tests/golden/make_async_golden.py (sequential oracle only)",
        "cite": "Alg. 1 (DF), Alg. 4 (Louvain driver), Alg. 5 (local moving, ascending id order), Eq. 1; "
                "random batches per Section 5.1.4; default parameters per Section 5.1.2",
        "vertices": int(e.n), "undirected_edges": int(e.m),
        "edges_sha256_32": edges_fingerprint(e),
        "batch_sizes": [int(s) for s in sizes], "batch_count": len(batches), "batch_seed": WORKLOADS[name]["seed"],
        "batches_sha256_32": batches_fingerprint(batches),
        "static_async": {"modularity": q0, "passes": st["passes"], "iterations": st["iterations"]},
        "df_chain_async": {"modularity": q_df},
        "static_async_final_graph": {"modularity": q_final, "passes": stf["passes"],
                                     "iterations": stf["iterations"]},
    }
    with open(path_of(name), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path_of(name), flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "rmat22")
