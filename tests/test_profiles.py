"""The committed counter summaries under profiles/: every traffic file
parses, its HBM bytes are FETCH_SIZE + WRITE_SIZE per launch, its commands
run the committed bench.py, and the one the benchmark reads for the
20M-vertex Chung-Lu updates belongs to the current scan source (else the
bench line reports no traffic, and the file needs taking again)."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*_df.txt")))


def _kv(path):
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_there_are_traffic_files():
    assert FILES


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(p) for p in FILES])
def test_traffic_file_is_consistent(path):
    kv = _kv(path)
    m = re.match(r"traffic_move_all_(\d+)_(\d+)_(\w+)_df\.txt", os.path.basename(path))
    assert m, path
    assert kv["kernel"] == f"k_move_all<{m.group(1)}, {m.group(2)}>"
    f, w, h = (int(kv[k]) for k in ("FETCH_SIZE_bytes_per_launch", "WRITE_SIZE_bytes_per_launch",
                                     "hbm_bytes_per_launch"))
    assert f > 0 and w > 0 and h == f + w
    assert int(kv["algorithmic_bytes_per_launch"]) > 0
    assert re.fullmatch(r"[0-9a-f]{16}", kv["move_hip_sha256_16"])
    text = open(path).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    assert "python -u bench.py" in text


def test_headline_traffic_matches_the_scan_source():
    import sys
    sys.path.insert(0, ROOT)
    import bench
    t = bench.traffic_for("move_all", "k_move_all<512, 7>", "chunglu20m")
    assert t is not None, "profiles/traffic_move_all_512_7_chunglu20m_df.txt was taken on another move.hip"
    assert t == float(_kv(os.path.join(ROOT, "profiles", "traffic_move_all_512_7_chunglu20m_df.txt"))
                      ["hbm_bytes_per_launch"])
