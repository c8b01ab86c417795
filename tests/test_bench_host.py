"""Host-side checks of the benchmark driver (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    """The step runs on one GPU; asking for more ends before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "asked for 2" in r.stderr
    assert r.stdout == ""


def test_committed_counter_table_is_consistent():
    """profiles/traffic.json: per storage, the scaled counters add up to the
    stated bytes (the table rounds the scales to four decimals), and the
    measured bytes sit at or above the algorithmic bytes per node (the
    lattice's bytes read once and written once) by less than 10%."""
    table = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    # bytes one lattice holds per node: 19 populations, the FP32-rest kinds
    # with the rest population in FP32
    per_node = {"f64": 152, "f32": 76, "f16s": 38, "bf16s": 38, "f16m": 40, "bf16m": 40}
    assert table and set(table) <= set(per_node)
    for st, t in table.items():
        total = (t["fetch_kib_raw"] * t["fetch_scale"] + t["write_kib_raw"] * t["write_scale"]) * 1024
        assert abs(total / t["bytes_per_launch"] - 1) < 1e-4, st
        assert abs(t["bytes_per_launch"] / t["nodes"] - t["bytes_per_node"]) < 0.01, st
        algorithmic = 2 * per_node[st]
        assert algorithmic <= t["bytes_per_node"] < 1.1 * algorithmic, st
        assert len(t["kernel_digest"]) == 16, st
