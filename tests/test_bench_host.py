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
    measured bytes sit at or above the algorithmic 38 values per node (19 read,
    19 written) by less than 10%."""
    table = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    width = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
    assert set(table) == set(width)
    for st, t in table.items():
        total = (t["fetch_kib_raw"] * t["fetch_scale"] + t["write_kib_raw"] * t["write_scale"]) * 1024
        assert abs(total / t["bytes_per_launch"] - 1) < 1e-4, st
        assert abs(t["bytes_per_launch"] / t["nodes"] - t["bytes_per_node"]) < 0.01, st
        algorithmic = 38 * width[st]
        assert algorithmic <= t["bytes_per_node"] < 1.1 * algorithmic, st
        assert len(t["kernel_digest"]) == 16, st
