"""Host logic of bench.py: the one-GPU contract, the algorithmic byte counts
behind the roofline figure, and the rule that a counter measurement is used
only while the dominant kernel's sources are unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1511_06103_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_launch():
    g = synth.grid_theta_random(1, 8, 8, 5, synth.GRID8)
    assert bench.algorithmic_bytes(g, 4) == 12 * 64 * 5 * 4
    c = synth.csr_instance(2, 100, 21, 4, True)
    # log q, u, log q' (4 B each) plus the node-major q written and gathered
    assert bench.algorithmic_bytes(c, 1) == 100 * 21 * (12 + 8)
    assert bench.algorithmic_bytes(c, 1, "bf16") == 100 * 21 * (12 + 4)
    d = synth.Instance(name="d", graph=synth.DENSE, n_labels=3, n_nodes=50,
                       unary=synth.grid_potts_normal(3, 1, 3, width=50).unary)
    assert bench.algorithmic_bytes(d, 1) == 2 * 50 * 50 + 12 * 50 * 3


def test_traffic_used_only_for_current_sources(tmp_path, monkeypatch):
    kind = "csr"
    entry = {"workload": "w", "steps_per_launch": 1, "kernel_source_sha256_16": bench.source_hash(kind),
             "hbm_bytes_per_launch": 1234}
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"entries": [entry]}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.load_traffic("w", 1, kind) == 1234
    assert bench.load_traffic("w", 2, kind) is None             # another launch depth
    assert bench.load_traffic("w", 1, kind, "bf16") is None     # taken with FP32 messages
    assert bench.load_traffic("other", 1, kind) is None
    entry["kernel_source_sha256_16"] = "0" * 16                # sources changed since
    p.write_text(json.dumps({"entries": [entry]}))
    assert bench.load_traffic("w", 1, kind) is None


@pytest.mark.parametrize("kind", sorted(bench.KERNEL_SOURCES))
def test_source_hash_covers_existing_files(kind):
    h = bench.source_hash(kind)
    assert len(h) == 16 and int(h, 16) >= 0
