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
    # log q, u, log q' (4 B each), the node-major q written and gathered, and
    # the graph: row_ptr, col and the weights
    graph = 4 * 101 + 8 * c.col.size
    assert bench.algorithmic_bytes(c, 1) == 100 * 21 * (12 + 8) + graph
    assert bench.algorithmic_bytes(c, 1, "bf16") == 100 * 21 * (12 + 4) + graph
    g = synth.grid_as_csr(synth.grid_theta_random(1, 6, 9, 5, synth.GRID8))
    assert bench.algorithmic_bytes(g, 1) == 54 * 5 * 20 + 4 * 55 + 4 * g.col.size     # unweighted
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


def test_counters_match_the_solver_options(tmp_path, monkeypatch):
    """An entry taken with solver options (one lane per node on the grid as
    CSR) serves only runs with those options, and every committed entry
    belongs to a workload bench.py runs, under its workload name."""
    kind = "csr"
    entry = {"workload": "w", "steps_per_launch": 1, "options": {"csr_lanes": 1},
             "kernel_source_sha256_16": bench.source_hash(kind), "hbm_bytes_per_launch": 99}
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"entries": [entry]}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.load_counters("w", 1, kind, "f32", {"csr_lanes": 1})["hbm_bytes_per_launch"] == 99
    assert bench.load_counters("w", 1, kind, "f32", {}) is None
    assert bench.load_counters("w", 1, kind, "f32", {"csr_lanes": 2}) is None
    with open(os.path.join(ROOT, "profiles", "step_kernel_traffic.json")) as f:
        committed = json.load(f)["entries"]
    for e in committed:
        assert e["workload"] in bench.WORKLOADS, e["workload"]
        opts = bench.SOLVER_OPTIONS.get((e["workload"], e.get("precision", "f32")), {})
        assert e.get("options", {}) == opts, (e["workload"], e.get("precision"))


@pytest.mark.parametrize("kind", sorted(bench.KERNEL_SOURCES))
def test_source_hash_covers_existing_files(kind):
    h = bench.source_hash(kind)
    assert len(h) == 16 and int(h, 16) >= 0


def test_roofline_bound_follows_the_counters():
    g = synth.grid_theta_random(1, 32, 32, 21, synth.GRID8)
    algo = bench.algorithmic_bytes(g, 4)
    t = 1e-5
    # no counters: HBM, with the effective figure
    r = bench.roofline_object(g, 4, "f32", t, 10, "k", None)
    assert r["bound"] == "hbm" and r["traffic"] is None
    assert abs(r["frac"] - algo / t / 1e9 / bench.HBM_PEAK_GBS) < 1e-4
    # the state stays in the cache and the VALU count is known: VALU issue
    c = {"hbm_bytes_per_launch": algo // 4, "sq_insts_valu_per_launch": 3.0e6, "rocprof_avg_us": 11.0}
    r = bench.roofline_object(g, 4, "f32", t, 10, "k", c)
    assert r["bound"] == "valu_issue" and r["unit"].startswith("G wave64")
    assert abs(r["frac"] - 3.0e6 / t / 1e9 / bench.VALU_ISSUE_PEAK_G) < 1e-4
    assert r["hbm"]["traffic_over_algorithmic"] == 0.25
    assert abs(r["rocprof"]["frac"] - 3.0e6 / 11e-6 / 1e9 / bench.VALU_ISSUE_PEAK_G) < 1e-4
    # bytes moved close to the algorithmic ones: HBM, whatever the VALU count
    c = {"hbm_bytes_per_launch": algo, "sq_insts_valu_per_launch": 3.0e6}
    assert bench.roofline_object(g, 4, "f32", t, 10, "k", c)["bound"] == "hbm"


def test_persistent_step_count_matches_the_header():
    import os
    import re
    from paper_1511_06103_amd import mf
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mf.h")).read()
    v = int(re.search(r"#define MF_PERSIST_STEPS_PER_LAUNCH (\d+)", text).group(1))
    assert v == mf.MF_PERSIST_STEPS_PER_LAUNCH == bench.PERSIST_STEPS


def test_persistent_kernel_reports_the_effective_fraction():
    """The persistent grid kernel is bound by the halo exchange: the line keeps
    the effective HBM fraction as frac and says why, counters or not."""
    g = synth.grid_theta_random(1, 32, 32, 21, synth.GRID8)
    algo = bench.algorithmic_bytes(g, 100)
    t = 3e-4
    c = {"hbm_bytes_per_launch": algo // 50, "sq_insts_valu_per_launch": 5.0e7, "rocprof_avg_us": 310.0}
    r = bench.roofline_object(g, 100, "f32", t, 10, "mf::persist::persist_kernel", c)
    assert r["bound"] == "hbm" and "exchange" in r["note"]
    assert abs(r["frac"] - algo / t / 1e9 / bench.HBM_PEAK_GBS) < 1e-4
    assert "valu" in r and abs(r["rocprof"]["frac"] - algo / 310e-6 / 1e9 / bench.HBM_PEAK_GBS) < 1e-4
    assert bench.step_kernel_name(g, 100, bench.PERSIST_STEPS) == "mf::persist::persist_kernel"
    assert bench.source_kind(g, bench.PERSIST_STEPS) == "persist" and bench.source_kind(g, 4) == "grid"


def test_many_label_grids_report_the_matrix_cores():
    g = synth.grid_theta_random(1, 4, 100, 128, synth.GRID8)
    fl = bench.mfma_flops_per_launch(g, 1, "f32")
    nodes = 4 * 128                      # the width rounded up to 64-node tiles
    assert fl["issued"] == 2.0 * 128 * 128 * nodes and fl["algorithmic"] == 2.0 * 128 * 128 * 400
    assert bench.mfma_flops_per_launch(g, 1, "bf16")["issued"] == 3 * fl["issued"]
    r = bench.roofline_object(g, 1, "f32", 1e-6, 10, "k", None)
    assert "mfma" in r and r["mfma"]["peak"] == bench.MFMA_F32_PEAK_TFLOPS
    assert r["bound"] in ("hbm", "mfma")
    assert bench.source_kind(g) == "large"
    assert bench.mfma_flops_per_launch(synth.workload_c1(), 1, "f32") is None


def test_parity_check_against_the_oracle():
    import numpy as np
    import oracle as O
    inst = synth.grid_theta_random(3, 12, 9, 5, synth.GRID8, iters=7)
    model = O.grid_model(inst.unary[0].astype(np.float64), 12, 9, 8, theta=inst.theta.astype(np.float64))
    q = np.exp(O.solve(model, inst.alpha, 7)[-1])[None]
    p = bench.parity_check(inst, q, "f32")
    assert p["max_abs_dq"] < 1e-12 and p["passed"] and p["argmax_agreement"] == 1.0
    assert 0 < p["fp32_floor_max_abs_dq"] < 1e-5
    q2 = q.copy()
    q2[0, :, 0] = q2[0, ::-1, 0]
    assert not bench.parity_check(inst, q2, "f32")["passed"]
    assert bench.parity_check(inst, q, "bf16")["passed"] is None
