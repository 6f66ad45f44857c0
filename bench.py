#!/usr/bin/env python3
"""Benchmark of the parallel mean-field solve on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

One bench step is one whole solve of the hot path: initialisation from the
unaries, T parallel proximal steps (neighbour aggregation, compatibility
product, damped natural-parameter step, per-node normalisation) and the
write-out of q, on synthetic inputs already resident in HBM.  The default
workload is the 256 x 256, 8-connected, L = 21 grid with a random symmetric
Theta, alpha = 0.5 and T = 100 iterations (FP32).

Prints one JSON line: node-label updates/s = B * N * L * T * K / time, with
p50/p99 solve latency, the roofline of the dominant kernel (the step kernel
as the solve launches it, K fused steps per launch, timed over back-to-back
launches between HIP events on the stream it runs on) and the FP64 CPU oracle
timed on a bounded sample of the same workload.

Profiling helpers (single GPU):
    --mode kernel   only the dominant kernel, --launches times (for counters)
    --mode copy     a plain device-to-device copy of --copy-mib MiB (the
                    reference that scales FETCH_SIZE / WRITE_SIZE readings)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak, published
BYTES_PER_UPDATE = 12          # read log q (4) + read u (4) + write log q' (4)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
# sources of each workload's dominant kernel: a traffic measurement holds
# only while they are unchanged
KERNEL_SOURCES = {
    "grid": ("grid_temporal.h", "grid_lanes.h", "msg_codec.h"),
    "csr": ("csr_kernels.hip", "msg_codec.h"),
    "dense": ("dense_kernels.hip",),
}

WORKLOADS = {
    "grid256_L21_theta": lambda s: s.workload_c2(),
    "grid2048_L21_theta": lambda s: s.workload_big(),
    "grid32_L2_potts": lambda s: s.workload_c1(),
    "batch16_grid128_L21": lambda s: s.workload_c5(),
    # one step = the forward solve with checkpoints and the adjoint back to u and Theta
    "batch16_grid128_L21_adjoint": lambda s: s.workload_c5(),
    "dense4096_L21_cooc": lambda s: s.workload_c3(),
    "csr65536_L21": lambda s: s.csr_instance(8, 65536, 21, avg_degree=8, weighted=True, alpha=0.5, iters=100,
                                             name="csr65536_L21"),
}
ADJOINT_CKPT = 5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(kind="grid"):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1511_06103_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def source_kind(inst):
    return {2: "csr", 3: "dense"}.get(inst.graph, "grid")


def make_solver(inst, torch, mf, **extra):
    dev = torch.device("cuda:0")
    u = torch.from_numpy(inst.unary).to(dev)
    kw = dict(alpha=inst.alpha, **extra)
    if inst.theta is not None:
        kw["theta"] = torch.from_numpy(inst.theta).to(dev)
    else:
        kw["potts_w"] = inst.potts_w
    if inst.graph in (0, 1):
        graph = "grid4" if inst.graph == 0 else "grid8"
        return mf.MeanField(u, graph, height=inst.height, width=inst.width, **kw)
    if inst.graph == 2:
        return mf.MeanField(u, "csr", csr_row_ptr=torch.from_numpy(inst.row_ptr).to(dev),
                            csr_col=torch.from_numpy(inst.col).to(dev),
                            csr_w=None if inst.csr_w is None else torch.from_numpy(inst.csr_w).to(dev), **kw)
    K = mf.dense_kernel(torch.from_numpy(inst.features).to(dev))
    cooc = None if inst.cooc is None else torch.from_numpy(inst.cooc).to(dev)
    return mf.MeanField(u, "dense", dense_K=K, cooc=cooc, **kw)


def algorithmic_bytes(inst, k, precision="f32"):
    """Unique bytes one launch of the dominant kernel must move, k steps."""
    B, L, N = inst.unary.shape
    if inst.graph == 3:      # dense: the BF16 K stream (2 N^2 B) and the state (12 B per node-label)
        return k * B * (2 * N * N + BYTES_PER_UPDATE * N * L)
    if inst.graph == 2:      # CSR: log q, u, log q' and the node-major q copy written and gathered
        qb = 4 if precision == "f32" else 2
        return k * B * N * L * (BYTES_PER_UPDATE + 2 * qb)
    return BYTES_PER_UPDATE * B * N * L * k


def time_step_launches(solver, torch, launches):
    """Average duration of one launch of the step kernel as the solve runs it:
    each mf_step(K) with K = steps fused per launch is exactly one launch.
    The launches run back to back on the solver's stream between one pair of
    HIP events, as inside a solve, so the average includes no per-launch
    event overhead (only the inter-kernel gap of a queued stream)."""
    stream = solver.stream
    k = solver.steps_per_launch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    solver.step(k)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        a.record(stream)
        for _ in range(launches):
            solver.step(k)
        b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3 / launches, k


def step_kernel_name(inst, k):
    """The kernel one mf_step(k) launches for this workload (the library's
    dispatch rule: a grid of at most 1024 nodes and 8 labels whole in one
    workgroup, up to 256 steps per launch; otherwise fused steps for k > 1,
    Theta S on the matrix cores for a general Theta with 8 < L <= 32)."""
    L, N = inst.unary.shape[1], inst.unary.shape[2]
    if inst.graph == 3:      # one step is the MFMA kernel and the per-node kernel, back to back
        return "mf::dense_step_kernel + mf::dense_epilogue_kernel"
    if inst.graph == 2:
        return "mf::csr_step_kernel"
    if L <= 8 and N <= 1024 and k > 4:   # the fused kernels take at most 4 steps
        return "mf::whole_grid_kernel"
    if k == 1:
        return "mf::lanes::step_kernel"
    if inst.theta is not None and 8 < L <= 32:
        return "mf::temporal::multi_step_mfma_kernel"
    return "mf::temporal::multi_step_kernel"


METRIC = "node-label updates/s (N*L*iters/s) at oracle-matched marginals"
GRAPH_NAMES = {0: "grid4", 1: "grid8", 2: "csr", 3: "dense"}


def workload_config(inst, step):
    B, L, N = inst.unary.shape
    cfg = {"workload": inst.name, "graph": GRAPH_NAMES[inst.graph], "nodes": N, "labels": L, "batch": B,
           "compat": "theta" if inst.theta is not None else "potts", "alpha": inst.alpha, "iters": inst.iters,
           "step": step}
    if inst.graph in (0, 1):
        cfg.update(height=inst.height, width=inst.width, connectivity=4 if inst.graph == 0 else 8)
    if inst.graph == 2:
        cfg["edges"] = int(inst.col.size)
    if inst.graph == 3:
        cfg["cooc"] = inst.cooc is not None
    return cfg


def bench_adjoint(args, inst, torch, mf):
    """One step = the forward solve of T steps (one per launch, checkpoints every
    ADJOINT_CKPT) and the hand-written adjoint back to the unaries and Theta,
    through torch.autograd on the library (paper_1511_06103_amd.autograd)."""
    from paper_1511_06103_amd import autograd, synth
    B, L, N = inst.unary.shape
    T = inst.iters
    dev = torch.device("cuda:0")
    u = torch.from_numpy(inst.unary).to(dev).requires_grad_(True)
    th = torch.from_numpy(inst.theta).to(dev).requires_grad_(True)
    c = torch.from_numpy(synth.adjoint_loss_weights(55, inst.unary.shape)).to(dev)

    def step():
        u.grad = None
        th.grad = None
        ell = autograd.unrolled_mean_field(u, th, height=inst.height, width=inst.width, connectivity=8,
                                           alpha=inst.alpha, iters=T, ckpt_every=ADJOINT_CKPT)
        (torch.exp(ell) * c).sum().backward()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        lat.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in lat])
    value = B * N * L * T * args.steps / wall
    # forward 12 B, recompute 12 B and adjoint about 24 B per node-label-step
    algo = 48 * B * N * L * T
    per = wall / args.steps
    out = {"metric": METRIC, "value": value, "unit": "node-label updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": per * 1e3, "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": workload_config(inst, "forward solve with checkpoints + adjoint to u and Theta"),
           "roofline": {"bound": "hbm", "achieved": round(algo / per / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(algo / per / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "forward + backward (all kernels of one training step)",
                        "algorithmic_bytes_per_step": algo},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(inst, budget_s=8.0):
    """The FP64 oracle, untuned, timed on this host on a bounded sample: once
    with one thread, once with the BLAS pool at its default size (only the
    Theta S products use it; the rest of the oracle is single-threaded NumPy)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle as O
    b = 0
    th = None if inst.theta is None else inst.theta.astype(np.float64)
    pw = None if inst.theta is not None else inst.potts_w
    u = inst.unary[b].astype(np.float64)
    if inst.graph in (0, 1):
        model = O.grid_model(u, inst.height, inst.width, 4 if inst.graph == 0 else 8, theta=th, potts_w=pw)
    elif inst.graph == 2:
        model = O.csr_model(u, inst.row_ptr, inst.col, inst.csr_w, theta=th, potts_w=pw)
    else:
        K = O.round_to_bf16(O.gaussian_kernel(inst.features))
        cooc = None if inst.cooc is None else inst.cooc.astype(np.float64)
        model = O.dense_model(u, K, theta=th, potts_w=pw, cooc=cooc)
    L, N = model.unary.shape

    def timed():
        ell = O.init_state(model.unary)
        O.prox_step(ell, model, inst.alpha)     # build caches outside the timing
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            ell = O.prox_step(ell, model, inst.alpha)
            steps += 1
        el = time.perf_counter() - t0
        return steps, el

    with threadpool_limits(1):
        steps, el = timed()
    blas_threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    steps_all, el_all = timed()
    return {"value": steps * N * L / el, "unit": "node-label updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 proximal steps of one {inst.name} problem (N={N}, L={L}) "
                      f"({el:.1f} s, 1 thread)",
            "all_threads": {"value": steps_all * N * L / el_all, "blas_threads": blas_threads,
                            "sample": f"{steps_all} steps ({el_all:.1f} s)"},
            "host": {"cpu_count": os.cpu_count(), "cpu_model": cpu_model()}}


def load_traffic(workload, k, kind, precision="f32"):
    """HBM bytes per launch of the dominant kernel measured with rocprofv3
    counters (profiles/), or None when none was taken for this workload,
    launch depth and message precision or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    for e in t.get("entries", []):
        if (e.get("workload") == workload and e.get("steps_per_launch") == k
                and e.get("precision", "f32") == precision
                and e.get("kernel_source_sha256_16") == source_hash(kind)):
            return e.get("hbm_bytes_per_launch")
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid256_L21_theta", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="bench", choices=["bench", "kernel", "copy"])
    ap.add_argument("--launches", type=int, default=200)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", default="f32", choices=["f32", "bf16", "f16"],
                    help="neighbour-message precision (the state and the step stay FP32)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(a grid would shard into row slabs with one halo exchange per step).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_06103_amd import mf, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mf.lib()
    torch.cuda.set_device(0)

    if args.mode == "copy":
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for i in range(5):
            b.copy_(a)
            torch.cuda.synchronize()
            log(f"copy {i}: {args.copy_mib} MiB")
        return

    inst = WORKLOADS[args.workload](synth)
    B, L, N = inst.unary.shape
    T = inst.iters
    log(f"workload {inst.name}: B={B} N={N} L={L} T={T} alpha={inst.alpha}")
    if args.workload.endswith("_adjoint"):
        if args.precision != "f32":
            sys.exit("the adjoint runs with FP32 messages only")
        return bench_adjoint(args, inst, torch, mf)
    solver = make_solver(inst, torch, mf, precision=args.precision)
    q = torch.empty_like(solver.unary)

    if args.mode == "kernel":
        solver.solve(0)
        k = solver.steps_per_launch
        for i in range(args.launches):
            solver.step(k)
        torch.cuda.synchronize()
        log(f"kernel mode: {args.launches} launches of {k} steps done")
        return

    for i in range(args.warmup):
        solver.solve(T, q)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(solver.stream)
        solver.solve(T, q)
        ends[i].record(solver.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])    # ms
    ev_total = starts[0].elapsed_time(ends[-1]) * 1e-3
    total = wall
    updates = B * N * L * T * args.steps
    value = updates / total
    log(f"timed {args.steps} solves: wall {wall * 1e3:.3f} ms, HIP events {ev_total * 1e3:.3f} ms")

    # dominant kernel: one step-kernel launch = K steps over all B * N * L node-labels
    mean_d, k = time_step_launches(solver, torch, args.launches)
    algo = algorithmic_bytes(inst, k, args.precision)
    achieved = algo / mean_d / 1e9
    traffic = load_traffic(inst.name, k, source_kind(inst), args.precision)
    kname = step_kernel_name(inst, k)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "steps_per_launch": k, "launch_us_mean": round(mean_d * 1e6, 3),
                "algorithmic_bytes_per_launch": algo}
    log(f"{kname} (K={k}): {mean_d * 1e6:.2f} us mean per launch over {args.launches} back-to-back "
        f"launches -> {achieved:.0f} GB/s")
    if inst.graph == 3:
        # the K Q product on the BF16 matrix cores: what they issue (N rounded
        # up to 64, 32 label slots, one product per BF16 plane of q) and the
        # algorithmic 2 N^2 L, both per launch over the same launch time
        Np = -(-N // 64) * 64
        planes = {"f32": 3, "f16": 2, "bf16": 1}[args.precision]
        issued = 2.0 * B * Np * Np * 32 * planes / mean_d / 1e12
        algo_fl = 2.0 * B * N * N * L / mean_d / 1e12
        roofline["mfma"] = {"unit": "TFLOP/s", "peak": MFMA_BF16_PEAK_TFLOPS, "issued": round(issued, 1),
                            "issued_frac": round(issued / MFMA_BF16_PEAK_TFLOPS, 4),
                            "algorithmic": round(algo_fl, 1),
                            "algorithmic_frac": round(algo_fl / MFMA_BF16_PEAK_TFLOPS, 4)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst)
        log(f"cpu oracle: {cpu['value']:.3e} updates/s ({cpu['sample']})")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-label updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total * 1e3 / args.steps,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(workload_config(inst, "init + iters proximal steps + write q"), messages=args.precision),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
