"""Continuous-batching solve server over the HIP library.

Requests carry a grid problem (unaries, Theta, size, alpha, iterations).
They arrive over time, wait in a FIFO queue and are admitted while their
device-memory footprint fits a budget (optionally at most a fixed number
per scheduler tick, so that stepping starts while later requests are still
uploading).
Every tick advances all admitted problems by one proximal step (optionally
a few) through ``mf_step_many``: one launch per label count and group of up
to 48 problems, tiles of every problem of the group in the same launch.  A problem that
reaches its iteration count has q written out and copied to pinned host
memory asynchronously; its memory returns to the budget when the copy has
landed, and queued requests are admitted at the next tick.  Work of newly
admitted requests therefore overlaps on the device with the work of requests
already in flight.

The per-problem arithmetic is exactly that of a solo solve at one step per
launch (the batched kernel shares the tile body), so every result equals,
bitwise, the result of solving the same request alone.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import mf


@dataclass
class SolveRequest:
    """One grid problem: unary [1, L, N] and theta [L, L] FP32 on the host."""
    rid: int
    arrival_s: float
    unary: np.ndarray
    theta: np.ndarray
    height: int
    width: int
    alpha: float = 0.5
    iters: int = 100
    connectivity: int = 8
    # filled in by the server
    status: str = "pending"          # pending | queued | running | done | rejected
    error: str = ""
    q: Optional[np.ndarray] = None   # [1, L, N] result
    t_admit: float = float("nan")
    t_done: float = float("nan")

    @property
    def n_labels(self):
        return self.unary.shape[1]

    @property
    def n_nodes(self):
        return self.unary.shape[2]

    @property
    def latency_s(self):
        return self.t_done - self.arrival_s

    @property
    def updates(self):
        return self.n_nodes * self.n_labels * self.iters


def footprint_bytes(req: SolveRequest) -> int:
    """Device bytes a request holds while admitted: state (2 copies), unary,
    q output, theta and the library workspace (bounded by a small margin)."""
    LN = req.n_labels * req.n_nodes
    return 4 * (2 * LN + LN + LN + req.n_labels * req.n_labels) + 8 * (req.n_nodes // 256 + 64) + 4096


@dataclass
class _Slot:
    req: SolveRequest
    solver: mf.MeanField
    nbytes: int
    q_dev: Optional[torch.Tensor] = None
    q_host: Optional[torch.Tensor] = None
    done_event: Optional[torch.cuda.Event] = None


@dataclass
class ServerStats:
    n_done: int = 0
    n_rejected: int = 0
    makespan_s: float = 0.0
    updates: int = 0
    latencies_s: List[float] = field(default_factory=list)
    max_active: int = 0
    max_used_bytes: int = 0
    ticks: int = 0
    kernel_s: float = 0.0     # device time of the stepping launches (HIP events around each tick)

    def summary(self):
        lat = np.array(self.latencies_s) if self.latencies_s else np.array([np.nan])
        return {"requests_done": self.n_done, "requests_rejected": self.n_rejected,
                "makespan_s": self.makespan_s,
                "throughput_updates_per_s": self.updates / self.makespan_s if self.makespan_s > 0 else 0.0,
                "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                "max_active": self.max_active, "max_used_bytes": self.max_used_bytes, "ticks": self.ticks,
                "step_kernels_s": self.kernel_s,
                "staging_and_host_s": self.makespan_s - self.kernel_s}


class Server:
    """Admission by device-memory footprint, one batched launch per tick."""

    def __init__(self, budget_bytes: int = 64 << 30, precision: str = "bf16", device: str = "cuda:0",
                 max_ahead_ticks: int = 2, admit_per_tick: int = 0, steps_per_tick: int = 1):
        self.budget = int(budget_bytes)
        self.precision = precision
        self.device = torch.device(device)
        self.max_ahead = max_ahead_ticks
        # admissions per tick (0: all that fit), so that stepping starts while
        # later requests are still uploading
        self.admit_per_tick = int(admit_per_tick)
        # steps per tick: every active problem advances by up to this many
        # steps, each stopping at its own iteration count
        self.steps_per_tick = max(1, int(steps_per_tick))
        self.used = 0
        self.queue: List[SolveRequest] = []
        self.active: List[_Slot] = []
        self.draining: List[_Slot] = []
        self.stats = ServerStats()

    # -- admission --------------------------------------------------------
    def submit(self, req: SolveRequest):
        u, th = req.unary, req.theta
        if (u.ndim != 3 or u.shape[0] != 1 or th.shape != (u.shape[1], u.shape[1])
                or req.height * req.width != u.shape[2] or not (0.0 < req.alpha <= 1.0) or req.iters < 0
                or req.connectivity not in (4, 8)):
            return self._reject(req, "malformed request")
        if not 1 <= req.n_labels <= mf.MF_MAX_LABELS:
            return self._reject(req, f"label count outside 1..{mf.MF_MAX_LABELS}")
        if req.n_labels * req.n_nodes >= mf.MF_MAX_LABEL_NODES:
            return self._reject(req, "n_labels * n_nodes at or above the library's per-problem limit")
        if not (np.isfinite(u).all() and np.isfinite(th).all()):
            return self._reject(req, "non-finite unary or theta")
        if footprint_bytes(req) > self.budget:
            return self._reject(req, "request larger than the whole device-memory budget")
        req.status = "queued"
        self.queue.append(req)

    def _reject(self, req, why):
        req.status, req.error = "rejected", why
        self.stats.n_rejected += 1

    def _admit(self, now):
        n = 0
        while self.queue and self.used + footprint_bytes(self.queue[0]) <= self.budget:
            if self.admit_per_tick and n >= self.admit_per_tick:
                break
            n += 1
            req = self.queue.pop(0)
            nb = footprint_bytes(req)
            u = torch.from_numpy(req.unary).pin_memory().to(self.device, non_blocking=True)
            th = torch.from_numpy(req.theta).pin_memory().to(self.device, non_blocking=True)
            graph = "grid4" if req.connectivity == 4 else "grid8"
            try:
                s = mf.MeanField(u, graph, height=req.height, width=req.width, theta=th, alpha=req.alpha,
                                 precision=self.precision, steps_per_launch=1)
            except mf.MFError as e:
                # refused by the library: this request alone fails, the budget is not charged
                self._reject(req, str(e))
                continue
            self.used += nb
            self.stats.max_used_bytes = max(self.stats.max_used_bytes, self.used)
            req.status, req.t_admit = "running", now
            slot = _Slot(req, s, nb)
            if req.iters == 0:
                self._finish(slot)
            else:
                self.active.append(slot)

    # -- completion -------------------------------------------------------
    def _finish(self, slot: _Slot):
        B, L, N = slot.solver.shape
        # q = exp(log q) written by the library, then an asynchronous copy to pinned memory
        slot.q_dev = slot.solver.marginals()
        slot.q_host = torch.empty((B, L, N), dtype=torch.float32, pin_memory=True)
        slot.q_host.copy_(slot.q_dev, non_blocking=True)
        slot.done_event = torch.cuda.Event()
        slot.done_event.record()
        self.draining.append(slot)

    def _poll(self, now):
        still = []
        for slot in self.draining:
            if slot.done_event.query():
                req = slot.req
                req.q = slot.q_host.numpy()
                req.t_done = now
                req.status = "done"
                self.stats.n_done += 1
                self.stats.updates += req.updates
                self.stats.latencies_s.append(req.latency_s)
                self.used -= slot.nbytes
                slot.solver.close()
            else:
                still.append(slot)
        self.draining = still

    # -- the loop ---------------------------------------------------------
    def run(self, requests: List[SolveRequest], realtime: bool = True) -> ServerStats:
        """Serve requests arriving at their arrival_s offsets (realtime) or all at once."""
        pending = sorted(requests, key=lambda r: r.arrival_s)
        t0 = time.perf_counter()
        tick_events: List[torch.cuda.Event] = []
        spans: List[tuple] = []
        i = 0
        while i < len(pending) or self.queue or self.active or self.draining:
            now = time.perf_counter() - t0
            while i < len(pending) and (not realtime or pending[i].arrival_s <= now):
                if not realtime:
                    pending[i].arrival_s = 0.0
                self.submit(pending[i])
                i += 1
            self._admit(now)
            if self.active:
                # each problem advances at its own pace: up to steps_per_tick, never past its count
                ks = [min(self.steps_per_tick, s.req.iters - s.solver.iteration) for s in self.active]
                t_a = torch.cuda.Event(enable_timing=True)
                t_a.record()
                mf.step_many([s.solver for s in self.active], ks)
                self.stats.ticks += 1
                ev = torch.cuda.Event(enable_timing=True)
                ev.record()
                spans.append((t_a, ev))
                tick_events.append(ev)
                still = []
                for s in self.active:
                    if s.solver.iteration >= s.req.iters:
                        self._finish(s)
                    else:
                        still.append(s)
                self.active = still
                self.stats.max_active = max(self.stats.max_active, len(self.active))
                # keep the host at most a few ticks ahead of the device
                if len(tick_events) > self.max_ahead:
                    tick_events.pop(0).synchronize()
            self._poll(time.perf_counter() - t0)
            if not self.active and not self.queue and self.draining:
                time.sleep(0.0002)
            elif not self.active and not self.queue and i < len(pending):
                time.sleep(max(0.0, min(0.001, pending[i].arrival_s - (time.perf_counter() - t0))))
        self.stats.makespan_s = time.perf_counter() - t0 - (min(r.arrival_s for r in requests) if requests else 0)
        torch.cuda.synchronize()
        self.stats.kernel_s = sum(a.elapsed_time(b) for a, b in spans) * 1e-3
        return self.stats


def requests_from_trace(trace, alpha=0.5, iters=100):
    """Build SolveRequests from synth.serving_trace (inputs drawn per request seed)."""
    from . import synth
    out = []
    for r in trace:
        inst = synth.serving_request_instance(r, alpha=alpha, iters=iters)
        out.append(SolveRequest(r.index, r.arrival_s, inst.unary, inst.theta, inst.height, inst.width,
                                inst.alpha, iters))
    return out


def solve_alone(req: SolveRequest, precision="bf16", device="cuda:0", steps_per_launch=1, timing=None) -> np.ndarray:
    """The plain path: one request, its own solver, one solve.  With
    steps_per_launch = 1 every step is its own launch (the per-tile
    arithmetic of the batched kernel, so the results are bitwise the
    server's); 0 leaves the launch shape to the library (fused steps on
    small grids).  ``timing`` (a list) collects the device time of the solve."""
    dev = torch.device(device)
    u = torch.from_numpy(req.unary).to(dev)
    th = torch.from_numpy(req.theta).to(dev)
    graph = "grid4" if req.connectivity == 4 else "grid8"
    s = mf.MeanField(u, graph, height=req.height, width=req.width, theta=th, alpha=req.alpha,
                     precision=precision, steps_per_launch=steps_per_launch)
    q = torch.empty_like(u)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    s.solve(req.iters, q)
    b.record()
    out = q.cpu().numpy()     # synchronises
    if timing is not None:
        timing.append(a.elapsed_time(b) * 1e-3)
    s.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="Serve the synthetic request stream and report latency/throughput.")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-mib", type=int, default=64 * 1024)
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--saturation", action="store_true", help="also replay all requests at t = 0 and "
                    "compare with solving them one by one")
    ap.add_argument("--admit-per-tick", type=int, default=0, help="admissions per scheduler tick (0: all that fit)")
    ap.add_argument("--steps-per-tick", type=int, default=1)
    args = ap.parse_args(argv)
    sched = dict(admit_per_tick=args.admit_per_tick, steps_per_tick=args.steps_per_tick)
    from . import synth
    trace = synth.serving_trace(4, args.n, args.rate)
    print(f"generating {args.n} requests", file=sys.stderr, flush=True)
    reqs = requests_from_trace(trace, iters=args.iters)
    mf.lib()
    # warm-up: one small request through both paths
    warm = requests_from_trace(synth.serving_trace(9, 2, 1000.0), iters=5)
    Server(precision=args.precision).run(warm, realtime=False)
    solve_alone(warm[0], args.precision)
    out = {"workload": f"serving: {args.n} requests, Poisson {args.rate}/s, sides 64-512, L in {{2, 21}}, "
                       f"{args.iters} iterations, {args.precision} messages"}
    srv = Server(budget_bytes=args.budget_mib << 20, precision=args.precision, **sched)
    st = srv.run(reqs, realtime=True)
    out["poisson"] = st.summary()
    print(json.dumps(out["poisson"]), file=sys.stderr, flush=True)
    if args.saturation:
        reqs2 = requests_from_trace(trace, iters=args.iters)
        srv2 = Server(budget_bytes=args.budget_mib << 20, precision=args.precision, **sched)
        out["saturation_batched"] = srv2.run(reqs2, realtime=False).summary()
        print(json.dumps(out["saturation_batched"]), file=sys.stderr, flush=True)
        tot = sum(r.updates for r in reqs2)
        for name, spl in (("saturation_alone_one_step_per_launch", 1), ("saturation_alone_library_default", 0)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            dev_s = []
            for r in reqs2:
                solve_alone(r, args.precision, steps_per_launch=spl, timing=dev_s)
            dt = time.perf_counter() - t
            out[name] = {"makespan_s": dt, "throughput_updates_per_s": tot / dt, "solve_kernels_s": sum(dev_s),
                         "staging_and_host_s": dt - sum(dev_s)}
            print(json.dumps({name: out[name]}), file=sys.stderr, flush=True)
        bt = out["saturation_batched"]["throughput_updates_per_s"]
        out["batched_over_alone_one_step_per_launch"] = bt / out["saturation_alone_one_step_per_launch"][
            "throughput_updates_per_s"]
        out["batched_over_alone_library_default"] = bt / out["saturation_alone_library_default"][
            "throughput_updates_per_s"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
