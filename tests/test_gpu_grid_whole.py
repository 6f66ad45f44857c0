"""Small grids held whole by one workgroup (N <= 1024 nodes, L <= 8), every
requested step in one launch: parity with the FP64 oracle (one step from an
identical state, and end to end), agreement with the tile kernels, and the
library's choice of the path."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import cases  # noqa: E402
import oracle as O  # noqa: E402
from paper_1511_06103_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WHOLE_STEPS = 256


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_state(s):
    torch.cuda.synchronize()
    return s.current_state().detach().cpu().numpy().astype(np.float64)


def random_state(rng, inst):
    x = rng.standard_normal(inst.unary.shape) * 1.5
    return (x - np.log(np.exp(x).sum(1, keepdims=True))).astype(np.float32)


CASES = [
    ("c1_32x32_L2_potts_grid4", lambda: synth.workload_c1()),
    ("1x1_L3", lambda: synth.grid_theta_random(41, 1, 1, 3, synth.GRID8, iters=10)),
    ("1x1000_L2_potts", lambda: synth.grid_potts_normal(42, 1, 2, synth.GRID8, w=0.7, width=1000, iters=10)),
    ("32x32_L8_theta_grid8", lambda: synth.grid_theta_random(43, 32, 32, 8, synth.GRID8, iters=10)),
    ("17x23_L5_theta_grid4_batch3", lambda: synth.grid_theta_random(44, 17, 23, 5, synth.GRID4, batch=3, iters=10)),
    ("9x70_L1", lambda: synth.grid_theta_random(45, 9, 70, 1, synth.GRID8, iters=10)),
    ("31x33_L4_potts_grid8", lambda: synth.grid_potts_normal(46, 31, 4, synth.GRID8, w=0.9, width=33, iters=10)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[n for n, _ in CASES])
def test_whole_grid_one_step_and_end_to_end(name, make):
    inst = make()
    B = inst.batch
    start = random_state(np.random.default_rng(7), inst)
    st = torch.empty((2,) + inst.unary.shape, dtype=torch.float32, device="cuda:0")
    st[0].copy_(torch.from_numpy(start))
    s = cases.gpu_solver(inst, init="state", state=st)
    assert s.steps_per_launch == WHOLE_STEPS
    s.step(1)
    g = gpu_state(s)
    for b in range(B):
        ref = O.prox_step(start[b].astype(np.float64), cases.oracle_model(inst, b), inst.alpha)
        assert cases.max_dq(g[b], ref) <= 1e-6, b
    s = cases.gpu_solver(inst)
    s.step(10)               # one launch of ten steps
    assert s.iteration == 10
    g = gpu_state(s)
    for b in range(B):
        ref = O.solve(cases.oracle_model(inst, b), inst.alpha, 10)[-1]
        assert cases.max_dq(g[b], ref) <= 1e-5, b


@pytest.mark.parametrize("precision,tol", [("f32", 2e-6), ("bf16", 2e-3), ("f16", 2e-4)])
def test_whole_grid_matches_tile_kernels(precision, tol):
    inst = synth.grid_theta_random(47, 32, 32, 6, synth.GRID8, iters=20)
    a = cases.gpu_solver(inst, precision=precision)
    b = cases.gpu_solver(inst, precision=precision, steps_per_launch=1)
    assert a.steps_per_launch == WHOLE_STEPS and b.steps_per_launch == 1
    a.step(7)
    a.step(13)
    b.step(20)
    assert cases.max_dq(gpu_state(a)[0], gpu_state(b)[0]) <= tol


def test_whole_grid_only_when_it_fits_and_is_not_overridden():
    small = synth.grid_theta_random(48, 32, 32, 8, synth.GRID8)
    assert cases.gpu_solver(small, steps_per_launch=3).steps_per_launch == 3
    wide = synth.grid_theta_random(49, 32, 33, 2, synth.GRID8)        # 1056 nodes
    assert cases.gpu_solver(wide).steps_per_launch != WHOLE_STEPS
    many = synth.grid_theta_random(50, 16, 16, 9, synth.GRID8)        # L = 9
    assert cases.gpu_solver(many).steps_per_launch != WHOLE_STEPS


def test_whole_grid_long_solve_spans_launches():
    """600 steps: three launches (256, 256, 88), the iterate carried in the
    state buffers between them, against the oracle."""
    inst = synth.grid_potts_normal(51, 12, 3, synth.GRID4, w=0.3, alpha=0.4, width=20, iters=600)
    s = cases.gpu_solver(inst)
    q = torch.empty_like(s.unary)
    s.solve(600, q)
    torch.cuda.synchronize()
    ref = O.solve(cases.oracle_model(inst), inst.alpha, 600)[-1]
    assert cases.max_dq(np.log(q.cpu().numpy()[0].astype(np.float64)), ref) <= 1e-5


FUSED = [
    ("L2_unary_50", lambda: synth.grid_potts_normal(52, 32, 2, synth.GRID4, w=1.0), "unary", 50),
    ("L3_unary_300", lambda: synth.grid_theta_random(53, 20, 30, 3, synth.GRID8), "unary", 300),
    ("L5_unary_batch2", lambda: synth.grid_theta_random(54, 12, 40, 5, synth.GRID8, batch=2), "unary", 37),
    ("L8_uniform", lambda: synth.grid_theta_random(55, 31, 32, 8, synth.GRID4), "uniform", 20),
    ("L6_state", lambda: synth.grid_theta_random(56, 16, 16, 6, synth.GRID8), "state", 12),
]


@pytest.mark.parametrize("name,make,init,iters", FUSED, ids=[f[0] for f in FUSED])
def test_whole_grid_solve_in_one_launch_equals_separate_kernels(name, make, init, iters):
    """mf_solve on a small grid runs the initialisation, the steps and the
    write-out of q inside the whole-grid launches; the state and q equal,
    bitwise, the initialisation kernel, the steps and the write-out kernel
    launched one by one (solve(0), step(n), marginals())."""
    inst = make()
    if init == "state":
        start = torch.from_numpy(random_state(np.random.default_rng(8), inst)).to("cuda:0")
        sts = []
        for _ in range(2):
            st = torch.empty((2,) + inst.unary.shape, dtype=torch.float32, device="cuda:0")
            st[0].copy_(start)
            sts.append(st)
    a = cases.gpu_solver(inst, init=init, **({"state": sts[0]} if init == "state" else {}))
    b = cases.gpu_solver(inst, init=init, **({"state": sts[1]} if init == "state" else {}))
    qa = torch.empty_like(a.unary)
    a.solve(iters, qa)
    b.solve(0)
    b.step(iters)
    qb = b.marginals()
    torch.cuda.synchronize()
    assert a.iteration == b.iteration == iters
    assert torch.equal(a.current_state(), b.current_state())
    assert torch.equal(qa, qb)
    a.check()


def test_whole_grid_solve_reports_a_non_finite_unary():
    """The initialisation inside the one-launch solve flags a non-finite
    unary as the initialisation kernel does: the report from creating the
    handle is taken first (a check clears it), so the second one can only
    come from the solve."""
    from paper_1511_06103_amd import mf
    inst = synth.grid_potts_normal(57, 8, 2, synth.GRID4)
    inst.unary = inst.unary.copy()
    inst.unary[0, 1, 5] = np.inf
    s = cases.gpu_solver(inst)
    for _ in range(2):
        with pytest.raises(mf.MFError) as e:
            s.check()
        assert e.value.status == mf.MF_ENONFINITE
        s.solve(4)
