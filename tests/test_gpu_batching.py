"""Continuous batching on the GPU: several problems of different sizes, label
counts and step sizes advanced by shared launches give bitwise the iterates
each gets when solved alone, and match the FP64 oracle."""
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def mix():
    out = []
    for k, (side, L) in enumerate([(64, 2), (97, 21), (130, 21), (64, 21), (77, 2), (200, 2)]):
        inst = synth.serving_request_instance(synth.Request(k, 0.0, side, L, 4000 + k), iters=100)
        if k % 3 == 1:
            inst.alpha = float(np.float32(0.3))
        out.append(inst)
    return out


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_mix_equals_alone_bitwise(precision):
    from paper_1511_06103_amd import mf
    insts = mix()
    alone = []
    for inst in insts:
        s = cases.gpu_solver(inst, precision=precision, steps_per_launch=1)
        s.step(9)
        torch.cuda.synchronize()
        alone.append(s.current_state().clone())
    solvers = [cases.gpu_solver(inst, precision=precision) for inst in insts]
    # staggered starts: solvers join the batch at different iterations
    mf.step_many(solvers[:2], 3)
    mf.step_many(solvers[:4], 2)
    mf.step_many(solvers, 4)
    mf.step_many(solvers[2:], 3)
    mf.step_many(solvers[4:], 2)
    torch.cuda.synchronize()
    for s, a in zip(solvers, alone):
        assert s.iteration == 9
        assert torch.equal(s.current_state(), a)


def test_mix_matches_oracle():
    from paper_1511_06103_amd import mf
    insts = mix()
    solvers = [cases.gpu_solver(inst) for inst in insts]
    mf.step_many(solvers, 6)
    torch.cuda.synchronize()
    for inst, s in zip(insts, solvers):
        ref = O.solve(cases.oracle_model(inst), inst.alpha, 6)[-1]
        assert cases.max_dq(s.current_state()[0].cpu().numpy(), ref) <= 1e-5


def test_more_problems_than_slots():
    from paper_1511_06103_amd import mf
    insts = [synth.grid_theta_random(900 + k, 16 + k, 20, 3, synth.GRID8) for k in range(60)]
    solvers = [cases.gpu_solver(i) for i in insts]
    mf.step_many(solvers, 2)
    torch.cuda.synchronize()
    for inst, s in zip(insts[::7], solvers[::7]):
        ref = O.solve(cases.oracle_model(inst), inst.alpha, 2)[-1]
        assert cases.max_dq(s.current_state()[0].cpu().numpy(), ref) <= 1e-5


def test_step_many_rejects_duplicates_and_dense():
    from paper_1511_06103_amd import mf
    inst = synth.grid_theta_random(1, 8, 8, 3, synth.GRID8)
    s = cases.gpu_solver(inst)
    with pytest.raises(mf.MFError):
        mf.step_many([s, s], 1)


def test_streaming_step_equals_batched_step_bitwise():
    """1024 x 1024, L = 21: the three arrays of a step (264 MB) exceed the
    last-level cache, so the solo step kernel reads the unaries and writes
    the new state with non-temporal hints; the batched kernel runs the same
    tile body with ordinary accesses.  The iterates must agree bitwise."""
    inst = synth.grid_theta_random(31, 1024, 1024, 21, synth.GRID8, iters=3)
    a = cases.gpu_solver(inst, steps_per_launch=1)
    b = cases.gpu_solver(inst, steps_per_launch=1)
    from paper_1511_06103_amd import mf
    for _ in range(3):
        a.step(1)
        mf.step_many([b], 1)
    torch.cuda.synchronize()
    assert torch.equal(a.current_state(), b.current_state())
    # and one step against the oracle on a sample of rows
    ell = O.init_state(inst.unary[0].astype(np.float64))
    s = cases.gpu_solver(inst, steps_per_launch=1)
    s.step(1)
    g = s.current_state()[0].cpu().numpy().astype(np.float64).reshape(21, 1024, 1024)
    th = inst.theta.astype(np.float64)
    for y0 in (0, 511, 1020):
        rows = slice(max(0, y0 - 1), min(1024, y0 + 5))
        sub_u = inst.unary[0].reshape(21, 1024, 1024)[:, rows, :].reshape(21, -1).astype(np.float64)
        sub_ell = ell.reshape(21, 1024, 1024)[:, rows, :].reshape(21, -1)
        h = sub_u.shape[1] // 1024
        ref = O.prox_step(sub_ell, O.grid_model(sub_u, h, 1024, 8, theta=th), inst.alpha).reshape(21, h, 1024)
        lo = 1 if y0 > 0 else 0
        hi = h - 1 if y0 + 5 < 1024 else h
        got = g[:, rows, :][:, lo:hi, :]
        assert cases.max_dq(got.reshape(21, -1), ref[:, lo:hi, :].reshape(21, -1)) <= 1e-6, y0


def test_step_many_per_handle_counts_bitwise():
    """One call advances three problems by 2, 5 and 9 steps (rounds in which
    the shorter ones drop out); each equals, bitwise, the same problem
    stepped alone at one step per launch, and the rest of the mix (a
    different label count and a zero count) moves as asked."""
    from paper_1511_06103_amd import mf
    insts = mix()[:5]
    counts = [2, 5, 9, 0, 4]
    alone = []
    for inst, k in zip(insts, counts):
        s = cases.gpu_solver(inst, steps_per_launch=1)
        s.step(k)
        torch.cuda.synchronize()
        alone.append(s.current_state().clone())
    solvers = [cases.gpu_solver(inst) for inst in insts]
    mf.step_many(solvers, counts)
    torch.cuda.synchronize()
    for s, a, k in zip(solvers, alone, counts):
        assert s.iteration == k
        assert torch.equal(s.current_state(), a)


def test_step_many_rejects_bad_counts_before_enqueueing():
    from paper_1511_06103_amd import mf
    insts = mix()[:2]
    solvers = [cases.gpu_solver(inst) for inst in insts]
    before = [s.current_state().clone() for s in solvers]
    with pytest.raises(mf.MFError) as e:
        mf.step_many(solvers, [3, -1])
    assert e.value.status == mf.MF_EINVAL
    torch.cuda.synchronize()
    for s, b in zip(solvers, before):
        assert s.iteration == 0 and torch.equal(s.current_state(), b)
