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
