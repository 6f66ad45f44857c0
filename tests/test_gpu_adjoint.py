"""GPU adjoint of unrolled steps (autograd.Function over the library's reverse
pass) against the FP64 oracle's reverse pass, which is itself pinned to
central finite differences on the CPU (tests/test_oracle_pins.py).

Tolerance: max |grad_gpu - grad_oracle| <= 1e-4 * max |grad_oracle| (FP32
forward and reverse arithmetic over T = 10 steps).
"""
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


def run_autograd(inst, weights, ckpt_every=5, iters=None):
    from paper_1511_06103_amd.autograd import unrolled_mean_field
    dev = "cuda:0"
    iters = inst.iters if iters is None else iters
    u = torch.from_numpy(inst.unary).to(dev).requires_grad_(True)
    th = torch.from_numpy(inst.theta).to(dev).requires_grad_(True)
    logq = unrolled_mean_field(u, th, height=inst.height, width=inst.width,
                               connectivity=4 if inst.graph == synth.GRID4 else 8,
                               alpha=inst.alpha, iters=iters, ckpt_every=ckpt_every)
    c = torch.from_numpy(weights).to(dev)
    loss = (c * torch.exp(logq)).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (logq.detach().cpu().numpy().astype(np.float64), u.grad.cpu().numpy().astype(np.float64),
            th.grad.cpu().numpy().astype(np.float64))


def oracle_grads(inst, weights, iters=None):
    iters = inst.iters if iters is None else iters
    gu = np.zeros(inst.unary.shape)
    gt = np.zeros((inst.n_labels, inst.n_labels))
    ends = []
    for b in range(inst.batch):
        model = cases.oracle_model(inst, b)
        ell_T = O.solve(model, inst.alpha, iters)[-1]
        ends.append(ell_T)
        u_b, t_b = O.adjoint(model, inst.alpha, iters, weights[b].astype(np.float64) * np.exp(ell_T))
        gu[b] = u_b
        gt += t_b
    return np.array(ends), gu, gt


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(1e-30, np.abs(b).max()))


def test_adjoint_fd_instance():
    inst = synth.workload_fd()
    c = synth.adjoint_loss_weights(56, inst.unary.shape)
    ell, gu, gt = run_autograd(inst, c)
    ends, ou, ot = oracle_grads(inst, c)
    assert cases.max_dq(ell, ends) <= 1e-5
    assert rel_err(gu, ou) <= 1e-4, rel_err(gu, ou)
    assert rel_err(gt, ot) <= 1e-4, rel_err(gt, ot)


def test_adjoint_batch16_workload():
    inst = synth.workload_c5()
    c = synth.adjoint_loss_weights(57, inst.unary.shape)
    ell, gu, gt = run_autograd(inst, c)
    ends, ou, ot = oracle_grads(inst, c)
    assert cases.max_dq(ell, ends) <= 1e-5
    e_u, e_t = rel_err(gu, ou), rel_err(gt, ot)
    print("batch16 128x128 L=21 T=10: rel err grad u %.2e, grad Theta %.2e" % (e_u, e_t))
    assert e_u <= 1e-4 and e_t <= 1e-4


@pytest.mark.parametrize("ckpt_every", [1, 3, 10])
def test_checkpoint_spacing_does_not_change_gradients(ckpt_every):
    inst = synth.grid_theta_random(31, 40, 52, 6, synth.GRID8, iters=10)
    c = synth.adjoint_loss_weights(3, inst.unary.shape)
    _, gu5, gt5 = run_autograd(inst, c, ckpt_every=5)
    _, gu, gt = run_autograd(inst, c, ckpt_every=ckpt_every)
    np.testing.assert_array_equal(gu, gu5)
    np.testing.assert_array_equal(gt, gt5)


@pytest.mark.parametrize("H,W,L,conn,iters", [(9, 70, 2, synth.GRID4, 7), (33, 20, 13, synth.GRID8, 4),
                                                 (5, 5, 32, synth.GRID8, 3), (20, 20, 3, synth.GRID8, 0)])
def test_adjoint_shapes(H, W, L, conn, iters):
    inst = synth.grid_theta_random(50 + H + L, H, W, L, conn, iters=max(iters, 1))
    c = synth.adjoint_loss_weights(4, inst.unary.shape)
    _, gu, gt = run_autograd(inst, c, ckpt_every=3, iters=iters)
    _, ou, ot = oracle_grads(inst, c, iters=iters)
    assert rel_err(gu, ou) <= 1e-4
    if iters > 0:
        assert rel_err(gt, ot) <= 1e-4
    else:
        assert np.all(gt == 0)
