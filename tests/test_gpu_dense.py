"""GPU parity of the fully connected CRF path (BF16 Gaussian kernel, K Q on
MFMA, co-occurrence term) against the FP64 oracle.

Tolerances, max |q_gpu - q_oracle|:
* FP32 mode (q split into three BF16 planes, FP32 accumulation): 2e-6 per
  step from an identical state; end to end 1e-5 up to t = 10 and twice the
  FP32 rounding floor (the oracle's arithmetic run in FP32) after that;
* BF16 messages (one plane): 2e-3 per step.
Both sides receive the same BF16 kernel matrix (built by the input
generator from the features).  The library's own kernel builder
(mf_dense_kernel, FP32 on the device) is checked separately against the
oracle's FP64 kernel rounded the same way: they agree to one BF16 unit in
the last place (a handful of entries sit on a rounding edge).
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


def gpu_state(s):
    torch.cuda.synchronize()
    return s.current_state().detach().cpu().numpy().astype(np.float64)


def gpu_K(inst):
    """The instance's kernel matrix, as the input generator builds it, on the device."""
    return cases.dense_K_device(inst)


def built_K(inst):
    """The kernel matrix built by the library from the features."""
    from paper_1511_06103_amd import mf
    K = mf.dense_kernel(torch.from_numpy(inst.features).to("cuda:0"))
    torch.cuda.synchronize()
    return K


def K_to_f64(K):
    return K.float().cpu().numpy().astype(np.float64)


def bf16_ulps(a, b):
    ia = a.astype(np.float32).view(np.int32).astype(np.int64)
    ib = b.astype(np.float32).view(np.int32).astype(np.int64)
    return np.abs(ia - ib) >> 16


@pytest.mark.parametrize("n", [1, 7, 300, 1024])
def test_dense_kernel_builder(n):
    inst = synth.dense_instance(60 + n, n, 3)
    K = K_to_f64(built_K(inst))
    ref = O.round_to_bf16(O.gaussian_kernel(inst.features))
    assert np.all(np.diag(K) == 0)
    d = bf16_ulps(K, ref)
    assert d.max() <= 1
    assert (d == 0).mean() >= 0.999
    np.testing.assert_array_equal(K, K.T)


@pytest.fixture(scope="module")
def small():
    inst = synth.dense_instance(11, 300, 5, pos_high=12.0, iters=12)
    K = gpu_K(inst)
    return inst, K, O.dense_model(inst.unary[0], K_to_f64(K), potts_w=inst.potts_w,
                                  cooc=inst.cooc.astype(np.float64))


@pytest.mark.parametrize("precision,tol", [("f32", 2e-6), ("f16", 1e-4), ("bf16", 2e-3)])
def test_dense_one_step_from_identical_state(small, precision, tol):
    inst, K, model = small
    start = O.solve(model, 0.5, 4)[-1].astype(np.float32)
    B, L, N = inst.unary.shape
    st = torch.empty((2, B, L, N), dtype=torch.float32, device="cuda:0")
    st[0].copy_(torch.from_numpy(start[None]))
    s = cases.gpu_solver(inst, init="state", state=st, precision=precision, dense_K=K)
    s.step(1)
    err = cases.max_dq(gpu_state(s)[0], O.prox_step(start.astype(np.float64), model, 0.5))
    assert err <= tol, (precision, err)


def test_dense_small_end_to_end_and_free_energy(small):
    inst, K, model = small
    s = cases.gpu_solver(inst, dense_K=K)
    ref = O.solve(model, 0.5, 12)
    assert cases.max_dq(gpu_state(s)[0], ref[0]) <= 1e-6
    for t in (1, 5, 12):
        s.step(t - s.iteration)
        g = gpu_state(s)[0]
        assert cases.max_dq(g, ref[t]) <= 1e-5, t
        F = s.free_energy()[0]
        Fr = O.free_energy(g, model)
        assert abs(F - Fr) <= 1e-9 * max(1.0, abs(Fr)), (t, F, Fr)


@pytest.mark.parametrize("n,L,cooc,potts", [(1, 3, True, True), (7, 5, False, False), (64, 2, False, True),
                                            (129, 21, True, True), (517, 7, False, False),
                                            (1000, 32, True, False), (300, 21, True, False), (776, 21, False, False)])
def test_dense_variants(n, L, cooc, potts):
    base = synth.dense_instance(5 + n, n, L, pos_high=16.0, iters=6, with_cooc=cooc)
    if not potts:
        rng = np.random.default_rng(n)
        base.theta = synth.symmetric_zero_diag(rng, L, 0.0, 1.0)
        base.compat = synth.COMPAT_GENERAL
    K = gpu_K(base)
    model = O.dense_model(base.unary[0], K_to_f64(K), potts_w=base.potts_w if potts else None,
                          theta=None if potts else base.theta.astype(np.float64),
                          cooc=None if base.cooc is None else base.cooc.astype(np.float64))
    s = cases.gpu_solver(base, dense_K=K)
    s.step(6)
    g = gpu_state(s)[0]
    assert cases.max_dq(g, O.solve(model, base.alpha, 6)[-1]) <= 1e-5
    F = s.free_energy()[0]
    Fr = O.free_energy(g, model)
    assert abs(F - Fr) <= 1e-9 * max(1.0, abs(Fr))


def test_dense_batch_of_two():
    inst = synth.dense_instance(21, 256, 4, pos_high=10.0, iters=5)
    inst.unary = np.ascontiguousarray(np.concatenate([inst.unary, inst.unary[:, ::-1, :]], axis=0))
    K = gpu_K(inst)
    s = cases.gpu_solver(inst, dense_K=K)
    s.step(5)
    g = gpu_state(s)
    for b in range(2):
        model = O.dense_model(inst.unary[b], K_to_f64(K), potts_w=inst.potts_w, cooc=inst.cooc.astype(np.float64))
        assert cases.max_dq(g[b], O.solve(model, 0.5, 5)[-1]) <= 1e-5


def test_dense_workload_4096_end_to_end():
    inst = synth.workload_c3()
    K = gpu_K(inst)
    Kh = K_to_f64(K)
    model = O.dense_model(inst.unary[0], Kh, potts_w=inst.potts_w, cooc=inst.cooc.astype(np.float64))
    ref = O.solve(model, 0.5, 50)
    floor = O.solve(model.astype(np.float32), 0.5, 50)
    s = cases.gpu_solver(inst, dense_K=K)
    report = []
    t = 0
    for target in (1, 10, 25, 50):
        s.step(target - t)
        t = target
        g = gpu_state(s)[0]
        err, fl = cases.max_dq(g, ref[t]), cases.max_dq(floor[t], ref[t])
        report.append((t, err, fl))
        bound = 1e-5 if t <= 10 else max(1e-5, 2 * fl)
        assert err <= bound, report
    # the library's kernel builder agrees with the oracle's kernel to one BF16 ulp
    ref_rows = O.round_to_bf16(O.gaussian_kernel(inst.features)[:64])
    assert bf16_ulps(K_to_f64(built_K(inst))[:64], ref_rows).max() <= 1
    print("dense 4096 t, max|dq|, fp32 floor:", report)


def test_dense_workload_bf16_messages():
    inst = synth.workload_c3()
    K = gpu_K(inst)
    model = O.dense_model(inst.unary[0], K_to_f64(K), potts_w=inst.potts_w, cooc=inst.cooc.astype(np.float64))
    ref = O.solve(model, 0.5, 50)
    emul = O.solve(model, 0.5, 50, operand=O.round_to_bf16)
    s = cases.gpu_solver(inst, dense_K=K, precision="bf16")
    s.step(50)
    g = gpu_state(s)[0]
    err, fl = cases.max_dq(g, ref[50]), cases.max_dq(emul[50], ref[50])
    agree = float((g.argmax(0) == ref[50].argmax(0)).mean())
    print("dense 4096 bf16 messages: max|dq| %.3e, bf16 rounding floor %.3e, argmax agreement %.5f" % (err, fl, agree))
    assert err <= max(2e-3, 1.25 * fl)


def test_dense_monotone_free_energy_at_admissible_alpha():
    inst = synth.dense_instance(3, 1024, 21, pos_high=32.0)
    K = gpu_K(inst)
    model = O.dense_model(inst.unary[0], K_to_f64(K), potts_w=inst.potts_w, cooc=inst.cooc.astype(np.float64))
    lip, _ = O.lipschitz_power(model, iters=300)
    alpha = float(np.float32(O.admissible_alpha(1.02 * lip)))
    s = cases.gpu_solver(inst, dense_K=K, alpha=alpha)
    F = [s.free_energy()[0]]
    for _ in range(20):
        s.step(1)
        F.append(s.free_energy()[0])
    F = np.array(F)
    assert np.all(np.diff(F) <= 1e-6 * np.abs(F[:-1])), F
    assert F[-1] < F[0]
