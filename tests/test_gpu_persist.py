"""The persistent grid kernel: every step of a launch in one resident
workgroup per 16 x 16 tile, the halo exchanged through tagged words.

The library takes it for grids with a general Theta, 8 < L <= 32 and at
most 256 tiles when the launch shape is left to it.  Its per-node
arithmetic is that of the fused multi-step kernel, so with the same launch
boundaries the iterates are compared bitwise with that kernel's, and over
longer horizons against the FP64 oracle (Sec. 3.1-3.2, Eq. 15-16; Jacobi
order of Sec. 2.2.2).
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

from paper_1511_06103_amd.mf import MF_PERSIST_STEPS_PER_LAUNCH as PERSIST_STEPS  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_06103_amd import mf
    mf.lib()


def state(s):
    torch.cuda.synchronize()
    return s.current_state().detach().cpu().numpy()


@pytest.fixture(scope="module")
def c2():
    return synth.workload_c2()


def test_chosen_for_small_theta_grids(c2):
    assert cases.gpu_solver(c2).steps_per_launch == PERSIST_STEPS
    # explicit launch shapes, Potts, few labels and grids of more than 256 tiles keep the other kernels
    assert cases.gpu_solver(c2, steps_per_launch=4).steps_per_launch == 4
    potts = synth.grid_potts_normal(3, 64, 21, synth.GRID8, w=0.5, iters=5)
    assert cases.gpu_solver(potts).steps_per_launch != PERSIST_STEPS
    few = synth.grid_theta_random(4, 64, 64, 8, synth.GRID8, iters=5)
    assert cases.gpu_solver(few).steps_per_launch != PERSIST_STEPS
    batch = synth.workload_c5()
    assert cases.gpu_solver(batch).steps_per_launch != PERSIST_STEPS


def fused_like(inst, n_fused=4, **kw):
    """The fused multi-step kernel at up to n_fused steps per launch, and the
    depth the library clamps that to for this label count."""
    f = cases.gpu_solver(inst, steps_per_launch=n_fused, **kw)
    return f, f.steps_per_launch


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16"])
def test_bitwise_equal_to_fused_kernel_per_launch(c2, precision):
    """With the same launch boundaries (each call of 2 to 4 steps is one
    launch of either kernel; a single step would take the one-step kernel)
    the two kernels give the same bits: q inside a launch comes from the
    log-sum-exp's terms, at a launch's start from exp(log q), in both."""
    a = cases.gpu_solver(c2, precision=precision)
    b, k = fused_like(c2, precision=precision)
    assert k == 4
    for n in (3, 2, 4, 4, 2, 4):
        a.step(n)
        b.step(n)
        ga, gb = state(a), state(b)
        assert np.array_equal(ga, gb), (n, float(np.abs(ga - gb).max()))
    assert a.check() is None and b.check() is None


def test_long_solve_against_oracle(c2):
    """100 steps of the benchmark grid in one launch (alpha = 0.5): within the
    bound of the parity report, 1e-5 or twice the oracle's own FP32 drift."""
    s = cases.gpu_solver(c2)
    s.step(100)
    assert s.check() is None
    model = cases.oracle_model(c2)
    ref = O.solve(model, c2.alpha, 100)[-1]
    floor = cases.max_dq(O.solve(model.astype(np.float32), np.float32(c2.alpha), 100)[-1], ref)
    err = cases.max_dq(state(s)[0].astype(np.float64), ref)
    assert err <= max(1e-5, 2.0 * floor), (err, floor)


def test_launches_continue_the_exchange(c2):
    """Launches of one handle continue its tags (a re-initialising solve and
    a second handle stepped in between included): the iterates match the
    fused kernel launched at the same boundaries."""
    a = cases.gpu_solver(c2)
    other = cases.gpu_solver(c2, alpha=0.3)
    b, _ = fused_like(c2)
    for n in (2, 4, 2, 3, 4, 4, 2):
        a.step(n)
        other.step(3)
        b.step(n)
    assert np.array_equal(state(a), state(b))
    a.solve(3)
    b.solve(3)
    assert np.array_equal(state(a), state(b))
    assert a.check() is None and other.check() is None


@pytest.mark.parametrize("H,W,L,conn,B,alpha", [
    (100, 75, 21, synth.GRID8, 2, 0.5),     # ragged tiles on both edges, a batch of two
    (33, 131, 13, synth.GRID8, 1, 0.5),
    (40, 33, 21, synth.GRID4, 1, 0.6),
    (17, 17, 32, synth.GRID8, 1, 0.4),
    (16, 16, 9, synth.GRID4, 1, 0.5),       # one tile: no neighbours at all
    (1, 200, 16, synth.GRID8, 1, 0.5),      # one row of tiles, one node high
    (256, 16, 24, synth.GRID8, 1, 0.5),     # one column of tiles
])
def test_shapes_against_oracle_and_fused(H, W, L, conn, B, alpha):
    inst = synth.grid_theta_random(200 + H + 3 * W + L, H, W, L, conn, batch=B, alpha=alpha, iters=10)
    s = cases.gpu_solver(inst)
    assert s.steps_per_launch == PERSIST_STEPS
    f, k = fused_like(inst)
    s.step(k)
    f.step(k)
    assert np.array_equal(state(s), state(f)), k
    s.step(10 - k)
    assert s.check() is None
    g = state(s)
    for b in range(B):
        ref = O.solve(cases.oracle_model(inst, b), alpha, 10)[-1]
        assert cases.max_dq(g[b].astype(np.float64), ref) <= 1e-5, b


@pytest.mark.parametrize("precision,tol", [("bf16", 2e-3), ("f16", 2e-4)])
def test_message_precisions_against_oracle(precision, tol):
    """Per-step message-precision bound times the steps."""
    inst = synth.grid_theta_random(77, 48, 80, 21, synth.GRID8, alpha=0.5, iters=3)
    s = cases.gpu_solver(inst, precision=precision)
    assert s.steps_per_launch == PERSIST_STEPS
    s.step(3)
    ref = O.solve(cases.oracle_model(inst), 0.5, 3)[-1]
    assert cases.max_dq(state(s)[0].astype(np.float64), ref) <= 3 * tol


@pytest.mark.parametrize("init", ["unary", "uniform", "state"])
def test_solve_in_one_launch_matches_separate_kernels(c2, init):
    """solve() runs the initialisation, the steps and the write-out of q in
    one launch; mf_init's initialisation kernel, one launch of the same steps
    and the separate write-out give the same bits (Eq. 6 reading of q^0)."""
    B, L, N = c2.unary.shape
    st = None
    if init == "state":
        st = torch.empty((2, B, L, N), dtype=torch.float32, device="cuda:0")
        g = np.random.default_rng(5).standard_normal((B, L, N)).astype(np.float32)
        st[0].copy_(torch.from_numpy(g - np.log(np.exp(g).sum(1, keepdims=True))))
    kw = {} if st is None else {"state": st.clone()}
    a = cases.gpu_solver(c2, init=init, **kw)
    qa = torch.empty_like(a.unary)
    a.solve(7, qa)
    kw = {} if st is None else {"state": st.clone()}
    b = cases.gpu_solver(c2, init=init, **kw)
    b.step(7)
    qb = b.marginals()
    torch.cuda.synchronize()
    assert np.array_equal(state(a), state(b))
    assert torch.equal(qa, qb)
    assert a.check() is None and b.check() is None


def test_non_finite_unary_reported_by_the_one_launch_solve():
    inst = synth.grid_theta_random(9, 40, 40, 21, synth.GRID8, iters=3)
    inst.unary[0, 3, 77] = np.nan
    from paper_1511_06103_amd import mf
    s = cases.gpu_solver(inst)
    assert s.steps_per_launch == PERSIST_STEPS
    with pytest.raises(mf.MFError) as e:      # mf_init's own initialisation reports it first
        s.check()
    assert e.value.status == mf.MF_ENONFINITE
    s.solve(3)                                # reporting cleared it: this one comes from the solve's launch
    with pytest.raises(mf.MFError) as e:
        s.check()
    assert e.value.status == mf.MF_ENONFINITE


def test_wait_bound_gives_up_into_the_flags(c2, monkeypatch):
    """With the halo-wait bound set to zero (MF_PERSIST_WAIT_US=0) every wait
    that finds a tag not yet written gives up at once: the launch still ends,
    and mf_check reports it; with the default bound the next solve is clean."""
    from paper_1511_06103_amd import mf
    s = cases.gpu_solver(c2)
    monkeypatch.setenv("MF_PERSIST_WAIT_US", "0")
    s.solve(20)
    with pytest.raises(mf.MFError) as e:
        s.check()
    assert e.value.status == mf.MF_EDEVICE and "halo" in str(e.value)
    monkeypatch.delenv("MF_PERSIST_WAIT_US")
    s.solve(20)
    assert s.check() is None
    ref = cases.gpu_solver(c2)
    ref.solve(20)
    assert np.array_equal(state(s), state(ref))


def test_launches_on_two_streams(c2):
    """Persistent launches of two handles on two streams run one after the
    other (never sharing the compute units): each matches its solo result."""
    other = synth.grid_theta_random(31, 256, 256, 21, synth.GRID8, alpha=0.4, iters=30)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = cases.gpu_solver(c2, stream=s1)
    b = cases.gpu_solver(other, stream=s2)
    for n in (3, 2, 4, 3):
        a.step(n)
        b.step(n)
    ra, rb = cases.gpu_solver(c2), cases.gpu_solver(other)
    for n in (3, 2, 4, 3):
        ra.step(n)
        rb.step(n)
    assert a.check() is None and b.check() is None
    assert np.array_equal(state(a), state(ra)) and np.array_equal(state(b), state(rb))


@pytest.mark.parametrize("L", [9, 12, 16, 17, 21, 24, 25, 32])
@pytest.mark.parametrize("conn", [synth.GRID4, synth.GRID8])
def test_every_label_count(L, conn):
    """Each label-slot instantiation (4, 6 or 8 slots per lane, the L = 21
    one compiled in) on a 40 x 50 grid: bitwise equal to the fused kernel
    over one launch of two steps, then 8 more steps against the oracle."""
    inst = synth.grid_theta_random(500 + L + conn, 40, 50, L, conn, alpha=0.5, iters=10)
    s = cases.gpu_solver(inst)
    assert s.steps_per_launch == PERSIST_STEPS
    f, k = fused_like(inst)
    s.step(2)
    f.step(2)
    assert np.array_equal(state(s), state(f))
    s.step(8)
    assert s.check() is None
    ref = O.solve(cases.oracle_model(inst), 0.5, 10)[-1]
    assert cases.max_dq(state(s)[0].astype(np.float64), ref) <= 1e-5


def test_batch_of_small_grids():
    """Four 64 x 64 problems (64 tiles in one launch) against the oracle."""
    inst = synth.grid_theta_random(77, 64, 64, 21, synth.GRID8, batch=4, alpha=0.5, iters=10)
    s = cases.gpu_solver(inst)
    assert s.steps_per_launch == PERSIST_STEPS
    s.solve(10)
    assert s.check() is None
    g = state(s)
    for b in range(4):
        ref = O.solve(cases.oracle_model(inst, b), 0.5, 10)[-1]
        assert cases.max_dq(g[b].astype(np.float64), ref) <= 1e-5, b
