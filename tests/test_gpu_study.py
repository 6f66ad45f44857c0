"""The damping-sensitivity study (paper_1511_06103_amd.study) against the
FP64 oracle: F after T steps of OURS-FIXED (Eq. 15-16), ADHOC (Eq. 9) and
OURS-ADAPTIVE (Eq. 19) at each eta of a small log grid on a frustrated
(repulsive, 8-connected) binary grid, and the eta it reports for d = L-hat
(Sec. 3.2) against the grid closed form."""
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


def _oracle_F(model, rule, eta, iters):
    ell = O.init_state(model.unary)
    d = float(np.float32(1.0 / eta - 1.0))     # the kernels hold d in FP32
    for _ in range(iters):
        if rule == "fixed":
            ell = O.prox_step(ell, model, eta)
        elif rule == "adhoc":
            ell = O.adhoc_step(ell, model, eta)
        else:
            ell = O.adaptive_binary_step(ell, model, d)
    return O.free_energy(ell, model)


def test_sensitivity_sweep_matches_oracle():
    from paper_1511_06103_amd import study
    T = 15
    inst = synth.grid_repulsive(21, 16, w=2.0, iters=T)
    etas = study.log_grid(0.05, 0.4, 3)
    res = study.sensitivity(inst, etas, T, lipschitz_iters=4000)
    assert set(res["F"]) == {"fixed", "adhoc", "adaptive"}
    model = cases.oracle_model(inst)
    for rule, fs in res["F"].items():
        for eta, F in zip(etas, fs):
            ref = _oracle_F(model, rule, eta, T)
            assert abs(F - ref) <= 1e-5 * max(1.0, abs(ref)), (rule, eta, F, ref)
    exact = cases.oracle_lipschitz(inst)
    assert exact * (1 - 2e-3) <= res["lipschitz"] <= exact * (1 + 1e-6), (res["lipschitz"], exact)
    assert abs(res["eta_adm"] - O.admissible_alpha(res["lipschitz"])) < 1e-12


def test_sensitivity_skips_adaptive_beyond_binary():
    from paper_1511_06103_amd import study
    inst = synth.grid_theta_random(22, 12, 12, 5, synth.GRID8, iters=4)
    res = study.sensitivity(inst, [0.5], 4, lipschitz_iters=50)
    assert set(res["F"]) == {"fixed", "adhoc"}
    ref = _oracle_F(cases.oracle_model(inst), "fixed", 0.5, 4)
    assert abs(res["F"]["fixed"][0] - ref) <= 1e-5 * max(1.0, abs(ref))
