"""The oracle's pins bite: each plausible mistake planted in the oracle fails
at least one pin of tests/test_oracle_pins.py.

Every case below replaces one oracle function (in ``oracle.mf`` and in the
``oracle`` package namespace, so that both the pins and the other oracle
functions see it) with a copy that carries one planted mistake, then runs a
chosen set of pins and requires at least one of them to fail.  The
mutations live only in this file and only for the duration of a case
(pytest's monkeypatch); nothing runs on a GPU.
"""
import numpy as np
import pytest

import oracle as O
import oracle.mf as M
import test_oracle_pins as P


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

def energy_without_half(q, model):
    # every pair counted twice
    return float((q * model.unary).sum() + (q * M.pairwise_message(q, model)).sum())


def entropy_wrong_sign(ell):
    return float((np.exp(ell) * ell).sum())


def messages_pairwise_sign_flipped(ell, model, operand=None):
    q = np.exp(ell)
    if operand is not None:
        q = operand(q)
    return model.unary - M.pairwise_message(q, model)


def pairwise_message_sign_flipped(q, model):
    out = -(model.theta @ M.neighbour_sum(q, model))
    if model.cooc is not None:
        T = q.sum(axis=1, keepdims=True)
        out = out + model.cooc @ (T - q) / q.shape[1]
    return out


def pairwise_message_cooc_keeps_self_pair(q, model):
    out = model.theta @ M.neighbour_sum(q, model)
    if model.cooc is not None:
        out = out + model.cooc @ q.sum(axis=1, keepdims=True) / q.shape[1]
    return out


def prox_step_plus_message(ell, model, alpha, operand=None):
    m = M.messages(ell, model, operand)
    return M.normalise((1.0 - alpha) * ell + alpha * m)


def prox_step_swapped_weights(ell, model, alpha, operand=None):
    m = M.messages(ell, model, operand)
    return M.normalise(alpha * ell - (1.0 - alpha) * m)


def normalise_without_logsumexp(z):
    z = np.asarray(z)
    return z - z.max(axis=0, keepdims=True)


def init_state_wrong_sign(unary, mode=0):
    u = np.asarray(unary)
    if mode == 0:
        return M.normalise(u)
    return np.full(u.shape, -np.log(u.shape[0]), dtype=u.dtype)


def potts_theta_with_diagonal(n_labels, w):
    return w * np.ones((n_labels, n_labels))


def grid_edges_one_diagonal(height, width, conn):
    edges = []
    for y in range(height):
        for x in range(width):
            i = y * width + x
            nbrs = [(0, 1), (1, 0)] + ([(1, 1)] if conn == 8 else [])
            for dy, dx in nbrs:
                yy, xx = y + dy, x + dx
                if 0 <= yy < height and 0 <= xx < width:
                    j = yy * width + xx
                    edges.append((min(i, j), max(i, j)))
    return np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)


def adjacency_eigs_8conn_as_4conn(height, width, conn):
    a = 2 * np.cos(np.pi * np.arange(1, height + 1) / (height + 1))
    b = 2 * np.cos(np.pi * np.arange(1, width + 1) / (width + 1))
    return (a[:, None] + b[None, :]).ravel()


def lipschitz_grid_largest_products_only(height, width, conn, theta, w=1.0):
    lam = M.adjacency_eigs_grid(height, width, conn) * w
    mu = M.tangent_compat_eigs(np.asarray(theta, dtype=np.float64))
    return float(lam.max() * mu.max()) if mu.size else 0.0


def hv_without_projection(v, model):
    # the Hessian of E on the whole space, all-ones directions included
    return M.pairwise_message(v, model)


def round_to_bf16_truncating(x):
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32) & np.uint32(0xFFFF0000)
    return bits.view(np.float32).astype(np.float64)


def gaussian_kernel_without_half(features):
    f = np.asarray(features, dtype=np.float64)
    K = np.exp(-((f[:, None, :] - f[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(K, 0.0)
    return K


def sweep_jacobi(ell, model, n_sweeps=1, order=None):
    # every node reads the q of the previous sweep (no Gauss-Seidel)
    q = np.exp(np.asarray(ell, dtype=np.float64)).copy()
    for _ in range(n_sweeps):
        m = model.unary + model.theta @ M.neighbour_sum(q, model)
        e = np.exp(-m - (-m).max(axis=0, keepdims=True))
        q = e / e.sum(axis=0, keepdims=True)
    return np.log(q)


def _adjoint_variant(kind):
    """The reverse pass with one planted mistake ("theta_bar_transposed" or
    "q_dropped": the q factor of the exp in the state gradient left out)."""
    def adjoint(model, alpha, iters, grad_ell_T, init_mode=0):
        traj = M.solve(model, alpha, iters, init_mode)
        g = np.asarray(grad_ell_T, dtype=np.float64).copy()
        u_bar = np.zeros_like(model.unary)
        th_bar = np.zeros_like(model.theta)
        for t in range(iters - 1, -1, -1):
            q_t, q_n = np.exp(traj[t]), np.exp(traj[t + 1])
            z_bar = g - q_n * g.sum(axis=0, keepdims=True)
            m_bar = -alpha * z_bar
            u_bar += m_bar
            S = M.neighbour_sum(q_t, model)
            th_bar += (S @ m_bar.T) if kind == "theta_bar_transposed" else (m_bar @ S.T)
            q_bar = M._neighbour_sum_transpose(model.theta.T @ m_bar, model)
            if model.cooc is not None:
                c_bar = model.cooc.T @ m_bar / q_t.shape[1]
                q_bar = q_bar + c_bar.sum(axis=1, keepdims=True) - c_bar
            g = (1.0 - alpha) * z_bar + (q_bar if kind == "q_dropped" else q_t * q_bar)
        if init_mode == 0:
            q0 = np.exp(traj[0])
            u_bar += -(g - q0 * g.sum(axis=0, keepdims=True))
        return u_bar, th_bar
    return adjoint


def _adam_variant(kind):
    """ADAM of the oracle with one planted mistake: "uncentred" (g not
    centred over labels), "swapped" (gamma2 on the new g^2, as printed),
    "late_v" (the step from the previous second moment), "abs" (|g| for g^2)."""
    def adam_solve(model, d, iters, gamma1=0.9, gamma2=0.999, eps=1e-8, v0=1.0, init_mode=0, ell0=None):
        ell = M.init_state(model.unary, init_mode) if ell0 is None else np.asarray(ell0, dtype=np.float64)
        mom = M.messages(ell, model)
        v = np.full_like(ell, v0)
        out = [ell]
        for _ in range(iters):
            m = M.messages(ell, model)
            mom = gamma1 * mom + (1.0 - gamma1) * m
            g = m + ell
            if kind != "uncentred":
                g = g - g.mean(axis=0, keepdims=True)
            g2 = np.abs(g) if kind == "abs" else g * g
            v_new = (1.0 - gamma2) * v + gamma2 * g2 if kind == "swapped" else gamma2 * v + (1.0 - gamma2) * g2
            dt = np.maximum(np.sqrt(v if kind == "late_v" else v_new) * d + eps - 1.0, 1e-6)
            v = v_new
            eta = 1.0 / (1.0 + dt)
            ell = M.normalise((1.0 - eta) * ell - eta * mom)
            out.append(ell)
        return out
    return adam_solve


# ---------------------------------------------------------------------------
# which pins must catch which mistake
# ---------------------------------------------------------------------------

def _pin(fn, *args):
    return (f"{fn.__name__}{args if args else ''}", lambda: fn(*args))


ADAM_PINS = [_pin(P.test_adam_second_moment_binary_theta_zero_recursion, 0.5),
             _pin(P.test_adam_second_moment_binary_theta_zero_recursion, 0.999)]

CASES = {
    "free energy: pairs counted twice": (
        {"energy": energy_without_half},
        [_pin(P.test_two_node_closed_forms), _pin(P.test_free_energy_plus_logz_is_kl_3x3)]),
    "free energy: entropy sign": (
        {"entropy": entropy_wrong_sign},
        [_pin(P.test_two_node_closed_forms), _pin(P.test_free_energy_plus_logz_is_kl_3x3)]),
    "message: pairwise sign in m": (
        {"messages": messages_pairwise_sign_flipped},
        [_pin(P.test_two_node_closed_forms), _pin(P.test_alpha_one_is_naive_parallel)]),
    "message: pairwise sign in Theta S": (
        {"pairwise_message": pairwise_message_sign_flipped},
        [_pin(P.test_message_is_energy_gradient, "grid8_theta"), _pin(P.test_two_node_closed_forms)]),
    "message: co-occurrence keeps the self pair": (
        {"pairwise_message": pairwise_message_cooc_keeps_self_pair},
        [_pin(P.test_message_is_energy_gradient, "dense_cooc"),
         _pin(P.test_dense_cooc_free_energy_against_enumeration)]),
    "step: message added instead of subtracted": (
        {"prox_step": prox_step_plus_message},
        [_pin(P.test_step_satisfies_kkt_and_minimises_prox_objective), _pin(P.test_theta_zero_closed_form)]),
    "step: alpha and 1 - alpha swapped": (
        {"prox_step": prox_step_swapped_weights},
        [_pin(P.test_step_satisfies_kkt_and_minimises_prox_objective), _pin(P.test_theta_zero_closed_form)]),
    "normalisation: max only, no log-sum-exp": (
        {"normalise": normalise_without_logsumexp},
        [_pin(P.test_normalisation_every_iterate), _pin(P.test_normalise_matches_library_log_softmax)]),
    "init: softmax(+u)": (
        {"init_state": init_state_wrong_sign},
        [_pin(P.test_init_modes)]),
    "Potts: nonzero diagonal": (
        {"potts_theta": potts_theta_with_diagonal},
        [_pin(P.test_two_node_closed_forms)]),
    "grid: one diagonal missing": (
        {"grid_edges": grid_edges_one_diagonal},
        [_pin(P.test_grid_edge_counts, 4, 7), _pin(P.test_grid_neighbour_sets_by_hand)]),
    "spectrum: 8-connected grid as 4-connected": (
        {"adjacency_eigs_grid": adjacency_eigs_8conn_as_4conn},
        [_pin(P.test_adjacency_closed_form_matches_eigvalsh, 4, 6, 8)]),
    "Lipschitz: only the product of the largest eigenvalues": (
        {"lipschitz_grid": lipschitz_grid_largest_products_only},
        [_pin(P.test_lipschitz_constants_of_the_potts_workloads),
         _pin(P.test_lipschitz_closed_form_against_dense_tangent_hessian)]),
    "power method: no projection on the tangent space": (
        {"_hv_tangent": hv_without_projection},
        [_pin(P.test_power_method_theta_grid8)]),
    "BF16 rounding truncates": (
        {"round_to_bf16": round_to_bf16_truncating},
        [_pin(P.test_round_to_bf16_matches_torch)]),
    "Gaussian kernel without the 1/2": (
        {"gaussian_kernel": gaussian_kernel_without_half},
        [_pin(P.test_gaussian_kernel_matches_cdist)]),
    "SWEEP: Jacobi instead of Gauss-Seidel": (
        {"sweep": sweep_jacobi},
        [_pin(P.test_sweep_two_node_by_hand)]),
    "adjoint: Theta_bar transposed": (
        {"adjoint": _adjoint_variant("theta_bar_transposed")},
        [_pin(P.test_adjoint_dense_cooc_small)]),
    "adjoint: q dropped from the state gradient": (
        {"adjoint": _adjoint_variant("q_dropped")},
        [_pin(P.test_adjoint_dense_cooc_small)]),
    "ADAM: g not centred": ({"adam_solve": _adam_variant("uncentred")}, ADAM_PINS),
    "ADAM: gamma2 placement as printed": ({"adam_solve": _adam_variant("swapped")}, ADAM_PINS),
    "ADAM: step from the previous second moment": ({"adam_solve": _adam_variant("late_v")}, ADAM_PINS),
    "ADAM: |g| for g^2": ({"adam_solve": _adam_variant("abs")}, ADAM_PINS),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_planted_mistake_fails_a_pin(name, monkeypatch):
    patches, pins = CASES[name]
    # the pins pass on the unmutated oracle (checked once per case, cheaply)
    for fn_name, repl in patches.items():
        assert hasattr(M, fn_name), fn_name
        monkeypatch.setattr(M, fn_name, repl)
        if hasattr(O, fn_name):
            monkeypatch.setattr(O, fn_name, repl)
    caught = []
    for label, run in pins:
        try:
            run()
        except (AssertionError, FloatingPointError, ValueError):
            caught.append(label)
    assert caught, f"no pin caught the planted mistake '{name}' (ran {[p[0] for p in pins]})"


def test_pins_pass_without_mutation():
    """The same pin calls pass on the oracle as it stands, so a failure above
    is the planted mistake's doing."""
    seen = set()
    for _, pins in CASES.values():
        for label, run in pins:
            if label not in seen:
                seen.add(label)
                run()
