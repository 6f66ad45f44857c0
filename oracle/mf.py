"""FP64 oracle: models, messages, the proximal step, free energy, enumeration,
sequential sweep, Lipschitz constants and the reverse pass.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation (Baque et al., "Principled Parallel Mean-Field Inference for
Discrete Random Fields"):

* ``u[l, i]``: unary energy of node i taking label l.  Energies follow the
  reading P(x) proportional to exp(-sum_i u_i(x_i) - sum_{(i,j)} w_ij Theta(x_i, x_j))
  of Eq. 2 (Sec. 2.1), so that the natural parameters of Eq. 6 are
  theta = -log q + const.
* ``q[l, i]``: mean parameters of the factorised Q (Eq. 3-4), one simplex per node.
* ``ell = log q``: the log-space state; it equals -theta up to a per-node constant.
* ``S[:, i] = sum_j w_ij q[:, j]``: neighbour aggregation.
* ``m[:, i] = u[:, i] + Theta @ S[:, i]``: the message, equal to the gradient of
  the expected energy (theta* of Eq. 15, Sec. 3.1).
* ``alpha = eta = 1 / (1 + d)`` (Eq. 16, Sec. 3.2).

All arrays are label-major, ``[L, N]``, float64.

Pins (tests/test_oracle_pins.py): every function here is checked against
closed forms, brute force, independent library routines or special cases
that reduce it to another pinned function.  The ADAM reading of Sec. 3.5
(``adam_solve``) is pinned for gamma2 = 1 by the fixed step and for
gamma2 < 1 by a scalar recursion worked out by hand for Theta = 0, L = 2.
tests/test_oracle_mutations.py plants plausible mistakes in these functions
and checks that a pin fails for each.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse

__all__ = [
    "Model", "potts_theta", "grid_edges", "grid_model", "csr_model", "dense_model", "gaussian_kernel",
    "round_to_bf16", "round_to_f16", "normalise", "init_state", "neighbour_sum", "pairwise_message", "messages",
    "prox_step", "prox_objective", "solve", "energy", "energy_edge_sum", "entropy",
    "free_energy", "brute_force", "kl_divergence", "sweep", "naive_parallel_step",
    "adjacency_eigs_grid", "tangent_compat_eigs", "lipschitz_grid", "lipschitz_power",
    "admissible_alpha", "unrolled_loss", "adjoint", "fd_grad",
    "adhoc_step", "adaptive_binary_step", "momentum_solve", "adam_solve",
]


# ----------------------------------------------------------------------------
# Models
# ----------------------------------------------------------------------------

@dataclass
class Model:
    """A pairwise discrete random field (Eq. 2, Sec. 2.1) with a shared compatibility.

    ``theta`` is the full L x L compatibility, ``theta[l, k]`` being the energy
    of (x_i = l, x_j = k) on an edge of unit weight.  Sparse graphs are given
    as directed arcs (``arc_dst[e]`` receives ``w[e] * q[:, arc_src[e]]``) and,
    for the energy, as undirected edges listed once.  Dense graphs carry the
    N x N kernel ``K`` (zero diagonal) and an optional global co-occurrence
    compatibility ``cooc`` applied with weight 1/N per node pair.
    """
    unary: np.ndarray
    theta: np.ndarray
    arc_dst: Optional[np.ndarray] = None
    arc_src: Optional[np.ndarray] = None
    arc_w: Optional[np.ndarray] = None
    edges: Optional[np.ndarray] = None    # [E, 2] undirected, i < j
    edge_w: Optional[np.ndarray] = None   # [E]
    K: Optional[np.ndarray] = None        # [N, N]
    cooc: Optional[np.ndarray] = None     # [L, L]

    @property
    def n_labels(self):
        return self.unary.shape[0]

    def astype(self, dtype):
        """The same model with its floating-point arrays cast to ``dtype``.

        FP64 is the oracle's precision; an FP32 copy runs the same arithmetic
        in single precision, which measures how far rounding alone moves an
        iterate (the floor any FP32 implementation shares).
        """
        cast = lambda a: None if a is None else np.asarray(a).astype(dtype)
        return Model(unary=cast(self.unary), theta=cast(self.theta), arc_dst=self.arc_dst,
                     arc_src=self.arc_src, arc_w=cast(self.arc_w), edges=self.edges,
                     edge_w=cast(self.edge_w), K=cast(self.K), cooc=cast(self.cooc))

    @property
    def n_nodes(self):
        return self.unary.shape[1]


def grid_edges(height, width, conn):
    """Undirected edges of a height x width grid with a free (non-periodic) boundary.

    Node index n = y * width + x.  4-connectivity links horizontal and
    vertical neighbours; 8-connectivity adds both diagonals.  Each edge is
    listed once as (i, j) with i < j.  The paper leaves the boundary and the
    diagonal weight unstated; the reading here is a free boundary and unit
    weight on every edge.
    """
    edges = []
    for y in range(height):
        for x in range(width):
            i = y * width + x
            nbrs = [(0, 1), (1, 0)]
            if conn == 8:
                nbrs += [(1, 1), (1, -1)]
            for dy, dx in nbrs:
                yy, xx = y + dy, x + dx
                if 0 <= yy < height and 0 <= xx < width:
                    j = yy * width + xx
                    edges.append((min(i, j), max(i, j)))
    return np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)


def potts_theta(n_labels, w):
    """Potts compatibility w * (1 1^T - I): energy w when the labels differ, 0 otherwise."""
    return w * (np.ones((n_labels, n_labels)) - np.eye(n_labels))


def _arcs_from_edges(edges, w):
    dst = np.concatenate([edges[:, 0], edges[:, 1]])
    src = np.concatenate([edges[:, 1], edges[:, 0]])
    return dst, src, np.concatenate([w, w])


def grid_model(unary, height, width, conn, theta=None, potts_w=None):
    """Grid model: ``conn`` is 4 or 8; either a full ``theta`` or a Potts weight."""
    unary = np.asarray(unary, dtype=np.float64)
    L, N = unary.shape
    assert N == height * width
    th = potts_theta(L, potts_w) if theta is None else np.asarray(theta, dtype=np.float64)
    edges = grid_edges(height, width, conn)
    ew = np.ones(edges.shape[0])
    dst, src, aw = _arcs_from_edges(edges, ew)
    return Model(unary=unary, theta=th, arc_dst=dst, arc_src=src, arc_w=aw, edges=edges, edge_w=ew)


def csr_model(unary, row_ptr, col, w, theta=None, potts_w=None):
    """General sparse graph given in CSR form: row i lists the neighbours j of node i.

    The message of node i sums ``w[e] * q[:, col[e]]`` over the entries e of
    row i.  The energy (and therefore the free energy) assumes the adjacency
    is symmetric, and takes each undirected edge from the entry with i < j.
    """
    unary = np.asarray(unary, dtype=np.float64)
    L, N = unary.shape
    th = potts_theta(L, potts_w) if theta is None else np.asarray(theta, dtype=np.float64)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    w = np.ones(col.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    dst = np.repeat(np.arange(N), np.diff(row_ptr))
    upper = dst < col
    edges = np.stack([dst[upper], col[upper]], axis=1)
    return Model(unary=unary, theta=th, arc_dst=dst, arc_src=col, arc_w=w,
                 edges=edges, edge_w=w[upper])


def gaussian_kernel(features):
    """K_ij = exp(-|f_i - f_j|^2 / 2) with K_ii = 0, in FP64 (dense CRF of Sec. 4.2).

    The zero diagonal removes the self pair from the pairwise energy.
    """
    f = np.asarray(features, dtype=np.float64)
    d2 = ((f[:, None, :] - f[None, :, :]) ** 2).sum(-1)
    K = np.exp(-0.5 * d2)
    np.fill_diagonal(K, 0.0)
    return K


def round_to_bf16(x):
    """Round FP64 values to bfloat16 (round to nearest, ties to even), returned as FP64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits
    of an IEEE binary32.  The value is first rounded to binary32 (the
    precision in which a kernel holds it), then the low 16 bits are rounded
    away with ties going to an even result.
    """
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = (bits + 0x7FFF + lsb) >> 16
    out = (rounded << 16).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def dense_model(unary, K, potts_w=None, theta=None, cooc=None):
    """Fully connected model: pairwise term K_ij * theta(x_i, x_j) for every pair i < j,
    plus an optional global co-occurrence term cooc(x_i, x_j) / N for every pair i < j.

    The paper uses co-occurrence potentials without giving a formula (Sec. 4.2,
    semantic segmentation); this global L x L term with weight 1/N is the
    reading used throughout.
    """
    unary = np.asarray(unary, dtype=np.float64)
    L, N = unary.shape
    th = potts_theta(L, potts_w) if theta is None else np.asarray(theta, dtype=np.float64)
    return Model(unary=unary, theta=th, K=np.asarray(K, dtype=np.float64),
                 cooc=None if cooc is None else np.asarray(cooc, dtype=np.float64))


# ----------------------------------------------------------------------------
# The update (Sec. 3.1-3.2)
# ----------------------------------------------------------------------------

def normalise(z):
    """Per-node log normalisation: z - logsumexp(z) over labels, max-subtracted.

    Implements the proportionality sign of Eq. 14 so that each q_i lies on
    the simplex of Eq. 4.
    """
    z = np.asarray(z)
    mx = z.max(axis=0, keepdims=True)
    return z - (mx + np.log(np.exp(z - mx).sum(axis=0, keepdims=True)))


def init_state(unary, mode=0):
    """Initial log q.  The paper does not fix q^0; mode 0 is q^0 = softmax(-u)
    (the mean field of the unaries alone), mode 1 is the uniform distribution."""
    u = np.asarray(unary)
    if mode == 0:
        return normalise(-u)
    if mode == 1:
        return np.full(u.shape, -np.log(u.shape[0]), dtype=u.dtype)
    raise ValueError(mode)


def _adjacency(model):
    """Sparse N x N matrix A with A[dst, src] = sum of the arc weights (built once)."""
    A = getattr(model, "_A", None)
    if A is None:
        N = model.unary.shape[1]
        A = scipy.sparse.csr_matrix((model.arc_w, (model.arc_dst, model.arc_src)), shape=(N, N),
                                    dtype=model.arc_w.dtype)
        model._A = A
    return A


def neighbour_sum(q, model):
    """S[:, i] = sum over neighbours j of w_ij q[:, j] (sparse) or K @ q (dense).

    The sparse case is the product with the weighted adjacency matrix.
    """
    if model.K is not None:
        return q @ model.K.T
    return np.asarray((_adjacency(model) @ q.T).T)


def pairwise_message(q, model):
    """Gradient of the pairwise part of the expected energy with respect to q.

    theta* of Eq. 15 (Sec. 3.1) minus the unary: Theta @ S_i, plus for the
    co-occurrence reading cooc @ (T - q_i) / N with T = sum_i q_i.  The
    expression is linear in q; applied to a direction v it is the
    Hessian-vector product of the expected energy (Sec. 3.2).
    """
    S = neighbour_sum(q, model)
    out = model.theta @ S
    if model.cooc is not None:
        T = q.sum(axis=1, keepdims=True)
        out = out + model.cooc @ (T - q) / q.shape[1]
    return out


def round_to_f16(x):
    """Round to IEEE binary16 (round to nearest even, via binary32), returned as FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def messages(ell, model, operand=None):
    """m = u + pairwise message at q = exp(ell): the coordinate-wise optimum
    theta* = -E_{Q/X_i}[log P] of Eq. 15 (Sec. 3.1).

    ``operand`` (optional) rounds q where it enters the neighbour aggregation,
    which is what the reduced-precision message variants compute; the
    accumulation and everything after it stay in the model's precision.
    """
    q = np.exp(ell)
    if operand is not None:
        q = operand(q)
    return model.unary + pairwise_message(q, model)


def prox_step(ell, model, alpha, operand=None):
    """One parallel KL-proximal step (Eq. 13-15, Sec. 3.1) with D = d I (Eq. 16, Sec. 3.2).

    In natural parameters theta^{t+1} = eta theta* + (1 - eta) theta^t with
    eta = alpha = 1 / (1 + d); in log space that reads
    log q^{t+1} = normalise((1 - alpha) log q^t - alpha m).
    All nodes read iteration t and write t + 1 (a Jacobi update).
    """
    m = messages(ell, model, operand)
    a = ell.dtype.type(alpha)
    return normalise((ell.dtype.type(1.0) - a) * ell - a * m)


def prox_objective(q_new_i, grad_i, q_old_i, d):
    """Per-node objective of Eq. 13: <q, grad> - H(q) + d KL(q || q^t)."""
    q = np.asarray(q_new_i)
    with np.errstate(divide="ignore", invalid="ignore"):
        neg_h = np.where(q > 0, q * np.log(q), 0.0).sum()
        kl = np.where(q > 0, q * (np.log(q) - np.log(q_old_i)), 0.0).sum()
    return float(q @ grad_i + neg_h + d * kl)


def solve(model, alpha, iters, init_mode=0, ell0=None, operand=None):
    """Run ``iters`` parallel proximal steps from q^0; return every iterate (list of [L, N]).

    The paper stops after a fixed number of iterations in practice (Sec. 3.1).
    """
    ell = init_state(model.unary, init_mode) if ell0 is None else np.asarray(ell0, dtype=model.unary.dtype)
    out = [ell]
    for _ in range(iters):
        ell = prox_step(ell, model, alpha, operand)
        out.append(ell)
    return out


def naive_parallel_step(ell, model):
    """Textbook parallel mean field: every q_i set to softmax(-m_i) at once (Sec. 2.2.2)."""
    return normalise(-messages(ell, model))


# ----------------------------------------------------------------------------
# Objective (Eq. 5 and 7, Sec. 2.2)
# ----------------------------------------------------------------------------

def energy(q, model):
    """Expected energy E(q) = sum q u + 1/2 sum_i q_i . pairwise_message_i.

    The 1/2 counts each pair once, since every pair appears in the message of
    both its ends.  Valid for symmetric adjacency and symmetric compatibility.
    """
    return float((q * model.unary).sum() + 0.5 * (q * pairwise_message(q, model)).sum())


def energy_edge_sum(q, model):
    """Expected energy as an explicit sum over pairs i < j (small problems only).

    sum_i q_i . u_i + sum_{edges} w_ij q_i^T Theta q_j (sparse), or
    sum_{i<j} [K_ij q_i^T Theta q_j + q_i^T cooc q_j / N] (dense).
    """
    e = float((q * model.unary).sum())
    if model.K is not None:
        N = q.shape[1]
        G = q.T @ model.theta @ q              # G[i, j] = q_i^T Theta q_j
        iu = np.triu_indices(N, k=1)
        e += float((model.K[iu] * G[iu]).sum())
        if model.cooc is not None:
            C = q.T @ model.cooc @ q
            e += float(C[iu].sum()) / N
        return e
    for (i, j), w in zip(model.edges, model.edge_w):
        e += float(w * (q[:, i] @ model.theta @ q[:, j]))
    return e


def entropy(ell):
    """H(q) = -sum q log q, with q = exp(ell)."""
    return float(-(np.exp(ell) * ell).sum())


def free_energy(ell, model):
    """Variational free energy F(q) = E(q) - H(q) of Eq. 7 (Sec. 2.2.1).

    F = KL(Q || P) - log Z (Eq. 5); the tables of the paper report this
    quantity under the name KL, which is why their values are negative.
    """
    q = np.exp(ell)
    return energy(q, model) - entropy(ell)


def brute_force(model, max_states=200_000):
    """Enumerate every labelling x of a tiny model.

    Returns (log Z, exact marginals [L, N], the energy of every state and the
    state array).  The energy of a state is
    sum_i u_i(x_i) + sum_{edges} w_ij Theta(x_i, x_j), plus for a dense model
    sum_{i<j} [K_ij Theta(x_i, x_j) + cooc(x_i, x_j) / N].
    """
    L, N = model.unary.shape
    n_states = L ** N
    if n_states > max_states:
        raise ValueError("too many states for enumeration")
    states = np.array(list(itertools.product(range(L), repeat=N)), dtype=np.int64)
    E = model.unary[states, np.arange(N)[None, :]].sum(axis=1)
    if model.K is not None:
        for i in range(N):
            for j in range(i + 1, N):
                E = E + model.K[i, j] * model.theta[states[:, i], states[:, j]]
                if model.cooc is not None:
                    E = E + model.cooc[states[:, i], states[:, j]] / N
    else:
        for (i, j), w in zip(model.edges, model.edge_w):
            E = E + w * model.theta[states[:, i], states[:, j]]
    mx = (-E).max()
    log_z = mx + np.log(np.exp(-E - mx).sum())
    p = np.exp(-E - log_z)
    marg = np.zeros((L, N))
    for i in range(N):
        for l in range(L):
            marg[l, i] = p[states[:, i] == l].sum()
    return log_z, marg, E, states


def kl_divergence(ell, model, bf=None):
    """KL(Q || P) by enumeration (Eq. 5): sum_x Q(x) [log Q(x) + E(x)] + log Z."""
    if bf is None:
        bf = brute_force(model)
    log_z, _, E, states = bf
    N = model.n_nodes
    logq_x = ell[states, np.arange(N)[None, :]].sum(axis=1)
    Qx = np.exp(logq_x)
    return float((Qx * (logq_x + E)).sum() + log_z)


# ----------------------------------------------------------------------------
# Sequential mean field (Eq. 8, Sec. 2.2.1)
# ----------------------------------------------------------------------------

def sweep(ell, model, n_sweeps=1, order=None):
    """SWEEP: coordinate descent, q_i <- softmax(-m_i(current q)) node by node.

    Each node sees the values already updated earlier in the same sweep
    (Gauss-Seidel).  Default order: increasing node index (raster order).
    Sparse models only; pure-Python loop over nodes.
    """
    q = np.exp(np.asarray(ell, dtype=np.float64)).copy()
    L, N = q.shape
    nbr = [[] for _ in range(N)]
    for d, s, w in zip(model.arc_dst, model.arc_src, model.arc_w):
        nbr[d].append((s, w))
    order = range(N) if order is None else order
    for _ in range(n_sweeps):
        for i in order:
            S = np.zeros(L)
            for j, w in nbr[i]:
                S += w * q[:, j]
            m = model.unary[:, i] + model.theta @ S
            z = -m - (-m).max()
            e = np.exp(z)
            q[:, i] = e / e.sum()
    with np.errstate(divide="ignore"):
        return np.log(q)


# ----------------------------------------------------------------------------
# Lipschitz constant of the gradient of E (Sec. 3.2)
# ----------------------------------------------------------------------------

def adjacency_eigs_grid(height, width, conn):
    """Eigenvalues of the adjacency of a free-boundary grid, in closed form.

    A path of n nodes has eigenvalues 2 cos(pi k / (n + 1)), k = 1..n.  The
    4-connected grid is the Cartesian product of two paths (eigenvalues add);
    the 8-connected grid is the strong product, whose adjacency is
    (A_H + I) (x) (A_W + I) - I.
    """
    a = 2 * np.cos(np.pi * np.arange(1, height + 1) / (height + 1))
    b = 2 * np.cos(np.pi * np.arange(1, width + 1) / (width + 1))
    if conn == 4:
        return (a[:, None] + b[None, :]).ravel()
    return ((1 + a[:, None]) * (1 + b[None, :]) - 1).ravel()


def tangent_compat_eigs(theta):
    """Eigenvalues of Theta restricted to the zero-sum subspace {v : 1^T v = 0}.

    Differences of points on a simplex live in that subspace, so the curvature
    of the expected energy along the feasible set only involves this block.
    """
    L = theta.shape[0]
    if L == 1:
        return np.zeros(0)
    # orthonormal basis of 1^perp: the last L - 1 left singular vectors of 1
    U, _, _ = np.linalg.svd(np.ones((L, 1)))
    B = U[:, 1:]
    return np.linalg.eigvalsh(B.T @ theta @ B)


def lipschitz_grid(height, width, conn, theta, w=1.0):
    """Largest eigenvalue of the Hessian of E (constant in the pairwise case, Sec. 3.2)
    restricted to the tangent space of the product of simplices, on a grid.

    The Hessian is (w A) (x) Theta; on the tangent space its eigenvalues are the
    products lambda(A) mu, with mu the eigenvalues of Theta on 1^perp.
    """
    lam = adjacency_eigs_grid(height, width, conn) * w
    mu = tangent_compat_eigs(np.asarray(theta, dtype=np.float64))
    if mu.size == 0:
        return 0.0
    return float(max(lam.max() * mu.max(), lam.min() * mu.min(), lam.max() * mu.min(), lam.min() * mu.max()))


def _hv_tangent(v, model):
    v = v - v.mean(axis=0, keepdims=True)
    h = pairwise_message(v, model)
    return h - h.mean(axis=0, keepdims=True)


def lipschitz_power(model, iters=3000, seed=0, v0=None, v1=None):
    """Largest tangent-space eigenvalue of the Hessian by the power method (Sec. 3.2
    and the orange lines of Fig. 2, Sec. 4.3).

    Plain power iteration on P H P gives the spectral radius rho; a second run
    on P H P + rho I gives lambda_max + rho.  Returns (lambda_max, rho).
    The start vectors are standard normal draws of default_rng(seed), in the
    order (first run, second run), unless given as v0 and v1.
    """
    rng = np.random.default_rng(seed)
    L, N = model.unary.shape
    if L == 1:
        return 0.0, 0.0

    def power(shift):
        v = rng.standard_normal((L, N)) if v1 is None else np.array(v1, dtype=np.float64)
        v -= v.mean(axis=0, keepdims=True)
        v /= np.linalg.norm(v)
        lam = 0.0
        for _ in range(iters):
            w = _hv_tangent(v, model) + shift * v
            lam = float((v * w).sum())
            nrm = np.linalg.norm(w)
            if nrm == 0.0:
                return 0.0
            v = w / nrm
        return lam

    v = rng.standard_normal((L, N)) if v0 is None else np.array(v0, dtype=np.float64)
    v -= v.mean(axis=0, keepdims=True)
    rho = 0.0
    for _ in range(iters):
        w = _hv_tangent(v, model)
        nrm = np.linalg.norm(w)
        if nrm == 0.0:
            break
        rho = nrm / np.linalg.norm(v)
        v = w / nrm
    lam_max = power(rho) - rho
    return float(lam_max), float(rho)


def admissible_alpha(lip, margin=1.01):
    """alpha = 1 / (1 + d) with d = margin * L: the convergent regime d > L (Sec. 3.2).

    A non-positive L (concave expected energy) admits alpha = 1, the fully
    parallel update (Sec. 3.2).
    """
    if lip <= 0:
        return 1.0
    return 1.0 / (1.0 + margin * lip)


# ----------------------------------------------------------------------------
# Reverse pass of T unrolled steps
# ----------------------------------------------------------------------------

def unrolled_loss(unary, theta, model_template, alpha, iters, weights, init_mode=0):
    """Loss sum(weights * q_T) after ``iters`` steps from init(unary); a scalar."""
    m = Model(unary=np.asarray(unary, dtype=np.float64), theta=np.asarray(theta, dtype=np.float64),
              arc_dst=model_template.arc_dst, arc_src=model_template.arc_src,
              arc_w=model_template.arc_w, edges=model_template.edges,
              edge_w=model_template.edge_w, K=model_template.K, cooc=model_template.cooc)
    ell = solve(m, alpha, iters, init_mode)[-1]
    return float((weights * np.exp(ell)).sum())


def adjoint(model, alpha, iters, grad_ell_T, init_mode=0):
    """Gradients of a loss with respect to the unaries and Theta through T steps.

    ``grad_ell_T`` is dLoss/d(log q_T).  Reverse of each step
    ell' = normalise((1 - alpha) ell - alpha (u + Theta S(exp ell))):
      z_bar   = g - q' * sum_l g             (normalisation)
      m_bar   = -alpha z_bar;  u_bar += m_bar;  Theta_bar += m_bar S^T
      q_bar   = S^T-adjoint of Theta^T m_bar (the neighbour sum is symmetric)
      g_prev  = (1 - alpha) z_bar + q * q_bar
    and finally through ell_0 = normalise(-u) when init_mode is 0.
    Theta_bar covers all L x L entries as they appear in m = u + Theta S.
    """
    traj = solve(model, alpha, iters, init_mode)
    g = np.asarray(grad_ell_T, dtype=np.float64).copy()
    u_bar = np.zeros_like(model.unary)
    th_bar = np.zeros_like(model.theta)
    for t in range(iters - 1, -1, -1):
        ell_t, ell_n = traj[t], traj[t + 1]
        q_t, q_n = np.exp(ell_t), np.exp(ell_n)
        z_bar = g - q_n * g.sum(axis=0, keepdims=True)
        m_bar = -alpha * z_bar
        u_bar += m_bar
        S = neighbour_sum(q_t, model)
        th_bar += m_bar @ S.T
        S_bar = model.theta.T @ m_bar
        q_bar = _neighbour_sum_transpose(S_bar, model)
        if model.cooc is not None:
            N = q_t.shape[1]
            c_bar = model.cooc.T @ m_bar / N
            q_bar = q_bar + c_bar.sum(axis=1, keepdims=True) - c_bar
        g = (1.0 - alpha) * z_bar + q_t * q_bar
    if init_mode == 0:
        q0 = np.exp(traj[0])
        u_bar += -(g - q0 * g.sum(axis=0, keepdims=True))
    return u_bar, th_bar


def _neighbour_sum_transpose(S_bar, model):
    """Adjoint of neighbour_sum: S_bar @ K (dense) or the product with A^T (sparse)."""
    if model.K is not None:
        return S_bar @ model.K
    return np.asarray((_adjacency(model).T @ S_bar.T).T)


def fd_grad(model, alpha, iters, weights, eps=1e-3, init_mode=0):
    """Central finite differences of sum(weights * q_T) in every unary and Theta entry."""
    u0, th0 = model.unary.copy(), model.theta.copy()
    gu = np.zeros_like(u0)
    gt = np.zeros_like(th0)
    for idx in np.ndindex(*u0.shape):
        up, dn = u0.copy(), u0.copy()
        up[idx] += eps
        dn[idx] -= eps
        gu[idx] = (unrolled_loss(up, th0, model, alpha, iters, weights, init_mode)
                   - unrolled_loss(dn, th0, model, alpha, iters, weights, init_mode)) / (2 * eps)
    for idx in np.ndindex(*th0.shape):
        up, dn = th0.copy(), th0.copy()
        up[idx] += eps
        dn[idx] -= eps
        gt[idx] = (unrolled_loss(u0, up, model, alpha, iters, weights, init_mode)
                   - unrolled_loss(u0, dn, model, alpha, iters, weights, init_mode)) / (2 * eps)
    return gu, gt


# ----------------------------------------------------------------------------
# Variants and baselines (Sec. 2.2.2, 3.3-3.5)
# ----------------------------------------------------------------------------

def adhoc_step(ell, model, eta):
    """ADHOC damping in mean parameters (Eq. 9, Sec. 2.2.2):
    q^{t+1} = (1 - eta) q^t + eta softmax(-m)."""
    q = np.exp(ell)
    q_star = np.exp(normalise(-messages(ell, model)))
    with np.errstate(divide="ignore"):
        return np.log((1.0 - eta) * q + eta * q_star)


def adaptive_binary_step(ell, model, d):
    """OURS-ADAPTIVE for binary variables (Eq. 19, Sec. 3.3):
    d_{i,0} = d_{i,1} = q_{i,0} q_{i,1} d, so eta_i = 1 / (1 + q_{i,0} q_{i,1} d)."""
    assert ell.shape[0] == 2
    q = np.exp(ell)
    eta = 1.0 / (1.0 + q[0] * q[1] * d)
    m = messages(ell, model)
    return normalise((1.0 - eta)[None, :] * ell - eta[None, :] * m)


def momentum_solve(model, alpha, iters, gamma1=0.95, init_mode=0, ell0=None):
    """OURS-MOMENTUM (Eq. 20-21, Sec. 3.4).

    The gradient in the proximal step is replaced by its exponential average
    mom^{t+1} = gamma1 mom^t + (1 - gamma1) m(q^t); the step then uses the
    freshly updated average (the equation as printed indexes the previous
    one; the reading here uses mom^{t+1}).  mom^0 is taken as m(q^0), so
    the first step equals the fixed-step update.
    """
    ell = init_state(model.unary, init_mode) if ell0 is None else np.asarray(ell0, dtype=np.float64)
    mom = messages(ell, model)
    out = [ell]
    for _ in range(iters):
        mom = gamma1 * mom + (1.0 - gamma1) * messages(ell, model)
        ell = normalise((1.0 - alpha) * ell - alpha * mom)
        out.append(ell)
    return out


def adam_solve(model, d, iters, gamma1=0.9, gamma2=0.999, eps=1e-8, v0=1.0, init_mode=0,
               ell0=None):
    """OURS-ADAM (Eq. 22-23, Sec. 3.5), under these readings of a garbled passage.

    * The second moment uses the standard exponential-average placement,
      v^{t+1} = gamma2 v^t + (1 - gamma2) g^2, with g the natural gradient:
      the gap between the current natural parameters and theta*, which
      vanishes at a fixed point.  In log space it is -(log q^t + m) up to a
      per-node constant; the constant is removed by centring over labels,
      and only the square enters.
    * gamma1 = 0.9, the value of the original ADAM publication that the
      paper says it follows.
    * d^t = sqrt(v^{t+1}) d + eps - 1 is clamped to stay positive, so that
      eta = 1 / (1 + d^t) lies in (0, 1].
    * The momentum average of Sec. 3.4 supplies the gradient direction.
    """
    ell = init_state(model.unary, init_mode) if ell0 is None else np.asarray(ell0, dtype=np.float64)
    mom = messages(ell, model)
    v = np.full_like(ell, v0)
    out = [ell]
    for _ in range(iters):
        m = messages(ell, model)
        mom = gamma1 * mom + (1.0 - gamma1) * m
        g = m + ell
        g = g - g.mean(axis=0, keepdims=True)
        v = gamma2 * v + (1.0 - gamma2) * g * g
        dt = np.maximum(np.sqrt(v) * d + eps - 1.0, 1e-6)
        eta = 1.0 / (1.0 + dt)
        ell = normalise((1.0 - eta) * ell - eta * mom)
        out.append(ell)
    return out
