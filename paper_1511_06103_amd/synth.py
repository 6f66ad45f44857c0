"""Seeded synthetic inputs for the mean-field solver.

This module draws problem instances and nothing else: unaries, shared
pairwise compatibility matrices, graphs, dense-CRF features and request
streams.  It holds no step of the inference method (no messages, no
damping, no normalisation of q) so that the FP64 oracle and the HIP path
can both consume its output without sharing any of the method's arithmetic.

Every draw uses ``numpy.random.default_rng(seed)`` (PCG64) in FP64, in the
order documented on each function, and is then rounded to FP32: the values
a kernel receives are exactly representable, and the oracle widens the same
FP32 values back to FP64.  Scalar parameters (step size, Potts weight) are
rounded to FP32 for the same reason.

Sign convention: unaries and compatibilities are *energies*
(P(x) proportional to exp(-sum_i u_i(x_i) - sum_edges Theta(x_i, x_j))), the reading
of Eq. 2 (Sec. 2.1) combined with the natural parameters of Eq. 6 (Sec. 2.2).
Arrays are label-major: ``unary[b, l, n]`` with node index n = y * width + x.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

GRID4, GRID8, CSR, DENSE = 0, 1, 2, 3
COMPAT_GENERAL, COMPAT_POTTS = 0, 1


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def symmetric_zero_diag(rng, n_labels, low, high):
    """Draw an L x L symmetric matrix with zero diagonal.

    The strict upper triangle comes from ``uniform(low, high, (L, L))`` (one
    draw of the full square, of which only the part above the diagonal is
    kept), mirrored below the diagonal.
    """
    a = rng.uniform(low, high, (n_labels, n_labels))
    up = np.triu(a, k=1)
    return _f32(up + up.T)


def neg_log_softmax_unaries(rng, shape_labels_first, scale=2.0):
    """Unaries = -log_softmax of ``scale * standard_normal`` logits over axis 0.

    ``shape_labels_first`` is (L, ...); the label axis is the first axis.
    """
    logits = scale * rng.standard_normal(shape_labels_first)
    mx = logits.max(axis=0, keepdims=True)
    lse = mx + np.log(np.exp(logits - mx).sum(axis=0, keepdims=True))
    return _f32(-(logits - lse))


@dataclass
class Instance:
    """One (possibly batched) problem, with host FP32 arrays."""
    name: str
    graph: int
    n_labels: int
    n_nodes: int
    unary: np.ndarray                 # [B, L, N] float32
    height: int = 0
    width: int = 0
    theta: Optional[np.ndarray] = None  # [L, L] float32 (COMPAT_GENERAL)
    compat: int = COMPAT_GENERAL
    potts_w: float = 0.0
    alpha: float = 0.5
    iters: int = 1
    # CSR graphs
    row_ptr: Optional[np.ndarray] = None  # int32 [N+1]
    col: Optional[np.ndarray] = None      # int32 [nnz]
    csr_w: Optional[np.ndarray] = None    # float32 [nnz] or None
    # dense CRF
    features: Optional[np.ndarray] = None  # [N, F] float32
    cooc: Optional[np.ndarray] = None      # [L, L] float32
    extra: dict = field(default_factory=dict)

    @property
    def batch(self):
        return self.unary.shape[0]


def grid_potts_normal(seed, side, n_labels=2, conn=GRID4, w=1.0, alpha=0.5, iters=50, name=None,
                      width=None, batch=1):
    """Potts grid with iid N(0,1) unaries.

    Draw order: ``standard_normal((L, H, W))`` for a single problem, else
    ``standard_normal((B, L, H, W))``; H = side, W = width (default side).
    Potts weight ``w``.  Used for the 32 x 32, L = 2, 4-connected workload
    (seed 1) and the 3 x 3 brute-force instance (seed 11).
    """
    height = side
    width = side if width is None else width
    rng = np.random.default_rng(seed)
    shape = (n_labels, height, width) if batch == 1 else (batch, n_labels, height, width)
    u = rng.standard_normal(shape)
    return Instance(name=name or f"potts{height}x{width}L{n_labels}", graph=conn, n_labels=n_labels,
                    n_nodes=height * width, height=height, width=width,
                    unary=_f32(u.reshape(batch, n_labels, height * width)),
                    compat=COMPAT_POTTS, potts_w=float(np.float32(w)), alpha=float(np.float32(alpha)),
                    iters=iters)


def grid_theta_random(seed, height, width=None, n_labels=21, conn=GRID8, batch=1,
                      alpha=0.5, iters=100, theta_high=2.0, name=None):
    """Grid with a shared random symmetric Theta and -log_softmax unaries.

    Draw order: Theta via :func:`symmetric_zero_diag` on U[0, theta_high],
    then logits ``2 * standard_normal((batch, L, H, W))`` (the batch axis is
    dropped from the draw when batch == 1, so a single solve draws
    ``(L, H, W)``).  Used for 256 x 256 L = 21 (seed 2), the batched
    128 x 128 (seed 5), the 16 x 16 L = 3 finite-difference instance (seed
    55) and the 2048 x 2048 beyond-cache shape (seed 20).
    """
    width = height if width is None else width
    rng = np.random.default_rng(seed)
    theta = symmetric_zero_diag(rng, n_labels, 0.0, theta_high)
    if batch == 1:
        u = neg_log_softmax_unaries(rng, (n_labels, height, width)).reshape(1, n_labels, height * width)
    else:
        logits_shape = (n_labels, batch, height, width)
        u = neg_log_softmax_unaries(rng, logits_shape)            # [L, B, H, W]
        u = np.ascontiguousarray(np.transpose(u, (1, 0, 2, 3))).reshape(batch, n_labels, height * width)
    return Instance(name=name or f"grid{height}x{width}L{n_labels}", graph=conn, n_labels=n_labels,
                    n_nodes=height * width, height=height, width=width, unary=u, theta=theta,
                    compat=COMPAT_GENERAL, alpha=float(np.float32(alpha)), iters=iters)


def grid_repulsive(seed, side, w=2.0, conn=GRID8, alpha=0.5, iters=50, name=None):
    """Binary grid with a strongly repulsive coupling, Theta = -w (1 1^T - I)
    (neighbours pay -w for disagreeing), and iid N(0,1) unaries: the kind of
    model on which undamped parallel updates oscillate (the GRID benchmark's
    repulsive potentials, Sec. 4).  Draw order: ``standard_normal((2, side, side))``.
    """
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((2, side, side)).reshape(1, 2, side * side)
    theta = -float(w) * (np.ones((2, 2)) - np.eye(2))
    return Instance(name=name or f"repulsive{side}x{side}", graph=conn, n_labels=2, n_nodes=side * side,
                    height=side, width=side, unary=_f32(u), theta=_f32(theta), compat=COMPAT_GENERAL,
                    alpha=float(np.float32(alpha)), iters=iters)


def workload_c1():
    """32 x 32, 4-connected, L = 2, Potts w = 1, N(0,1) unaries, alpha 0.5, 50 iterations."""
    return grid_potts_normal(1, 32, 2, GRID4, 1.0, 0.5, 50, name="grid32_L2_potts")


def workload_3x3():
    """3 x 3, 4-connected, L = 2 Potts instance small enough for enumeration (512 states)."""
    return grid_potts_normal(11, 3, 2, GRID4, 1.0, 0.5, 50, name="grid3_L2_potts")


def workload_c2(side=256):
    """256 x 256, 8-connected, L = 21, random Theta U[0,2], alpha 0.5, 100 iterations."""
    return grid_theta_random(2, side, side, 21, GRID8, 1, 0.5, 100, name=f"grid{side}_L21_theta")


def workload_big():
    """2048 x 2048, 8-connected, L = 21: a state larger than the 256 MB last-level cache."""
    return grid_theta_random(20, 2048, 2048, 21, GRID8, 1, 0.5, 20, name="grid2048_L21_theta")


def workload_large_labels(side=512, n_labels=128):
    """512 x 512, 8-connected, L = 128, the 256 x 256 recipe (random Theta
    U[0,2], -log_softmax unaries, alpha 0.5) with many labels: Theta S is a
    real dense contraction; 20 iterations.  Its three arrays of a step
    (400 MB) exceed the 256 MB last-level cache."""
    return grid_theta_random(30, side, side, n_labels, GRID8, 1, 0.5, 20, name=f"grid{side}_L{n_labels}_theta")


def workload_c5():
    """Batch of 16 grids 128 x 128, 8-connected, L = 21, T = 10 unrolled steps."""
    return grid_theta_random(5, 128, 128, 21, GRID8, 16, 0.5, 10, name="batch16_grid128_L21")


def workload_fd():
    """16 x 16, 8-connected, L = 3: the finite-difference instance of the adjoint."""
    return grid_theta_random(55, 16, 16, 3, GRID8, 1, 0.5, 10, name="grid16_L3_fd")


def adjoint_loss_weights(seed, shape):
    """Loss weights c ~ N(0,1) for the loss sum(c * q_T), drawn after a fresh seed."""
    rng = np.random.default_rng(seed)
    return _f32(rng.standard_normal(shape))


def dense_instance(seed, n_nodes=4096, n_labels=21, pos_high=64.0, alpha=0.5, iters=50,
                   potts_w=1.0, with_cooc=True, name=None):
    """Fully connected CRF with Gaussian-kernel features.

    Draw order: positions ``uniform(0, pos_high, (N, 2))``, colours
    ``uniform(0, 1, (N, 3))``, co-occurrence matrix via
    :func:`symmetric_zero_diag` on U[0,1], logits
    ``2 * standard_normal((N, L))`` (node-major draw, stored label-major).
    The kernel matrix is built from the features by :func:`dense_kernel_bf16`
    (an input of the solver like the unaries); the library can also build it
    on the device (``mf_dense_kernel``), which its own tests compare with
    the oracle's kernel.
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, pos_high, (n_nodes, 2))
    col = rng.uniform(0.0, 1.0, (n_nodes, 3))
    cooc = symmetric_zero_diag(rng, n_labels, 0.0, 1.0)
    logits = 2.0 * rng.standard_normal((n_nodes, n_labels))
    mx = logits.max(axis=1, keepdims=True)
    lse = mx + np.log(np.exp(logits - mx).sum(axis=1, keepdims=True))
    u = _f32(-(logits - lse).T).reshape(1, n_labels, n_nodes)
    feats = _f32(np.concatenate([pos, col], axis=1))
    return Instance(name=name or f"dense{n_nodes}_L{n_labels}", graph=DENSE, n_labels=n_labels,
                    n_nodes=n_nodes, unary=u, compat=COMPAT_POTTS, potts_w=float(np.float32(potts_w)),
                    alpha=float(np.float32(alpha)), iters=iters, features=feats,
                    cooc=cooc if with_cooc else None)


def dense_kernel_bf16(features):
    """Bits of the dense CRF's kernel matrix as the solver receives it:
    K_ij = exp(-|f_i - f_j|^2 / 2) computed in FP64 from the FP32 features,
    K_ii = 0, rounded to FP32 and then to bfloat16 with ties to even.
    Returns uint16 [N, N] (row-major)."""
    f = np.asarray(features, dtype=np.float64)
    n = f.shape[0]
    d2 = np.empty((n, n))
    for r0 in range(0, n, 512):      # squared distances, a block of rows at a time
        blk = f[r0:r0 + 512, None, :] - f[None, :, :]
        d2[r0:r0 + 512] = (blk * blk).sum(-1)
    k = np.exp(-0.5 * d2)
    np.fill_diagonal(k, 0.0)
    bits = k.astype(np.float32).view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
    return np.ascontiguousarray(bits.astype(np.uint16))


def workload_c3():
    """N = 4096, L = 21 fully connected CRF with co-occurrence, 50 iterations."""
    return dense_instance(3, 4096, 21, 64.0, 0.5, 50, 1.0, True, name="dense4096_L21_cooc")


def power_start_vectors(seed, n_labels, n_nodes):
    """Start vectors of the two power-method runs, [L, N] each, standard
    normal in FP64 from default_rng(seed) in the order (v0, v1), rounded to
    FP32 (the values both the device and the oracle start from)."""
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal((n_labels, n_nodes))
    v1 = rng.standard_normal((n_labels, n_nodes))
    return _f32(v0), _f32(v1)


def random_csr_graph(rng, n_nodes, avg_degree, weighted=True):
    """Symmetric random graph in CSR form (rows sorted, no self loops, no duplicates).

    Draws ``n_nodes * avg_degree // 2`` candidate edges as pairs of
    ``integers(0, n_nodes)``; self loops and duplicates are dropped; weights
    (if any) are ``uniform(0.5, 1.5)`` per undirected edge.
    """
    m = max(1, n_nodes * avg_degree // 2)
    a = rng.integers(0, n_nodes, m)
    b = rng.integers(0, n_nodes, m)
    keep = a != b
    a, b = a[keep], b[keep]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo.astype(np.int64) * n_nodes + hi)
    lo, hi = key // n_nodes, key % n_nodes
    w_und = rng.uniform(0.5, 1.5, lo.shape[0]) if weighted else np.ones(lo.shape[0])
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    ww = np.concatenate([w_und, w_und])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return (row_ptr.astype(np.int32), dst.astype(np.int32),
            _f32(ww) if weighted else None)


def csr_instance(seed, n_nodes, n_labels, avg_degree=6, weighted=True, alpha=0.5, iters=20,
                 batch=1, name=None):
    """General sparse graph, shared random Theta, -log_softmax unaries.

    Draw order: graph (:func:`random_csr_graph`), Theta U[0,2], logits
    ``2 * standard_normal((batch, L, N))``.
    """
    rng = np.random.default_rng(seed)
    row_ptr, col, w = random_csr_graph(rng, n_nodes, avg_degree, weighted)
    theta = symmetric_zero_diag(rng, n_labels, 0.0, 2.0)
    u = neg_log_softmax_unaries(rng, (n_labels, batch, n_nodes))
    u = np.ascontiguousarray(np.transpose(u, (1, 0, 2)))
    return Instance(name=name or f"csr{n_nodes}_L{n_labels}", graph=CSR, n_labels=n_labels,
                    n_nodes=n_nodes, unary=u, theta=theta, compat=COMPAT_GENERAL,
                    alpha=float(np.float32(alpha)),
                    iters=iters, row_ptr=row_ptr, col=col, csr_w=w)


def grid_csr_graph(height, width, conn=GRID8):
    """The free-boundary grid of :func:`grid_theta_random` as a CSR graph in
    raster node order (n = y * width + x), rows sorted, unit weights (none
    stored): a general graph with the locality of a grid."""
    ys, xs = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    ys, xs = ys.ravel(), xs.ravel()
    offs = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
    if conn == GRID4:
        offs = [(-1, 0), (0, -1), (0, 1), (1, 0)]
    cols = []
    valid = []
    for dy, dx in offs:                       # in this order the columns of a row are sorted
        yy, xx = ys + dy, xs + dx
        valid.append((yy >= 0) & (yy < height) & (xx >= 0) & (xx < width))
        cols.append(yy * width + xx)
    cols = np.stack(cols, 1)
    valid = np.stack(valid, 1)
    row_ptr = np.concatenate([[0], np.cumsum(valid.sum(1))]).astype(np.int32)
    return row_ptr, np.ascontiguousarray(cols[valid].astype(np.int32))


def grid_as_csr(inst):
    """A grid instance of :func:`grid_theta_random` re-expressed as a CSR
    instance: the same unaries, Theta and step size on the same graph."""
    row_ptr, col = grid_csr_graph(inst.height, inst.width, inst.graph)
    return Instance(name=f"csr_{inst.name}", graph=CSR, n_labels=inst.n_labels, n_nodes=inst.n_nodes,
                    unary=inst.unary, theta=inst.theta, compat=inst.compat, potts_w=inst.potts_w,
                    alpha=inst.alpha, iters=inst.iters, row_ptr=row_ptr, col=col, csr_w=None)


@dataclass
class Request:
    index: int
    arrival_s: float
    side: int
    n_labels: int
    seed: int


def serving_trace(seed=4, n_requests=512, rate_per_s=200.0, side_lo=64, side_hi=512):
    """Poisson request stream of square 8-connected grids.

    Draw order: inter-arrival gaps ``exponential(1/rate, n)``, sides
    ``integers(side_lo, side_hi, n, endpoint=True)``, label counts
    ``choice([2, 21], n)``.  Request k carries seed 4000 + k for its own
    Theta and unaries (:func:`serving_request_instance`).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    sides = rng.integers(side_lo, side_hi, n_requests, endpoint=True)
    labels = rng.choice(np.array([2, 21]), n_requests)
    arrivals = np.cumsum(gaps)
    return [Request(k, float(arrivals[k]), int(sides[k]), int(labels[k]), 4000 + k)
            for k in range(n_requests)]


def serving_request_instance(req: Request, alpha=0.5, iters=100):
    """The grid problem of one request: Theta U[0,2] and -log_softmax unaries, 8-connected."""
    return grid_theta_random(req.seed, req.side, req.side, req.n_labels, GRID8, 1, alpha, iters,
                             name=f"req{req.index}")
