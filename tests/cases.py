"""Test helpers: the same seeded instance handed to the oracle and to the HIP library.

Inputs come only from ``paper_1511_06103_amd.synth``; the oracle side widens
the FP32 arrays to FP64, the GPU side uploads them unchanged.
"""
import numpy as np

import oracle as O
from paper_1511_06103_amd import synth

GRAPH_NAMES = {synth.GRID4: "grid4", synth.GRID8: "grid8", synth.CSR: "csr", synth.DENSE: "dense"}


def oracle_model(inst, b=0, K=None):
    u = inst.unary[b].astype(np.float64)
    potts = inst.compat == synth.COMPAT_POTTS
    th = None if potts else inst.theta.astype(np.float64)
    pw = inst.potts_w if potts else None
    if inst.graph in (synth.GRID4, synth.GRID8):
        conn = 4 if inst.graph == synth.GRID4 else 8
        return O.grid_model(u, inst.height, inst.width, conn, theta=th, potts_w=pw)
    if inst.graph == synth.CSR:
        return O.csr_model(u, inst.row_ptr, inst.col, inst.csr_w, theta=th, potts_w=pw)
    if K is None:
        K = dense_K_f64(inst)
    cooc = None if inst.cooc is None else inst.cooc.astype(np.float64)
    return O.dense_model(u, K, potts_w=pw, theta=th, cooc=cooc)


def dense_K_f64(inst):
    """The dense instance's kernel matrix (the input both sides receive), widened to FP64."""
    bits = synth.dense_kernel_bf16(inst.features)
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dense_K_device(inst, device="cuda:0"):
    """The same kernel matrix uploaded as a bfloat16 [N, N] device tensor."""
    import torch
    bits = synth.dense_kernel_bf16(inst.features).view(np.int16)
    return torch.from_numpy(bits).to(device).view(torch.bfloat16)


def oracle_lipschitz(inst):
    potts = inst.compat == synth.COMPAT_POTTS
    th = O.potts_theta(inst.n_labels, inst.potts_w) if potts else inst.theta.astype(np.float64)
    conn = 4 if inst.graph == synth.GRID4 else 8
    return O.lipschitz_grid(inst.height, inst.width, conn, th)


def admissible_alpha(inst):
    """1 / (1 + 1.01 L) for the instance, rounded to the FP32 value the kernels use."""
    return float(np.float32(O.admissible_alpha(oracle_lipschitz(inst))))


def gpu_solver(inst, alpha=None, precision="f32", init="unary", device="cuda:0", **kw):
    import torch
    from paper_1511_06103_amd import mf
    dev = torch.device(device)
    u = torch.from_numpy(inst.unary).to(dev)
    args = dict(alpha=inst.alpha if alpha is None else alpha, precision=precision, init=init)
    if inst.compat == synth.COMPAT_POTTS:
        args["potts_w"] = inst.potts_w
    else:
        args["theta"] = torch.from_numpy(inst.theta).to(dev)
    if inst.graph in (synth.GRID4, synth.GRID8):
        args.update(height=inst.height, width=inst.width)
    elif inst.graph == synth.CSR:
        args.update(csr_row_ptr=torch.from_numpy(inst.row_ptr).to(dev),
                    csr_col=torch.from_numpy(inst.col).to(dev),
                    csr_w=None if inst.csr_w is None else torch.from_numpy(inst.csr_w).to(dev))
    else:
        if "dense_K" not in kw:
            kw["dense_K"] = dense_K_device(inst, device)
        if inst.cooc is not None:
            args["cooc"] = torch.from_numpy(inst.cooc).to(dev)
    args.update(kw)
    return mf.MeanField(u, GRAPH_NAMES[inst.graph], **args)


def max_dq(ell_a, ell_b):
    """max |exp(a) - exp(b)| in FP64."""
    return float(np.abs(np.exp(np.asarray(ell_a, np.float64)) - np.exp(np.asarray(ell_b, np.float64))).max())
