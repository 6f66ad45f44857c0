"""Python binding of libmf.so (include/mf.h) over PyTorch device tensors.

Argument marshalling only: every step of the inference runs in the HIP
library.  PyTorch supplies device memory and the HIP stream.  There is no
CPU fallback: if the library is not built, or is used without a GPU, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

MF_ABI_VERSION = 4
MF_MAX_LABELS = 128   # grids with the fixed-step rule; 32 elsewhere
MF_SMALL_LABELS = 32
MF_STATIC_SCRATCH_BYTES = 64 << 20   # scratch array of mf_solve_static, per GPU
MF_PERSIST_STEPS_PER_LAUNCH = 4096   # steps per launch reported for the persistent grid kernel
MF_MAX_LABEL_NODES = 1 << 30   # n_labels * n_nodes of one problem must stay below this

MF_OK, MF_EINVAL, MF_ENONFINITE, MF_EDEVICE, MF_EUNSUPPORTED, MF_ENOWORKSPACE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "MF_OK", -1: "MF_EINVAL", -2: "MF_ENONFINITE", -3: "MF_EDEVICE",
                -4: "MF_EUNSUPPORTED", -5: "MF_ENOWORKSPACE"}

GRID4, GRID8, CSR, DENSE = 0, 1, 2, 3
COMPAT_GENERAL, COMPAT_POTTS = 0, 1
PRECISIONS = {"f32": 0, "bf16": 1, "f16": 2}
INIT_MODES = {"unary": 0, "uniform": 1, "state": 2}
RULES = {"fixed": 0, "adaptive": 1, "adhoc": 2, "momentum": 3, "adam": 4, "sweep": 5}


class MFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class MFDesc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("batch", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
        ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("n_labels", ctypes.c_int32),
        ("graph", ctypes.c_int32), ("compat", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("init", ctypes.c_int32), ("alpha", ctypes.c_double), ("potts_w", ctypes.c_float),
        ("steps_per_launch", ctypes.c_int32),
        ("rule", ctypes.c_int32), ("rule_gamma1", ctypes.c_float), ("rule_gamma2", ctypes.c_float),
        ("rule_eps", ctypes.c_float), ("rule_v0", ctypes.c_float),
        ("csr_row_ptr", ctypes.c_void_p), ("csr_col", ctypes.c_void_p), ("csr_w", ctypes.c_void_p),
        ("csr_nnz", ctypes.c_int64),
        ("dense_K", ctypes.c_void_p), ("cooc", ctypes.c_void_p),
        ("unary", ctypes.c_void_p), ("theta", ctypes.c_void_p), ("state", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("csr_lanes", ctypes.c_int32),
    ]


# name -> (restype, argtypes); every symbol include/mf.h declares
SIGNATURES = {
    "mf_abi_version": (ctypes.c_int32, []),
    "mf_desc_size": (ctypes.c_size_t, []),
    "mf_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(MFDesc)]),
    "mf_validate": (ctypes.c_int, [ctypes.POINTER(MFDesc)]),
    "mf_init": (ctypes.c_int, [ctypes.POINTER(MFDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "mf_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mf_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mf_free_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "mf_check": (ctypes.c_int, [ctypes.c_void_p]),
    "mf_marginals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mf_current_state": (ctypes.c_void_p, [ctypes.c_void_p]),
    "mf_iteration": (ctypes.c_int32, [ctypes.c_void_p]),
    "mf_steps_per_launch": (ctypes.c_int32, [ctypes.c_void_p]),
    "mf_destroy": (None, [ctypes.c_void_p]),
    "mf_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "mf_dense_kernel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "mf_step_many": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.c_int32]),
    "mf_backward_workspace_size": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int32]),
    "mf_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t]),
    "mf_lipschitz_workspace_size": (ctypes.c_size_t, [ctypes.c_void_p]),
    "mf_lipschitz": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    "mf_admissible_alpha": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
    "mf_solve_static": (ctypes.c_int, [ctypes.POINTER(MFDesc), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
}

_lib = None


def lib():
    """Load libmf.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1511_06103_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.mf_abi_version() != MF_ABI_VERSION:
            raise RuntimeError("libmf.so ABI version mismatch")
        if L.mf_desc_size() != ctypes.sizeof(MFDesc):
            raise RuntimeError("mf_desc layout mismatch between the binding and libmf.so")
        _lib = L
    return _lib


def admissible_alpha(lipschitz: float, margin: float = 1.01) -> float:
    """alpha = 1 / (1 + margin * L-hat) (mf_admissible_alpha)."""
    return float(lib().mf_admissible_alpha(float(lipschitz), float(margin)))


def last_error(handle=None):
    msg = lib().mf_last_error(handle)
    return msg.decode() if msg else ""


def _check(status, handle=None):
    if status != MF_OK:
        raise MFError(status, last_error(handle))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_tensor(t, dtype, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def dense_kernel(features: torch.Tensor, stream=None) -> torch.Tensor:
    """K_ij = exp(-|f_i - f_j|^2 / 2), K_ii = 0, rounded to bfloat16, built on the GPU."""
    f = _dev_tensor(features, torch.float32, "features", None)
    n, dim = f.shape
    K = torch.empty((n, n), dtype=torch.bfloat16, device=f.device)
    s = torch.cuda.current_stream(f.device).cuda_stream if stream is None else stream
    _check(lib().mf_dense_kernel(_ptr(f), n, dim, _ptr(K), ctypes.c_void_p(s)))
    return K


def step_many(solvers, n_steps=1):
    """Advance solver i by n_steps[i] steps (one int: the same for all) in
    shared launches (continuous batching, mf_step_many)."""
    solvers = list(solvers)
    if not solvers:
        return
    counts = [int(n_steps)] * len(solvers) if np.isscalar(n_steps) else [int(k) for k in n_steps]
    if len(counts) != len(solvers):
        raise ValueError("one step count per solver")
    arr = (ctypes.c_void_p * len(solvers))(*[s._h().value for s in solvers])
    cnt = (ctypes.c_int32 * len(solvers))(*counts)
    st = lib().mf_step_many(arr, cnt, len(solvers))
    if st != MF_OK:
        raise MFError(st, last_error())


def solve_static(desc: MFDesc, iters: int, q_out: Optional[torch.Tensor] = None,
                 F_out: Optional[torch.Tensor] = None, flags_out: Optional[torch.Tensor] = None):
    """mf_solve_static: initialise, run ``iters`` steps, write q into q_out
    ([B, L, N] float32) and the FP64 free energy into F_out ([B] float64),
    with the library's static device scratch as the workspace, so that the
    call allocates nothing.  flags_out (int32 [1]) receives the deferred
    error bits.  Every array stays the caller's; ``desc`` is an MFDesc
    (e.g. MeanField.descriptor()).  Asynchronous on desc.stream."""
    for t, dt, name in ((q_out, torch.float32, "q_out"), (F_out, torch.float64, "F_out"),
                        (flags_out, torch.int32, "flags_out")):
        if t is not None:
            _dev_tensor(t, dt, name, None)
    _check(lib().mf_solve_static(ctypes.byref(desc), int(iters), _ptr(q_out), _ptr(F_out), _ptr(flags_out)))


class MeanField:
    """One (batched) mean-field problem bound to device tensors.

    ``unary``: [B, L, N] float32 energies.  ``graph``: "grid4", "grid8",
    "csr" or "dense".  Either ``theta`` ([L, L] float32) or ``potts_w``.
    ``alpha`` = 1 / (1 + d).  The state ([2, B, L, N] float32) and the
    workspace are allocated here as torch tensors and owned by this object.
    """

    GRAPHS = {"grid4": GRID4, "grid8": GRID8, "csr": CSR, "dense": DENSE}

    def __init__(self, unary: torch.Tensor, graph: str, *, height: int = 0, width: int = 0,
                 theta: Optional[torch.Tensor] = None, potts_w: Optional[float] = None,
                 alpha: float = 0.5, precision: str = "f32", init: str = "unary",
                 csr_row_ptr: Optional[torch.Tensor] = None, csr_col: Optional[torch.Tensor] = None,
                 csr_w: Optional[torch.Tensor] = None, dense_K: Optional[torch.Tensor] = None,
                 cooc: Optional[torch.Tensor] = None, state: Optional[torch.Tensor] = None,
                 stream: Optional[torch.cuda.Stream] = None, steps_per_launch: int = 0,
                 rule: str = "fixed", gamma1: Optional[float] = None, gamma2: float = 0.999,
                 eps: float = 1e-8, v0: float = 1.0, csr_lanes: int = 0):
        L_ = lib()
        self._handle = None
        u = _dev_tensor(unary, torch.float32, "unary", None)
        dev = u.device
        if u.dim() == 2:
            u = u.unsqueeze(0)
        if u.dim() != 3:
            raise ValueError("unary must be [B, L, N]")
        B, Lb, N = u.shape
        self.device = dev
        self.shape = (B, Lb, N)
        self.unary = u
        self.theta = None if theta is None else _dev_tensor(theta, torch.float32, "theta", dev)
        self.cooc = None if cooc is None else _dev_tensor(cooc, torch.float32, "cooc", dev)
        self.csr = tuple(None if t is None else _dev_tensor(t, dt, nm, dev) for t, dt, nm in
                         ((csr_row_ptr, torch.int32, "csr_row_ptr"), (csr_col, torch.int32, "csr_col"),
                          (csr_w, torch.float32, "csr_w")))
        self.dense_K = None if dense_K is None else _dev_tensor(dense_K, torch.bfloat16, "dense_K", dev)
        if state is None:
            state = torch.empty((2, B, Lb, N), dtype=torch.float32, device=dev)
        self.state_buf = _dev_tensor(state, torch.float32, "state", dev)
        if tuple(self.state_buf.shape) != (2, B, Lb, N):
            raise ValueError("state must be [2, B, L, N]")
        if graph not in self.GRAPHS:
            raise ValueError(f"unknown graph {graph!r}")
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        d = MFDesc()
        d.abi_version = MF_ABI_VERSION
        d.batch, d.n_nodes, d.n_labels = B, N, Lb
        d.height, d.width = height, width
        d.graph = self.GRAPHS[graph]
        d.compat = COMPAT_GENERAL if potts_w is None else COMPAT_POTTS
        d.precision = PRECISIONS[precision]
        d.init = INIT_MODES[init]
        d.alpha = float(alpha)
        d.potts_w = 0.0 if potts_w is None else float(potts_w)
        d.steps_per_launch = int(steps_per_launch)
        d.csr_lanes = int(csr_lanes)
        if rule not in RULES:
            raise ValueError(f"unknown step rule {rule!r}")
        d.rule = RULES[rule]
        # momentum decay: 0.95 for OURS-MOMENTUM and 0.9 for OURS-ADAM (Sec. 4.1)
        d.rule_gamma1 = float(gamma1 if gamma1 is not None else (0.9 if rule == "adam" else 0.95))
        d.rule_gamma2, d.rule_eps, d.rule_v0 = float(gamma2), float(eps), float(v0)
        d.csr_row_ptr, d.csr_col, d.csr_w = (_ptr(t) for t in self.csr)
        d.csr_nnz = 0 if self.csr[1] is None else self.csr[1].numel()
        d.dense_K = _ptr(self.dense_K)
        d.cooc = _ptr(self.cooc)
        d.unary = _ptr(u)
        d.theta = _ptr(self.theta)
        d.state = _ptr(self.state_buf)
        d.stream = ctypes.c_void_p(self.stream.cuda_stream)
        ws = L_.mf_workspace_size(ctypes.byref(d))
        if ws == 0:
            _check(L_.mf_validate(ctypes.byref(d)))
            raise MFError(MF_EINVAL, "invalid descriptor")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=dev)
        d.workspace = _ptr(self.workspace)
        d.workspace_bytes = ws
        self.desc = d
        caller = torch.cuda.current_stream(dev)
        if self.stream != caller:
            # the inputs were produced on the caller's stream; the buffers this
            # object owns are used on its own stream from now on
            self.stream.wait_stream(caller)
            for t in (self.workspace, self.state_buf):
                t.record_stream(self.stream)
        h = ctypes.c_void_p()
        _check(L_.mf_init(ctypes.byref(d), ctypes.byref(h)))
        self._handle = h

    def descriptor(self, state: Optional[torch.Tensor] = None) -> MFDesc:
        """A copy of this problem's mf_desc with no workspace (for
        solve_static), on ``state`` ([2, B, L, N] float32) if given."""
        d = MFDesc()
        ctypes.pointer(d)[0] = self.desc
        if state is not None:
            _dev_tensor(state, torch.float32, "state", self.device)
            if tuple(state.shape) != (2,) + self.shape:
                raise ValueError("state must be [2, B, L, N]")
            d.state = _ptr(state)
        d.workspace = None
        d.workspace_bytes = 0
        return d

    # -- calls ------------------------------------------------------------
    def _h(self):
        if self._handle is None:
            raise RuntimeError("solver is closed")
        return self._handle

    def step(self, n: int = 1):
        _check(lib().mf_step(self._h(), int(n)), self._handle)
        return self

    def solve(self, iters: int, q_out: Optional[torch.Tensor] = None):
        if q_out is not None:
            _dev_tensor(q_out, torch.float32, "q_out", self.device)
            if tuple(q_out.shape) != self.shape:
                raise ValueError("q_out must be [B, L, N]")
        _check(lib().mf_solve(self._h(), int(iters), _ptr(q_out)), self._handle)
        return q_out

    def marginals(self, q_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """q = exp(log q) of the current state, written by the library into q_out [B, L, N]."""
        if q_out is None:
            q_out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _dev_tensor(q_out, torch.float32, "q_out", self.device)
        if tuple(q_out.shape) != self.shape:
            raise ValueError("q_out must be [B, L, N]")
        _check(lib().mf_marginals(self._h(), _ptr(q_out)), self._handle)
        return q_out

    def free_energy(self) -> np.ndarray:
        out = (ctypes.c_double * self.shape[0])()
        _check(lib().mf_free_energy(self._h(), out), self._handle)
        return np.array(out[:], dtype=np.float64)

    def backward(self, ckpt_states: torch.Tensor, iters: int, ckpt_every: int, grad_logq_T: torch.Tensor):
        """Reverse pass of ``iters`` steps: returns (dLoss/du [B, L, N], dLoss/dTheta [L, L])."""
        B, L, N = self.shape
        n_ckpt = (iters + ckpt_every - 1) // ckpt_every
        _dev_tensor(ckpt_states, torch.float32, "ckpt_states", self.device)
        _dev_tensor(grad_logq_T, torch.float32, "grad_logq_T", self.device)
        if ckpt_states.shape[0] < n_ckpt or tuple(ckpt_states.shape[1:]) != self.shape:
            raise ValueError("ckpt_states must be [ceil(iters / ckpt_every), B, L, N]")
        if tuple(grad_logq_T.shape) != self.shape:
            raise ValueError("grad_logq_T must be [B, L, N]")
        nbytes = lib().mf_backward_workspace_size(self._h(), int(ckpt_every))
        if nbytes == 0:
            _check(MF_EUNSUPPORTED if self.desc.graph not in (GRID4, GRID8) else MF_EINVAL, self._handle)
        work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        gu = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        gt = torch.empty((L, L), dtype=torch.float32, device=self.device)
        _check(lib().mf_backward(self._h(), _ptr(ckpt_states), int(iters), int(ckpt_every), _ptr(grad_logq_T),
                                 _ptr(gu), _ptr(gt), _ptr(work), nbytes), self._handle)
        self._bwd_work = work    # keep alive until the stream has consumed it
        return gu, gt

    def lipschitz(self, v0: torch.Tensor, v1: torch.Tensor, iters: int = 3000):
        """Tangent-space Lipschitz constant by the power method (mf_lipschitz).

        v0, v1: device [L, N] FP32 start vectors of the two runs.  Returns
        (lambda_max, rho): the largest eigenvalue and the spectral radius."""
        _, L, N = self.shape
        for name, v in (("v0", v0), ("v1", v1)):
            _dev_tensor(v, torch.float32, name, self.device)
            if tuple(v.shape) != (L, N):
                raise ValueError(f"{name} must be [L, N]")
        nbytes = lib().mf_lipschitz_workspace_size(self._h())
        work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        lam, rho = ctypes.c_double(), ctypes.c_double()
        _check(lib().mf_lipschitz(self._h(), int(iters), _ptr(v0), _ptr(v1), _ptr(work), nbytes,
                                  ctypes.byref(lam), ctypes.byref(rho)), self._handle)
        return lam.value, rho.value

    def check(self):
        _check(lib().mf_check(self._h()), self._handle)

    @property
    def iteration(self) -> int:
        return int(lib().mf_iteration(self._h()))

    @property
    def steps_per_launch(self) -> int:
        return int(lib().mf_steps_per_launch(self._h()))

    def current_index(self) -> int:
        p = lib().mf_current_state(self._h())
        return 0 if p == self.state_buf[0].data_ptr() else 1

    def current_state(self) -> torch.Tensor:
        """View of the current log q, [B, L, N]."""
        return self.state_buf[self.current_index()]

    def close(self):
        if self._handle is not None:
            lib().mf_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
