"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
rejects invalid descriptors on the host before any launch.  No compute call
is made (there is no GPU here); fake device addresses are only ever passed to
host-side validation."""
import ctypes
import os
import re

import pytest

from paper_1511_06103_amd import mf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")

pytestmark = pytest.mark.skipif(not os.path.exists(mf.LIB_PATH), reason="libmf.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for core in ("mf_init", "mf_step", "mf_solve", "mf_free_energy", "mf_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(mf.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert sorted(mf.SIGNATURES) == declared_functions()


def test_abi_version_and_descriptor_layout():
    L = mf.lib()
    assert L.mf_abi_version() == mf.MF_ABI_VERSION
    assert L.mf_desc_size() == ctypes.sizeof(mf.MFDesc)


FAKE = 0x7F0000000000   # never dereferenced: validation is host-only


def good_desc(**kw):
    d = mf.MFDesc()
    d.abi_version = mf.MF_ABI_VERSION
    d.batch, d.n_nodes, d.n_labels = 1, 64 * 64, 21
    d.height, d.width = 64, 64
    d.graph = mf.GRID8
    d.compat = mf.COMPAT_GENERAL
    d.precision = 0
    d.init = 0
    d.alpha = 0.5
    d.unary = FAKE
    d.theta = FAKE + (1 << 30)
    d.state = FAKE + (1 << 32)
    for k, v in kw.items():
        setattr(d, k, v)
    ws = mf.lib().mf_workspace_size(ctypes.byref(d))
    if "workspace" not in kw:
        d.workspace = FAKE + (1 << 34)
        d.workspace_bytes = ws
    return d


def validate(d):
    return mf.lib().mf_validate(ctypes.byref(d))


def test_valid_descriptor_passes():
    assert validate(good_desc()) == mf.MF_OK
    assert validate(good_desc(compat=mf.COMPAT_POTTS, theta=None, potts_w=1.0)) == mf.MF_OK
    assert validate(good_desc(alpha=1.0)) == mf.MF_OK           # fully parallel
    assert validate(good_desc(n_labels=1)) == mf.MF_OK          # trivial but legal


@pytest.mark.parametrize("field,value", [
    ("alpha", 0.0), ("alpha", -0.1), ("alpha", 1.5), ("alpha", float("nan")),
    ("n_labels", 0), ("batch", 0), ("n_nodes", 0),
    ("height", 63), ("width", 0),
    ("graph", 7), ("compat", 5), ("precision", 9), ("init", 3),
    ("unary", None), ("state", None), ("theta", None),
    ("abi_version", 99),
    ("potts_w", float("inf")),
])
def test_invalid_descriptor_rejected(field, value):
    d = good_desc()
    setattr(d, field, value)
    st = validate(d)
    assert st == mf.MF_EINVAL, (field, value, st)
    assert mf.last_error() != ""


def test_misaligned_pointer_rejected():
    assert validate(good_desc(unary=FAKE + 2)) == mf.MF_EINVAL


def test_state_overlapping_unary_rejected():
    d = good_desc()
    d.unary = d.state + 4 * 64 * 64 * 21   # inside the second state buffer
    assert validate(d) == mf.MF_EINVAL


def test_too_many_labels_unsupported():
    assert validate(good_desc(n_labels=mf.MF_MAX_LABELS + 1)) == mf.MF_EUNSUPPORTED


def test_label_node_limit():
    """One problem's L * N must stay below 2^30 (32-bit byte offsets in the kernels)."""
    far = dict(state=FAKE + (1 << 36), workspace=FAKE + (1 << 38), workspace_bytes=1 << 40)
    ok = good_desc(n_labels=1, height=32767, width=32769, n_nodes=32767 * 32769, **far)
    assert validate(ok) == mf.MF_OK
    big = good_desc(n_labels=32, height=8192, width=4096, n_nodes=8192 * 4096, **far)
    assert validate(big) == mf.MF_EUNSUPPORTED
    assert "MF_MAX_LABEL_NODES" in mf.last_error()


def test_workspace_checks():
    d = good_desc()
    need = mf.lib().mf_workspace_size(ctypes.byref(d))
    assert need > 0
    d.workspace_bytes = need - 1
    assert validate(d) == mf.MF_ENOWORKSPACE
    d.workspace_bytes = need
    d.workspace = None
    assert validate(d) == mf.MF_ENOWORKSPACE
    d.workspace = FAKE + 8
    assert validate(d) == mf.MF_EINVAL       # not 256-byte aligned


def test_workspace_size_zero_for_invalid():
    d = good_desc()
    d.batch = 0
    assert mf.lib().mf_workspace_size(ctypes.byref(d)) == 0


def test_init_rejects_before_launch():
    L = mf.lib()
    h = ctypes.c_void_p(1234)
    d = good_desc(alpha=2.0)
    assert L.mf_init(ctypes.byref(d), ctypes.byref(h)) == mf.MF_EINVAL
    assert not h.value
    assert "alpha" in mf.last_error()
    assert L.mf_init(None, ctypes.byref(h)) == mf.MF_EINVAL
    assert L.mf_step(None, 1) == mf.MF_EINVAL
    assert L.mf_solve(None, 1, None) == mf.MF_EINVAL
    assert L.mf_check(None) == mf.MF_EINVAL
    assert L.mf_current_state(None) is None
    assert L.mf_iteration(None) == -1
    L.mf_destroy(None)     # no-op


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises(ValueError, match="GPU tensor"):
        mf.MeanField(torch.zeros(1, 2, 9), "grid4", height=3, width=3, potts_w=1.0)


def csr_desc(**kw):
    base = dict(graph=mf.CSR, height=0, width=0, csr_row_ptr=FAKE + (1 << 36), csr_col=FAKE + (1 << 37),
                csr_nnz=1000)
    base.update(kw)
    return good_desc(**base)


def test_csr_gathered_rows_limit():
    """General graphs: the node-major q rows (N x LQ floats, LQ = 24 for
    L = 17) must stay below 4 GiB, besides L * N < 2^30."""
    far = dict(state=FAKE + (1 << 40), workspace=FAKE + (1 << 42), workspace_bytes=1 << 44)
    n_ok, n_big = 40 << 20, 50 << 20          # 40 Mi x 96 B < 4 GiB <= 50 Mi x 96 B; L N < 2^30 for both
    assert validate(csr_desc(n_labels=17, n_nodes=n_ok, **far)) == mf.MF_OK
    assert validate(csr_desc(n_labels=17, n_nodes=n_big, **far)) == mf.MF_EUNSUPPORTED
    assert "2^32" in mf.last_error()


def test_csr_descriptor_validation():
    assert validate(csr_desc()) == mf.MF_OK
    for lanes, want in ((0, mf.MF_OK), (1, mf.MF_OK), (2, mf.MF_OK), (3, mf.MF_EINVAL), (-1, mf.MF_EINVAL)):
        assert validate(csr_desc(csr_lanes=lanes)) == want, lanes
    assert validate(csr_desc(csr_w=FAKE + (1 << 38))) == mf.MF_OK
    assert validate(csr_desc(csr_nnz=0, csr_col=None)) == mf.MF_OK      # no edges
    assert validate(csr_desc(csr_row_ptr=None)) == mf.MF_EINVAL
    assert validate(csr_desc(csr_col=None)) == mf.MF_EINVAL
    assert validate(csr_desc(csr_nnz=-1)) == mf.MF_EINVAL
    assert validate(csr_desc(csr_nnz=1 << 33)) == mf.MF_EINVAL
    assert validate(csr_desc(csr_col=FAKE + (1 << 37) + 2)) == mf.MF_EINVAL


def test_csr_workspace_holds_node_major_q():
    g = mf.lib().mf_workspace_size(ctypes.byref(good_desc(steps_per_launch=1)))
    c = mf.lib().mf_workspace_size(ctypes.byref(csr_desc()))
    # two node-major copies of q, L = 21 padded to 24
    assert c - g >= 2 * 64 * 64 * 24 * 4


def test_workspace_holds_halo_exchange_of_small_theta_grids():
    """Grids the persistent kernel may take (library-chosen launch shape,
    general Theta, 8 < L <= 32, at most 256 tiles of 16 x 16) carry its
    exchange area: two slots of 64 tagged 8-byte words per label and tile."""
    def ws(**kw):
        return mf.lib().mf_workspace_size(ctypes.byref(good_desc(**kw)))
    base = ws(steps_per_launch=1)
    assert ws() - base == 16 * 2 * 21 * 64 * 8                        # 64 x 64: 16 tiles
    big = dict(n_nodes=256 * 256, height=256, width=256)
    assert ws(**big) - ws(steps_per_launch=4, **big) == 256 * 2 * 21 * 64 * 8
    for kw in (dict(n_labels=8), dict(compat=mf.COMPAT_POTTS), dict(steps_per_launch=3),
               dict(n_nodes=257 * 256, height=257, width=256)):      # 272 tiles
        d = dict(big if "n_nodes" not in kw else {}, **kw)
        assert ws(**d) == ws(**dict(d, steps_per_launch=1)), kw


def test_admissible_alpha_rule():
    """alpha = 1 / (1 + margin * L-hat) of Sec. 3.2, computed by the library (host code)."""
    assert mf.admissible_alpha(0.0) == 1.0
    assert mf.admissible_alpha(-3.0) == 1.0
    assert mf.admissible_alpha(float("nan")) == 1.0
    assert abs(mf.admissible_alpha(3.981888) - 1 / (1 + 1.01 * 3.981888)) < 1e-15
    assert abs(mf.admissible_alpha(2.0, 0.5) - 1 / 3) < 1e-15     # margin below 1 taken as 1


def test_step_rule_validation():
    """Rules other than the fixed step: grids with FP32 messages; ADAPTIVE needs
    L = 2; the decays lie in [0, 1); momentum and ADAM state sits in the workspace."""
    assert validate(good_desc(rule=9)) == mf.MF_EINVAL
    assert validate(good_desc(rule=mf.RULES["adaptive"])) == mf.MF_EINVAL            # L = 21
    assert validate(good_desc(rule=mf.RULES["adaptive"], n_labels=2)) == mf.MF_OK
    assert validate(good_desc(rule=mf.RULES["adhoc"], precision=1)) == mf.MF_EUNSUPPORTED
    assert validate(good_desc(rule=mf.RULES["momentum"], rule_gamma1=1.0)) == mf.MF_EINVAL
    assert validate(good_desc(rule=mf.RULES["momentum"], rule_gamma1=0.95)) == mf.MF_OK
    adam = dict(rule=mf.RULES["adam"], rule_gamma1=0.9, rule_gamma2=0.999, rule_eps=1e-8, rule_v0=1.0)
    assert validate(good_desc(**adam)) == mf.MF_OK
    assert validate(good_desc(**{**adam, "rule_gamma2": -0.1})) == mf.MF_EINVAL
    assert validate(good_desc(**{**adam, "rule_eps": float("inf")})) == mf.MF_EINVAL
    assert validate(good_desc(**{**adam, "rule_v0": -1.0})) == mf.MF_EINVAL
    assert validate(good_desc(rule=mf.RULES["sweep"])) == mf.MF_OK
    E = 64 * 64 * 21 * 4
    base = mf.lib().mf_workspace_size(ctypes.byref(good_desc(steps_per_launch=1)))
    mom = mf.lib().mf_workspace_size(ctypes.byref(good_desc(rule=mf.RULES["momentum"], rule_gamma1=0.95)))
    ad = mf.lib().mf_workspace_size(ctypes.byref(good_desc(**adam)))
    assert mom >= base + E and ad >= base + 2 * E


def test_step_rules_need_a_grid():
    rp = FAKE + (1 << 35)
    d = good_desc(graph=mf.CSR, height=0, width=0, csr_row_ptr=rp, csr_col=rp + 4096, csr_nnz=8,
                  rule=mf.RULES["adhoc"])
    assert validate(d) == mf.MF_EUNSUPPORTED


def test_step_many_argument_checks_without_a_gpu():
    """mf_step_many checks its arrays before touching any handle."""
    L = mf.lib()
    one = (ctypes.c_int32 * 1)(1)
    nul = (ctypes.c_void_p * 1)(None)
    assert L.mf_step_many(None, None, 0) == mf.MF_OK                 # nothing to do
    assert L.mf_step_many(nul, one, -1) == mf.MF_EINVAL              # negative count
    assert L.mf_step_many(None, one, 1) == mf.MF_EINVAL              # NULL handle array
    assert L.mf_step_many(nul, None, 1) == mf.MF_EINVAL              # NULL step counts
    assert "n_steps" in mf.last_error()
    assert L.mf_step_many(nul, one, 1) == mf.MF_EINVAL               # NULL handle inside
    assert "NULL handle" in mf.last_error()


def test_solve_static_checks_before_any_hip_call():
    """mf_solve_static rejects, on the host, a problem whose workspace
    exceeds its static scratch, and an invalid descriptor."""
    L = mf.lib()
    big = good_desc(graph=mf.DENSE, n_nodes=8192, height=0, width=0)
    big.dense_K = FAKE + (1 << 36)
    assert L.mf_solve_static(ctypes.byref(big), 1, None, None, None) == mf.MF_ENOWORKSPACE
    assert "MF_STATIC_SCRATCH_BYTES" in mf.last_error()
    bad = good_desc(alpha=0.0)
    assert L.mf_solve_static(ctypes.byref(bad), 1, None, None, None) == mf.MF_EINVAL
    assert L.mf_solve_static(None, 1, None, None, None) == mf.MF_EINVAL
    assert L.mf_solve_static(ctypes.byref(good_desc()), -1, None, None, None) == mf.MF_EINVAL
