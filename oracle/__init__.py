"""FP64 CPU oracle of the proximal-gradient parallel mean-field update.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
check of the graft entry point and the CPU-baseline leg of the benchmark
may import, call or execute anything in this package.  The product path
(the HIP library and its Python binding) never reaches it and must fail
loudly when the HIP library is missing instead of falling back here.

The oracle shares no code with the HIP path: no kernels, headers, helpers,
tables or pre/post-processing.  Both sides consume only the seeded input
arrays of ``paper_1511_06103_amd.synth``, which contains no step of the
method.  Everything here is plain NumPy in FP64; pure-Python loops appear
only in the small-case routines (sequential sweep, enumeration).

Every function that has no independent pin would be marked "parity
unpinned" in its docstring; at present none is.  The pins live in
``tests/test_oracle_pins.py``; ``tests/test_oracle_mutations.py`` checks
that they catch mistakes planted in the oracle.
"""
from .mf import *  # noqa: F401,F403
