"""Build libmf.so (the HIP library behind include/mf.h) for gfx950, in-tree.

    python -m paper_1511_06103_amd.build [--jobs N] [--sanitize]

Every ``csrc/*.hip`` file is compiled to an object under ``_build/`` and
linked into ``paper_1511_06103_amd/libmf.so``.  hipcc cross-compiles, so no
GPU is needed.  Packed FP32 instructions are disabled for all device code.

``--sanitize`` builds a second copy, ``_build_san/libmf_san.so``, whose host
code (validation, handles, dispatch) carries AddressSanitizer and
UndefinedBehaviorSanitizer checks; the device code is unchanged.  It is for
the CPU tests of the C ABI (tests/test_abi_sanitized.py), which load it into
a Python process with the sanitizer runtime preloaded (``sanitizer_runtime``).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


BUILD_SAN = os.path.join(ROOT, "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "libmf_san.so")
# host-only sanitizer flags: every -fsanitize= goes to the host pass alone
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sanitizer_runtime():
    """The clang AddressSanitizer runtime that a process loading libmf_san.so
    must preload (it also carries the UndefinedBehaviorSanitizer handlers)."""
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _compile(src, build_dir=None, extra=()):
    obj = os.path.join(build_dir or BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=None, verbose=False, sanitize=False):
    build_dir, lib = (BUILD_SAN, LIB_SAN) if sanitize else (BUILD, LIB)
    extra = SAN_FLAGS if sanitize else ()
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if not srcs:
        raise RuntimeError("no HIP sources found")
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--sanitize", action="store_true", help="also build _build_san/libmf_san.so (ASan + UBSan host code)")
    args = ap.parse_args(argv)
    build(args.jobs, verbose=True)
    if args.sanitize:
        build(args.jobs, verbose=True, sanitize=True)


if __name__ == "__main__":
    sys.exit(main())
