"""Build ``libcmlb.so`` (the HIP library behind include/cmlb.h) for gfx950.

Run ``python -m paper_2504_09024_amd.build`` or call :func:`build`.  The
library is built in-tree next to this file so it travels with the source
tree.  Packed FP32 instructions are disabled (``-packed-fp32-ops``): hipcc
otherwise forms v_pk_* FP32 ops from ordinary float code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcmlb.so")
SOURCES = [os.path.join(HERE, "csrc", "cmlb.hip"), os.path.join(HERE, "csrc", "cmlb3.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", f)
                  for f in ("kernels.hpp", "lattice.hpp", "device_common.hpp", "kernels3.hpp")] + [
    os.path.join(ROOT, "include", f) for f in ("cmlb.h", "cmlb3.h")]
ARCH = os.environ.get("CMLB_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libcmlb.so)")


# FP contraction only within one expression (-ffp-contract=on): with HIP's
# default (fusing across statements in the backend) the choice can differ
# between kernel instances of different launch shapes, and results would
# then differ in the last bits from one launch shape to another.
COMMON = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
EXTRA = {}  # per-source flags


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link."""
    import tempfile
    with tempfile.TemporaryDirectory(prefix="cmlb_build_") as tmp:
        procs, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [hipcc(), *COMMON, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = False
        for cmd, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed building libcmlb.so")
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking libcmlb.so failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True))
