"""Build the HIP library ``liblbm.so`` for gfx950 (in-tree, next to this file),
and its checked variant ``liblbm_checked.so`` (device-side bounds tests,
LBM_CHECKED=1; see ``lbm_check_flags`` in include/lbm.h).

hipcc cross-compiles without a GPU.  Packed-FP32 instructions are disabled
(-packed-fp32-ops) so the compiler emits plain VALU FP32 arithmetic.
Multiply-adds are fused only within one source expression
(-ffp-contract=on): fused across statements, the choice of which product to
fuse differs between kernels that inline the same collision code, and so do
their roundings (the in-place and two-buffer patterns then stop agreeing
bitwise).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbm.so")
# the same sources with the device-side bounds tests compiled in (LBM_CHECKED)
CHECKED_LIB = os.path.join(HERE, "liblbm_checked.so")
SOURCES = ["lbm_kernels.hip", "lbm_variants.hip", "lbm_runtime.hip", "lbm_fused.hip", "lbm_adjoint.hip",
           "lbm_structures.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def build(verbose: bool = False, jobs: int = 6, checked: bool = True) -> str:
    """Build liblbm.so and (checked) liblbm_checked.so; returns the first."""
    _build_one(LIB, [], verbose, jobs)
    if checked:
        _build_one(CHECKED_LIB, ["-DLBM_CHECKED=1"], verbose, jobs)
    return LIB


def _build_one(lib: str, defines, verbose: bool, jobs: int) -> None:
    csrc = os.path.join(HERE, "csrc")
    tag = "_checked" if defines else ""
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(csrc, os.path.splitext(src)[0] + tag + ".o")
        cmd = ["hipcc", *hipcc_flags(), *defines, "-c", os.path.join(csrc, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError(f"hipcc failed on {src}")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = lib + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, checked="--release-only" not in sys.argv))
