"""Build libsboxwalsh.so (HIP, gfx950) in the package directory.

Only hipcc is needed; the library links the HIP runtime and nothing else.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsboxwalsh.so")
ARCH = os.environ.get("SBOX_OFFLOAD_ARCH", "gfx950")

SOURCES = ["sbox_walsh.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
    # keep hipcc from fusing fp32 work into packed-fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the only floating point here (fp16/fp32 MFMA Hadamard passes) holds finite
    # integers: no NaN handling and no IEEE-mode canonicalisation around max.
    # (The kernels read their work-item and group ids through the compiler's
    # builtins: the device library's functions for them, built in IEEE mode,
    # cannot be inlined into non-IEEE kernels.)
    "-fno-honor-nans", "-mno-amdgpu-ieee",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + HIPCC_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if out.strip() and verbose:
        print(out, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
