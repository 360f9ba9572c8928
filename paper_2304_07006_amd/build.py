"""Build libxtc.so (all HIP kernels + the C ABI) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libxtc.so")
SOURCES = [os.path.join(HERE, "csrc", "xtc_api.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
    # MFMA accumulators in ordinary VGPRs (no per-iteration AGPR copies)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the C-ABI
# checks (device code is built as usual); load with the sanitizer runtime
# preloaded.
SANITIZE_FLAGS = ("-O1 -g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                  "-Xarch_host -fno-omit-frame-pointer -shared-libsan").split()


def build(verbose: bool = False, out: str | None = None, sanitize: bool = False) -> str:
    """Compile libxtc.so in-tree (or to `out`); `sanitize` adds the host-side
    sanitizers (a checking build, not the product library)."""
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *(SANITIZE_FLAGS if sanitize else ()), *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if verbose and out.strip():
        print(out, file=sys.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
