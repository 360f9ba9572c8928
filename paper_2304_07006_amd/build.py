"""Build libxtc.so (all HIP kernels + the C ABI) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libxtc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
]
# Translation units and their own flags.  xtc_api.hip: MFMA accumulators in
# ordinary VGPRs (no per-iteration AGPR copies).  occ_i8.hip: the integer
# occupied block keeps 216 accumulator registers per lane, beyond the 256
# ordinary VGPRs, so its accumulators stay in the AGPRs.
UNITS = [
    (os.path.join(HERE, "csrc", "xtc_api.hip"), ["-mllvm", "-amdgpu-mfma-vgpr-form"]),
    (os.path.join(HERE, "csrc", "occ_i8.hip"), []),
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
    extra = SANITIZE_FLAGS if sanitize else []
    objs, log = [], []
    jobs = []   # the units compile side by side
    for src, own in UNITS:
        obj = f"{tmp}.{os.path.splitext(os.path.basename(src))[0]}.o"
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, *own, *extra, "-c", src, "-o", obj]
        jobs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    for cmd, job in jobs:
        _check(job.communicate()[0], job.returncode, log)
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, *objs, "-o", tmp], log)
    for obj in objs:
        os.remove(obj)
    if verbose and log:
        print("\n".join(log), file=sys.stderr)
    os.replace(tmp, lib)
    return lib


def _run(cmd, log):
    res = subprocess.run(cmd, capture_output=True, text=True)
    _check(res.stdout + res.stderr, res.returncode, log)


def _check(text, rc, log):
    out = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
    if rc != 0:
        raise RuntimeError(f"hipcc failed ({rc}):\n{out}")
    if out.strip():
        log.append(out)


if __name__ == "__main__":
    print(build(verbose=True))
