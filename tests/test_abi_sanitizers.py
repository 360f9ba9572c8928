"""The host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer: the library is rebuilt with host-side sanitizers
(device code unchanged) and the C-ABI tests, which exercise validation,
workspace sizing, error messages and (with no device) the launch-failure
path, run against it in a child process with the sanitizer runtime
preloaded.  Any report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RUNTIME = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

RUNNER = """
import sys
sys.path.insert(0, {root!r})
import paper_2304_07006_amd.xtc as x
x.LIB_PATH = {lib!r}
import pytest
sys.exit(pytest.main([{t1!r}, {t2!r}, "-q", "-p", "no:cacheprovider"]))
"""


@pytest.mark.skipif(not RUNTIME, reason="no sanitizer runtime in this toolchain")
def test_abi_under_host_sanitizers(tmp_path):
    from paper_2304_07006_amd import build
    lib = build.build(out=str(tmp_path / "libxtc_san.so"), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=RUNTIME[-1], ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = RUNNER.format(root=ROOT, lib=lib, t1=os.path.join(ROOT, "tests", "test_abi.py"),
                         t2=os.path.join(ROOT, "tests", "test_abi_nodevice.py"))
    res = subprocess.run([sys.executable, "-c", code], env=env, cwd=str(tmp_path), capture_output=True, text=True,
                         timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
