"""A HIP failure after validation: with no HIP device in the process every
launch fails, and a call that passes host-side validation must report
XTC_E_HIP with the failing step in its message rather than crash.  The call
passes fake device pointers, so it only runs where no device exists (the
kernel driver's /dev/kfd absent); with a device present it is skipped."""
import ctypes
import os

import numpy as np
import pytest

from paper_2304_07006_amd import xtc

pytestmark = pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a HIP device is present: fake pointers would be used")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(xtc.LIB_PATH):
        pytest.skip("libxtc.so not built")
    return xtc.load()


def test_launch_failure_is_reported(lib):
    occ = np.arange(2, dtype=np.int32)
    c = xtc.XtcProblem()
    c.N, c.Ng, c.nocc = 8, 100, 2
    c.xyz, c.w, c.phi = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    c.occ = occ.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    n = lib.xtc_workspace_size(ctypes.byref(c), 0, 50)
    assert n > 0
    st = lib.xtc_prepare(ctypes.byref(c), 0, 50, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_HIP
    assert "prepare_pos" in xtc.last_error()
    # the next call is validated first, as always
    assert lib.xtc_prepare(ctypes.byref(c), 0, 50, None, n, None) == xtc.XTC_E_WORKSPACE
    assert "prepare_pos" not in xtc.last_error()
