"""Python binding: argument checks that run before anything reaches the C ABI
or the device (the library takes plain pointers and cannot check sizes)."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs, xtc


def _fake_dp(N=8, Ng=100):
    occ = np.array([0, 1], dtype=np.int32)
    c = xtc.XtcProblem(N, Ng, 2, 0, 0x1000, 0x1000, 0x1000, occ.ctypes.data_as(xtc.ctypes.POINTER(xtc.ctypes.c_int32)))
    return xtc.DeviceProblem(None, None, None, occ, c)


@pytest.mark.parametrize("xyz_shape,w_shape", [((99, 3), (100,)), ((100, 2), (100,)), ((100, 3), (99,))])
def test_device_problem_shapes(xyz_shape, w_shape):
    phi = np.zeros((8, 100))
    with pytest.raises(ValueError):
        xtc.device_problem(np.zeros(xyz_shape), np.zeros(w_shape), phi, [0, 1], device="cpu")


def test_host_tensors_are_refused():
    import os
    import torch
    if not os.path.exists(xtc.LIB_PATH):
        pytest.skip("libxtc.so not built")
    dp = _fake_dp()
    jas = xtc.make_jastrow(inputs.Jastrow("pade", b=1.0))
    ws = torch.zeros(1 << 10, dtype=torch.uint8)
    K = torch.zeros(3 * 10 * 128, dtype=torch.float64)
    with pytest.raises(ValueError, match="device tensor"):
        xtc.xtc_build_K(dp, jas, 0, 10, 0, K, ws)
    with pytest.raises(ValueError, match="device tensor"):
        xtc.xtc_contract_2body(dp, K, 0, 10, 0, xtc.XTC_FINALIZE, torch.zeros(8 ** 4, dtype=torch.float64), ws)
    with pytest.raises(ValueError, match="required"):
        xtc._dev(None, 1, "V2")
    xtc._dev(None, 1, "gV2", required=False)


def test_tc_two_body_gradient_shape():
    p = inputs.make_workload("N8-occ2-Ng2k")
    with pytest.raises(ValueError, match="dphi"):
        xtc.tc_two_body(p, np.zeros((3, 8, 1999)), device="cpu")
