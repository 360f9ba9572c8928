"""xtc_lowdin_noalloc (scratch in the library's static device array, nothing
allocated) against xtc_lowdin (caller workspace), through the C ABI: two
calls in a row on one device, the second with a smaller problem, each
bitwise equal to the workspace entry point's result (same kernels, same
launch shapes); and the size limit."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _both(torch, chi, w):
    from paper_2304_07006_amd import xtc
    N, Ng = chi.shape
    chi_t = torch.as_tensor(chi).cuda()
    w_t = torch.as_tensor(w).cuda()
    ws = torch.empty(xtc.load().xtc_lowdin_workspace_size(N, Ng), dtype=torch.uint8, device="cuda")
    ref, lref = torch.empty_like(chi_t), torch.empty(N, dtype=torch.float64, device="cuda")
    xtc.xtc_lowdin(N, Ng, chi_t, w_t, ref, lref, ws)
    got, lgot = torch.full_like(chi_t, np.nan), torch.full((N,), np.nan, dtype=torch.float64, device="cuda")
    xtc.xtc_lowdin_noalloc(N, Ng, chi_t, w_t, got, lgot)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), lref.cpu().numpy(), got.cpu().numpy(), lgot.cpu().numpy()


def test_noalloc_lowdin_matches_workspace_entry_point_twice(torch_cuda):
    for name, N, nocc, Ng, nc in (("large", 128, 16, 20000, 8), ("smaller", 24, 3, 3000, 3)):
        p = inputs.make_problem(N, nocc, Ng, nc, "chain", "pade", seed=71)
        _note(f"case: lowdin_noalloc {name} N={N} Ng={Ng}")
        ref, lref, got, lgot = _both(torch_cuda, p.chi, p.w)
        _note(f"  max |phi - phi_ws| = {np.abs(got - ref).max():.2e}")
        assert np.array_equal(got, ref) and np.array_equal(lgot, lref)
        # and the result is the orthonormalisation (oracle-independent check)
        lam = lref
        O = (got * p.w) @ got.T
        assert np.abs(O - np.eye(N)).max() < 50 * np.finfo(float).eps * lam.max() / lam.min()


def test_noalloc_lowdin_rejects_sizes_beyond_the_static_array(torch_cuda):
    from paper_2304_07006_amd import xtc
    # N = 256 on 2^20 points needs 256 segments of 512 KB of partials: above 64 MiB
    n = xtc.load().xtc_lowdin_workspace_size(256, 1 << 20)
    assert n > (64 << 20)
    import torch
    chi = torch.zeros(256 * 1024, dtype=torch.float64, device="cuda")   # never read: rejected before any launch
    st = xtc.load().xtc_lowdin_noalloc(256, 1 << 20, chi.data_ptr(), chi.data_ptr(), chi.data_ptr(), None, None)
    assert st == xtc.XTC_E_UNSUPPORTED and "static array" in xtc.last_error()
