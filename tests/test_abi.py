"""The C ABI: exported symbols and host-side validation (no kernel launches).

Every call here passes fake device pointers and is built to fail validation
before any HIP call, so the tests are safe with or without a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2304_07006_amd import xtc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "xtc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xtc_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(xtc.LIB_PATH):
        pytest.skip("libxtc.so not built")
    return xtc.load()


def test_every_declared_symbol_is_exported(lib):
    names = _header_functions()
    assert "xtc_build_K" in names and "xtc_contract_2body" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(xtc.exported_symbols())


def test_pair_ld(lib):
    assert lib.xtc_pair_ld(8) == 128
    assert lib.xtc_pair_ld(128) == 8320
    assert lib.xtc_pair_ld(0) == 0


def _problem(N=8, Ng=100, occ=(0, 1), fake=0x1000):
    occ = np.array(occ, dtype=np.int32)
    c = xtc.XtcProblem(N, Ng, len(occ), 0, fake, fake, fake, occ.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return c, occ


def _jas(kind=0, ncoef=0, b=1.0):
    j = xtc.XtcJastrow()
    j.kind, j.ncoef, j.b = kind, ncoef, b
    return j


def _call_build(lib, c, j, g0=0, g1=10, prec=0, K=0x2000, ws=None, nbytes=None):
    if nbytes is None:
        nbytes = lib.xtc_workspace_size(ctypes.byref(c), 0, 50) if ws is None else nbytes
    return lib.xtc_build_K(ctypes.byref(c), ctypes.byref(j), g0, g1, prec, ctypes.c_void_p(K),
                           ctypes.c_void_p(ws if ws is not None else 0x100000), nbytes, None)


@pytest.mark.parametrize("mut,expect", [
    (dict(N=0), xtc.XTC_E_ARG),
    (dict(N=257, occ=(0,)), xtc.XTC_E_ARG),                 # above the largest supported N (256)
    (dict(Ng=0), xtc.XTC_E_ARG),                             # empty grid
    (dict(Ng=(1 << 28) + 1), xtc.XTC_E_UNSUPPORTED),          # above the 32-bit grid indexing limit
    (dict(occ=()), xtc.XTC_E_ARG),                           # no occupied orbital
    (dict(N=256, occ=tuple(range(20))), xtc.XTC_E_UNSUPPORTED),   # nocc N 32 B over the on-chip staging
    (dict(occ=(0, 0)), xtc.XTC_E_ARG),
    (dict(occ=(0, 9)), xtc.XTC_E_ARG),
    (dict(occ=(-1,)), xtc.XTC_E_ARG),
])
def test_bad_problem(lib, mut, expect):
    kw = dict(N=8, Ng=100, occ=(0, 1))
    kw.update(mut)
    c, keep = _problem(**kw)
    assert lib.xtc_workspace_size(ctypes.byref(c), 0, 50) == 0
    st = _call_build(lib, c, _jas(), nbytes=1 << 30)
    assert st == expect
    assert xtc.last_error()


def test_lowdin_limits(lib):
    assert lib.xtc_lowdin_workspace_size(8, 0) == 0 and "out of range" in xtc.last_error()
    assert lib.xtc_lowdin_workspace_size(8, (1 << 28) + 1) == 0
    assert lib.xtc_lowdin_workspace_size(8, 1 << 28) > 0
    st = lib.xtc_lowdin(8, (1 << 28) + 1, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000),
                        None, ctypes.c_void_p(0x100000), 1 << 20, None)
    assert st == xtc.XTC_E_UNSUPPORTED


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_bad_occupation_numbers(lib, bad):
    c, keep = _problem(occ=(0, 1))
    occ_n = np.array([1.0, bad])
    c.occ_n = occ_n.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.xtc_workspace_size(ctypes.byref(c), 0, 50) == 0
    assert _call_build(lib, c, _jas(), nbytes=1 << 30) == xtc.XTC_E_ARG
    assert "occ_n" in xtc.last_error()


def test_bad_beta_occupations_and_open_shell_adjoint_workspace(lib):
    c, keep = _problem(occ=(0, 1))
    nb = np.array([1.0, float("nan")])
    c.occ_n_beta = nb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.xtc_workspace_size(ctypes.byref(c), 0, 50) == 0
    assert "occ_n_beta" in xtc.last_error()
    nb[1] = 0.0
    j = _jas(kind=1, ncoef=2)
    j.coef[0], j.coef[1] = 0.5, 0.1
    # the open-shell adjoint is supported: the call gets as far as the
    # workspace check (too small here, so nothing launches)
    st = lib.xtc_backward(ctypes.byref(c), ctypes.byref(j), xtc.XTC_WITH_BACKWARD, None, None, 1.0,
                          ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), 100, None)
    assert st == xtc.XTC_E_WORKSPACE
    cc, keep_c = _problem(occ=(0, 1))
    n_closed = lib.xtc_workspace_size(ctypes.byref(cc), xtc.XTC_WITH_BACKWARD | 2, 50)
    assert lib.xtc_workspace_size(ctypes.byref(c), xtc.XTC_WITH_BACKWARD | 2, 50) > n_closed


@pytest.mark.parametrize("core,act", [([0], [0, 1]), ([9], [1]), ([], []), ([-1], [2])])
def test_frozen_core_validation(lib, core, act):
    c = np.array(core, dtype=np.int32)
    a = np.array(act, dtype=np.int32)
    ip = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    f = ctypes.c_void_p(0x1000)
    st = lib.xtc_frozen_core(8, f, f, f, len(c), ip(c), len(a), ip(a), f, f, f, None)
    assert st == xtc.XTC_E_ARG and xtc.last_error()


def test_bad_jastrow_and_range(lib):
    c, keep = _problem()
    n = lib.xtc_workspace_size(ctypes.byref(c), 0, 50)
    assert n > 0
    assert _call_build(lib, c, _jas(b=-1.0), nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(b=float("nan")), nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(kind=1, ncoef=0), nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(kind=1, ncoef=17), nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(kind=7), nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(), g0=5, g1=5, nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(), g0=0, g1=101, nbytes=n) == xtc.XTC_E_ARG
    # every call below must fail validation (fake pointers: nothing may launch)
    assert _call_build(lib, c, _jas(), g0=0, g1=100, nbytes=n) == xtc.XTC_E_WORKSPACE  # > 64-row capacity
    assert _call_build(lib, c, _jas(), K=0, nbytes=n) == xtc.XTC_E_ARG
    assert _call_build(lib, c, _jas(), K=0x2008, nbytes=n) == xtc.XTC_E_ARG           # misaligned
    assert _call_build(lib, c, _jas(), nbytes=100) == xtc.XTC_E_WORKSPACE
    assert lib.xtc_build_K(ctypes.byref(c), ctypes.byref(_jas()), 0, 10, 0, ctypes.c_void_p(0x2000),
                           None, n, None) == xtc.XTC_E_WORKSPACE
    assert _call_build(lib, c, _jas(), prec=9, nbytes=n) == xtc.XTC_E_ARG


def test_contract_flags(lib):
    c, keep = _problem()
    n = lib.xtc_workspace_size(ctypes.byref(c), 0, 50)
    st = lib.xtc_contract_2body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10, 0, 8, None,
                                ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG
    st = lib.xtc_contract_2body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10, 0, xtc.XTC_FINALIZE, None,
                                ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG
    st = lib.xtc_contract_1body_0body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10, 0, xtc.XTC_FINALIZE,
                                      None, None, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG
    # the reuse assertion is a one-body flag only
    st = lib.xtc_contract_2body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10, 0, xtc.XTC_REUSE_INTERMEDIATES,
                                None, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG and "unknown bits" in xtc.last_error()
    st = lib.xtc_contract_1body_0body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10, 0,
                                      xtc.XTC_FINALIZE | xtc.XTC_REUSE_INTERMEDIATES,
                                      None, None, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG and "NULL" in xtc.last_error()        # past the flag check
    st = lib.xtc_contract_1body_0body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10, 0, 8,
                                      None, None, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG and "unknown bits" in xtc.last_error()


def test_backward_validation(lib):
    c, keep = _problem()
    n = lib.xtc_workspace_size(ctypes.byref(c), xtc.XTC_WITH_BACKWARD, 50)
    assert n > lib.xtc_workspace_size(ctypes.byref(c), 0, 50)
    j = _jas(kind=0)
    st = lib.xtc_backward(ctypes.byref(c), ctypes.byref(j), xtc.XTC_WITH_BACKWARD, None, None, 1.0,
                          ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_UNSUPPORTED                                 # Pade: no coefficients
    j = _jas(kind=1, ncoef=4)
    for k in range(4):
        j.coef[k] = 0.1
    st = lib.xtc_backward(ctypes.byref(c), ctypes.byref(j), 0, None, None, 1.0,
                          ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG                                         # workspace flag missing
    st = lib.xtc_backward(ctypes.byref(c), ctypes.byref(j), xtc.XTC_WITH_BACKWARD, None, None, 1.0,
                          None, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG                                         # gcoef NULL
    st = lib.xtc_backward(ctypes.byref(c), ctypes.byref(j), xtc.XTC_WITH_BACKWARD, None, None, float("inf"),
                          ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG                                         # gE0 not finite
    st = lib.xtc_backward(ctypes.byref(c), ctypes.byref(j), xtc.XTC_WITH_BACKWARD | 0x100, None, None, 1.0,
                          ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG                                         # unknown prec bits


def test_reduced_occ_flag_only_for_build_K(lib):
    """XTC_K_REDUCED_OCC is a per-call option of xtc_build_K: the workspace
    layout ignores it there and every other call rejects it."""
    c, keep = _problem()
    assert lib.xtc_workspace_size(ctypes.byref(c), xtc.XTC_BF16X3 | xtc.XTC_K_REDUCED_OCC, 50) == 0
    n = lib.xtc_workspace_size(ctypes.byref(c), xtc.XTC_BF16X3, 50)
    st = lib.xtc_contract_2body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10,
                                xtc.XTC_BF16X3 | xtc.XTC_K_REDUCED_OCC, 0, None, ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG
    # accepted by xtc_build_K's checks: an invalid range is what fails here
    j = _jas(kind=0)
    st = lib.xtc_build_K(ctypes.byref(c), ctypes.byref(j), 5, 5, xtc.XTC_BF16X3 | xtc.XTC_K_REDUCED_OCC,
                         ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG and "rows" in xtc.last_error()


def test_occ_fp64_flag_only_for_build_K(lib):
    """XTC_K_OCC_FP64 (the FP64 occupied block instead of the integer one) is
    a per-call option of xtc_build_K like XTC_K_REDUCED_OCC, and the two
    exclude each other."""
    c, keep = _problem()
    assert lib.xtc_workspace_size(ctypes.byref(c), xtc.XTC_BF16X3 | xtc.XTC_K_OCC_FP64, 50) == 0
    n = lib.xtc_workspace_size(ctypes.byref(c), xtc.XTC_BF16X3, 50)
    st = lib.xtc_contract_1body_0body(ctypes.byref(c), ctypes.c_void_p(0x2000), 0, 10,
                                      xtc.XTC_BF16X3 | xtc.XTC_K_OCC_FP64, 0, None, None,
                                      ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG
    j = _jas(kind=0)
    st = lib.xtc_build_K(ctypes.byref(c), ctypes.byref(j), 5, 5, xtc.XTC_BF16X3 | xtc.XTC_K_OCC_FP64,
                         ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG and "rows" in xtc.last_error()
    st = lib.xtc_build_K(ctypes.byref(c), ctypes.byref(j), 0, 10,
                         xtc.XTC_BF16X3 | xtc.XTC_K_OCC_FP64 | xtc.XTC_K_REDUCED_OCC,
                         ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG and "together" in xtc.last_error()


def test_workspace_grows_with_chunk(lib):
    c, keep = _problem(N=16, Ng=1000, occ=(0, 3, 5))
    a = lib.xtc_workspace_size(ctypes.byref(c), 0, 100)
    b = lib.xtc_workspace_size(ctypes.byref(c), 0, 1000)
    assert 0 < a < b
    assert lib.xtc_workspace_size(ctypes.byref(c), 0, 1001) == 0


def test_lowdin_validation(lib):
    assert lib.xtc_lowdin_workspace_size(0, 10) == 0
    assert lib.xtc_lowdin_workspace_size(8, 100) > 0
    n = lib.xtc_lowdin_workspace_size(8, 100)
    st = lib.xtc_lowdin(8, 100, None, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x4000), None,
                        ctypes.c_void_p(0x100000), n, None)
    assert st == xtc.XTC_E_ARG
    st = lib.xtc_lowdin(8, 100, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x4000), None,
                        ctypes.c_void_p(0x100000), n - 1, None)
    assert st == xtc.XTC_E_WORKSPACE


def test_lowdin_noalloc_validation(lib):
    """xtc_lowdin_noalloc rejects bad sizes, NULL arrays and problems whose
    scratch exceeds the static array before any HIP call (fake pointers)."""
    f = ctypes.c_void_p(0x1000)
    assert lib.xtc_lowdin_noalloc(0, 100, f, f, f, None, None) == xtc.XTC_E_ARG
    assert lib.xtc_lowdin_noalloc(8, 100, None, f, f, None, None) == xtc.XTC_E_ARG
    assert lib.xtc_lowdin_noalloc(8, (1 << 28) + 1, f, f, f, None, None) == xtc.XTC_E_UNSUPPORTED
    assert lib.xtc_lowdin_workspace_size(256, 1 << 20) > (64 << 20)
    st = lib.xtc_lowdin_noalloc(256, 1 << 20, f, f, f, None, None)
    assert st == xtc.XTC_E_UNSUPPORTED and "static array" in xtc.last_error()
