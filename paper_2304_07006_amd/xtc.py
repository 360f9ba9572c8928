"""Python binding of libxtc (include/xtc.h): argument marshalling only.

Every numerical step runs in the library's HIP kernels; torch is used to
hold device memory and to name the current HIP stream.  The functions named
``xtc_*`` mirror the C entry points one to one; ``forward`` strings them
together over grid chunks for a whole pass.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxtc.so")

XTC_OK, XTC_E_ARG, XTC_E_WORKSPACE, XTC_E_HIP, XTC_E_UNSUPPORTED = 0, -1, -2, -3, -4
XTC_FP64, XTC_FP32, XTC_BF16X3, XTC_BF16X6 = 0, 1, 2, 3
XTC_RESET, XTC_FINALIZE, XTC_REUSE_INTERMEDIATES = 1, 2, 4
XTC_WITH_BACKWARD = 0x10
XTC_WITH_TC2 = 0x20
XTC_K_REDUCED_OCC = 0x40
XTC_K_OCC_FP64 = 0x80
PRECISIONS = {"fp64": XTC_FP64, "fp32": XTC_FP32, "bf16x3": XTC_BF16X3, "bf16x6": XTC_BF16X6}


class XtcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"xtc status {status}: {message}")
        self.status = status


class XtcJastrow(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ncoef", ctypes.c_int32), ("b", ctypes.c_double),
                ("coef", ctypes.c_double * 16)]


class XtcProblem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("Ng", ctypes.c_int32), ("nocc", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("occ", ctypes.POINTER(ctypes.c_int32)),
                ("occ_n", ctypes.POINTER(ctypes.c_double)), ("occ_n_beta", ctypes.POINTER(ctypes.c_double))]


_SIGS = {
    "xtc_tc_2body": (ctypes.c_int, [ctypes.POINTER(XtcProblem), ctypes.POINTER(XtcJastrow), ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "xtc_frozen_core": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "xtc_pair_ld": (ctypes.c_int32, [ctypes.c_int32]),
    "xtc_last_error": (ctypes.c_char_p, []),
    "xtc_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(XtcProblem), ctypes.c_int32, ctypes.c_int32]),
    "xtc_prepare": (ctypes.c_int, [ctypes.POINTER(XtcProblem), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "xtc_build_K": (ctypes.c_int, [ctypes.POINTER(XtcProblem), ctypes.POINTER(XtcJastrow), ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]),
    "xtc_contract_2body": (ctypes.c_int, [ctypes.POINTER(XtcProblem), ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "xtc_contract_1body_0body": (ctypes.c_int, [ctypes.POINTER(XtcProblem), ctypes.c_void_p, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_size_t, ctypes.c_void_p]),
    "xtc_backward": (ctypes.c_int, [ctypes.POINTER(XtcProblem), ctypes.POINTER(XtcJastrow), ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "xtc_lowdin_workspace_size": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "xtc_lowdin": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]),
    "xtc_lowdin_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


def load():
    """Load the in-tree libxtc.so; fail loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2304_07006_amd/build.py (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def last_error() -> str:
    return load().xtc_last_error().decode()


def _check(status):
    if status != XTC_OK:
        raise XtcError(status, last_error())


# ------------------------------------------------------------ marshalling --
def make_jastrow(jas) -> XtcJastrow:
    """From an object with .kind ('pade'|'power'), .b, .coef."""
    j = XtcJastrow()
    if jas.kind == "pade":
        j.kind, j.ncoef, j.b = 0, 0, float(jas.b)
    elif jas.kind == "power":
        j.kind, j.ncoef, j.b = 1, len(jas.coef), 0.0
        for k, c in enumerate(jas.coef):
            j.coef[k] = float(c)
    else:
        raise ValueError(jas.kind)
    return j


@dataclass
class DeviceProblem:
    """Device copies of the inputs plus the C struct that points at them."""
    xyz: object
    w: object
    phi: object
    occ_host: np.ndarray
    c: XtcProblem
    occ_n_host: np.ndarray | None = None
    occ_n_beta_host: np.ndarray | None = None

    @property
    def open_shell(self):
        return self.occ_n_beta_host is not None

    @property
    def N(self):
        return self.c.N

    @property
    def Ng(self):
        return self.c.Ng


def _dev(t, numel, name, dtype="float64", required=True):
    """Check a tensor handed to the C ABI, which takes plain pointers and
    cannot check sizes itself: on a HIP device, contiguous, of the expected
    dtype and holding at least `numel` elements."""
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {numel} needed")


def device_problem(xyz, w, phi, occ, device="cuda", occ_n=None, occ_n_beta=None) -> DeviceProblem:
    """occ: orbitals of the reference density; occ_n: their per-spin
    occupations (None: 1 each, the closed-shell determinant); occ_n_beta: the
    beta occupations of an open-shell reference (then occ_n is alpha).
    xyz [Ng][3], w [Ng], phi [N][Ng]."""
    import torch
    if np.ndim(phi) != 2:
        raise ValueError("phi must be [N][Ng]")
    Ng = np.shape(phi)[1]
    if np.shape(xyz) != (Ng, 3) or np.shape(w) != (Ng,):
        raise ValueError(f"xyz must be [{Ng}][3] and w [{Ng}] for phi of shape {np.shape(phi)}")
    if np.ndim(occ) != 1:
        raise ValueError("occ must be a 1-D list of orbital indices")
    t_xyz = torch.as_tensor(np.ascontiguousarray(xyz, dtype=np.float64)).to(device)
    t_w = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(device)
    t_phi = torch.as_tensor(np.ascontiguousarray(phi, dtype=np.float64)).to(device)
    occ_h = np.ascontiguousarray(occ, dtype=np.int32)
    occ_n_h = None if occ_n is None else np.ascontiguousarray(occ_n, dtype=np.float64)
    occ_b_h = None if occ_n_beta is None else np.ascontiguousarray(occ_n_beta, dtype=np.float64)
    for a in (occ_n_h, occ_b_h):
        if a is not None and a.shape != occ_h.shape:
            raise ValueError("occupations must have one entry per listed orbital")
    dptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c = XtcProblem(int(phi.shape[0]), int(phi.shape[1]), int(len(occ_h)), 0, t_xyz.data_ptr(), t_w.data_ptr(),
                   t_phi.data_ptr(), occ_h.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), dptr(occ_n_h),
                   dptr(occ_b_h))
    return DeviceProblem(t_xyz, t_w, t_phi, occ_h, c, occ_n_h, occ_b_h)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------- entry points --
def xtc_pair_ld(N: int) -> int:
    return load().xtc_pair_ld(N)


def xtc_workspace_size(dp: DeviceProblem, prec: int, chunk_rows: int) -> int:
    n = load().xtc_workspace_size(ctypes.byref(dp.c), prec, chunk_rows)
    if n == 0:
        raise XtcError(XTC_E_ARG, last_error())
    return n


def xtc_prepare(dp, prec, chunk_rows, ws, stream=None):
    _dev(ws, 1, "ws", "uint8")
    _check(load().xtc_prepare(ctypes.byref(dp.c), prec, chunk_rows, _ptr(ws), ws.numel(), _stream(stream)))


def _nspin(dp):
    return 2 if getattr(dp, "open_shell", False) else 1


def xtc_build_K(dp, jas: XtcJastrow, g0, g1, prec, K, ws, stream=None):
    _dev(ws, 1, "ws", "uint8")
    _dev(K, 3 * max(0, g1 - g0) * xtc_pair_ld(dp.N), "K")
    _check(load().xtc_build_K(ctypes.byref(dp.c), ctypes.byref(jas), g0, g1, prec, _ptr(K), _ptr(ws),
                              ws.numel(), _stream(stream)))


def xtc_contract_2body(dp, K, g0, g1, prec, flags, V2, ws, stream=None):
    _dev(ws, 1, "ws", "uint8")
    _dev(K, 3 * max(0, g1 - g0) * xtc_pair_ld(dp.N), "K")
    _dev(V2, (3 if _nspin(dp) == 2 else 1) * dp.N ** 4, "V2", required=bool(flags & XTC_FINALIZE))
    _check(load().xtc_contract_2body(ctypes.byref(dp.c), _ptr(K), g0, g1, prec, flags, _ptr(V2), _ptr(ws),
                                     ws.numel(), _stream(stream)))


def xtc_contract_1body_0body(dp, K, g0, g1, prec, flags, h1, E0, ws, stream=None):
    _dev(ws, 1, "ws", "uint8")
    _dev(K, 3 * max(0, g1 - g0) * xtc_pair_ld(dp.N), "K")
    _dev(h1, _nspin(dp) * dp.N ** 2, "h1", required=bool(flags & XTC_FINALIZE))
    _dev(E0, 1, "E0", required=bool(flags & XTC_FINALIZE))
    _check(load().xtc_contract_1body_0body(ctypes.byref(dp.c), _ptr(K), g0, g1, prec, flags, _ptr(h1), _ptr(E0),
                                           _ptr(ws), ws.numel(), _stream(stream)))


def xtc_backward(dp, jas: XtcJastrow, prec, gV2, gh1, gE0, gcoef, ws, stream=None):
    _dev(ws, 1, "ws", "uint8")
    blocks = 3 if _nspin(dp) == 2 else 1          # open shell: spin-blocked seeds (aa, ab, bb) and (a, b)
    _dev(gV2, blocks * dp.N ** 4, "gV2", required=False)
    _dev(gh1, (2 if blocks == 3 else 1) * dp.N ** 2, "gh1", required=False)
    _dev(gcoef, max(1, jas.ncoef), "gcoef")
    _check(load().xtc_backward(ctypes.byref(dp.c), ctypes.byref(jas), prec, _ptr(gV2), _ptr(gh1), float(gE0),
                               _ptr(gcoef), _ptr(ws), ws.numel(), _stream(stream)))


def xtc_lowdin(N, Ng, chi, w, phi, lam, ws, stream=None):
    _dev(ws, 1, "ws", "uint8")
    _dev(chi, N * Ng, "chi")
    _dev(w, Ng, "w")
    _dev(phi, N * Ng, "phi")
    _dev(lam, N, "lambda", required=False)
    _check(load().xtc_lowdin(N, Ng, _ptr(chi), _ptr(w), _ptr(phi), _ptr(lam), _ptr(ws), ws.numel(),
                             _stream(stream)))


def xtc_lowdin_noalloc(N, Ng, chi, w, phi, lam, stream=None):
    """xtc_lowdin with the library's static device scratch (no workspace)."""
    _dev(chi, N * Ng, "chi")
    _dev(w, Ng, "w")
    _dev(phi, N * Ng, "phi")
    _dev(lam, N, "lambda", required=False)
    _check(load().xtc_lowdin_noalloc(N, Ng, _ptr(chi), _ptr(w), _ptr(phi), _ptr(lam), _stream(stream)))


def lowdin(chi, w, device="cuda"):
    """phi = S^{-1/2} chi and the eigenvalues of S on the device (FP64)."""
    import torch
    if np.ndim(chi) != 2 or np.shape(w) != (np.shape(chi)[1],):
        raise ValueError("chi must be [N][Ng] and w [Ng]")
    chi_t = torch.as_tensor(np.ascontiguousarray(chi, dtype=np.float64)).to(device)
    w_t = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(device)
    N, Ng = chi_t.shape
    n = load().xtc_lowdin_workspace_size(N, Ng)
    if n == 0:
        raise XtcError(XTC_E_ARG, last_error())
    ws = torch.empty(n, dtype=torch.uint8, device=device)
    phi = torch.empty_like(chi_t)
    lam = torch.empty(N, dtype=torch.float64, device=device)
    xtc_lowdin(N, Ng, chi_t, w_t, phi, lam, ws)
    return phi, lam


# ------------------------------------------------------------ whole pass --
def auto_chunk(dp: DeviceProblem, prec: int, chunk_rows: int | None, fraction: float = 0.4) -> int:
    """Grid rows per chunk: chunk_rows if given, else the largest of Ng, Ng/2,
    Ng/4, ... (multiples of 32) whose workspace takes at most `fraction` of
    the device memory that is free now."""
    import torch
    if chunk_rows:
        return min(dp.Ng, int(chunk_rows))
    free, _ = torch.cuda.mem_get_info()
    chunk = dp.Ng
    while chunk > 32 and xtc_workspace_size(dp, prec, chunk) > fraction * free:
        chunk = max(32, ((chunk // 2 + 31) // 32) * 32)
    return chunk


class Pass:
    """Device buffers of one forward pass: workspace, one K chunk, outputs."""

    def __init__(self, dp: DeviceProblem, prec: int = XTC_FP64, chunk_rows: int | None = None, device="cuda"):
        import torch
        self.dp, self.prec = dp, prec
        self.chunk = auto_chunk(dp, prec, chunk_rows)
        self.ldP = xtc_pair_ld(dp.N)
        nbytes = xtc_workspace_size(dp, prec, self.chunk)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.K = torch.empty((3, self.chunk, self.ldP), dtype=torch.float64, device=device)
        N = dp.N
        # open shell: spin blocks (aa, ab, bb) of V2 and (a, b) of h1
        ns = (3, 2) if dp.open_shell else None
        self.V2 = torch.empty(((ns[0],) if ns else ()) + (N, N, N, N), dtype=torch.float64, device=device)
        self.h1 = torch.empty(((ns[1],) if ns else ()) + (N, N), dtype=torch.float64, device=device)
        self.E0 = torch.empty((1,), dtype=torch.float64, device=device)

    def chunks(self):
        Ng = self.dp.Ng
        return [(g0, min(Ng, g0 + self.chunk)) for g0 in range(0, Ng, self.chunk)]

    def K_view(self, g0, g1):
        # a [3][g1-g0][ldP] contiguous view at the start of the chunk buffer
        import torch
        n = 3 * (g1 - g0) * self.ldP
        return self.K.view(-1)[:n].view(3, g1 - g0, self.ldP)

    def run(self, jas: XtcJastrow, two_body=True, one_body=True, stream=None, kflags=0):
        """The pass over all chunks; kflags: options of xtc_build_K only
        (XTC_K_OCC_FP64)."""
        xtc_prepare(self.dp, self.prec, self.chunk, self.ws, stream)
        ch = self.chunks()
        for i, (g0, g1) in enumerate(ch):
            flags = (XTC_RESET if i == 0 else 0) | (XTC_FINALIZE if i == len(ch) - 1 else 0)
            K = self.K_view(g0, g1)
            xtc_build_K(self.dp, jas, g0, g1, self.prec | kflags, K, self.ws, stream)
            if two_body:
                xtc_contract_2body(self.dp, K, g0, g1, self.prec, flags, self.V2, self.ws, stream)
            if one_body:
                reuse = XTC_REUSE_INTERMEDIATES if two_body else 0   # A, B of this chunk are in ws
                xtc_contract_1body_0body(self.dp, K, g0, g1, self.prec, flags | reuse, self.h1, self.E0, self.ws,
                                         stream)
        return self.V2, self.h1, self.E0


def forward(problem, prec="fp64", chunk_rows=None, device="cuda", jastrow=None, occ_fp64=False):
    """V2, h1, E0 (torch tensors on the device) for an inputs.Problem.
    occ_fp64: in the reduced forms, the occupied-occupied block of K with
    FP64 MFMA (XTC_K_OCC_FP64) instead of the integer-sliced products."""
    dp = device_problem(problem.xyz, problem.w, problem.phi, problem.occ, device,
                        getattr(problem, "occ_n", None), getattr(problem, "occ_n_beta", None))
    ps = Pass(dp, PRECISIONS[prec] if isinstance(prec, str) else prec, chunk_rows, device)
    V2, h1, E0 = ps.run(make_jastrow(jastrow or problem.jastrow), kflags=XTC_K_OCC_FP64 if occ_fp64 else 0)
    return V2, h1, E0


def tc_two_body(problem, dphi, prec="fp64", chunk_rows=None, device="cuda", jastrow=None, stream=None):
    """Two-body TC integrals K2[p][q][r][s] = K_pr^qs (xtc_tc_2body) for an
    inputs.Problem; dphi [3][N][Ng] host or device.  Builds K chunk by chunk."""
    import torch
    N, Ng = np.shape(problem.phi)
    if tuple(dphi.shape) != (3, N, Ng):
        raise ValueError(f"dphi must be [3][{N}][{Ng}], got {tuple(dphi.shape)}")
    dp = device_problem(problem.xyz, problem.w, problem.phi, problem.occ, device)
    p = (PRECISIONS[prec] if isinstance(prec, str) else prec) | XTC_WITH_TC2
    chunk = auto_chunk(dp, p, chunk_rows)
    L = load()
    ws = torch.empty(xtc_workspace_size(dp, p, chunk), dtype=torch.uint8, device=device)
    xtc_prepare(dp, p, chunk, ws, stream)
    ldP = xtc_pair_ld(dp.N)
    Kbuf = torch.empty((3 * chunk * ldP,), dtype=torch.float64, device=device)
    dphi_t = torch.as_tensor(np.ascontiguousarray(dphi, dtype=np.float64)).to(device) \
        if isinstance(dphi, np.ndarray) else dphi.to(device=device, dtype=torch.float64).contiguous()
    N = dp.N
    K2 = torch.empty((N, N, N, N), dtype=torch.float64, device=device)
    jas = make_jastrow(jastrow or problem.jastrow)
    ch = [(g0, min(dp.Ng, g0 + chunk)) for g0 in range(0, dp.Ng, chunk)]
    for i, (g0, g1) in enumerate(ch):
        flags = (XTC_RESET if i == 0 else 0) | (XTC_FINALIZE if i == len(ch) - 1 else 0)
        K = Kbuf[:3 * (g1 - g0) * ldP]
        xtc_build_K(dp, jas, g0, g1, p | XTC_K_REDUCED_OCC, K, ws, stream)
        _check(L.xtc_tc_2body(ctypes.byref(dp.c), ctypes.byref(jas), _ptr(dphi_t), _ptr(K), g0, g1, p, flags,
                              _ptr(K2), _ptr(ws), ws.numel(), _stream(stream)))
    return K2


def frozen_core(V2, h1, E0, core, active, stream=None):
    """Frozen-core folding (xtc_frozen_core) of closed-shell outputs on the device:
    returns (V2_act, h1_act, E_fc)."""
    import torch
    N = h1.shape[0]
    _dev(V2, N ** 4, "V2")
    _dev(h1, N ** 2, "h1")
    _dev(E0, 1, "E0")
    c = np.ascontiguousarray(core, dtype=np.int32)
    a = np.ascontiguousarray(active, dtype=np.int32)
    na = len(a)
    V = torch.empty((na,) * 4, dtype=torch.float64, device=V2.device)
    h = torch.empty((na, na), dtype=torch.float64, device=V2.device)
    E = torch.empty((1,), dtype=torch.float64, device=V2.device)
    ip = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(load().xtc_frozen_core(N, _ptr(V2), _ptr(h1), _ptr(E0), len(c), ip(c), na, ip(a), _ptr(V), _ptr(h),
                                  _ptr(E), _stream(stream)))
    return V, h, E


def power_jastrow(coef) -> XtcJastrow:
    j = XtcJastrow()
    j.kind, j.ncoef, j.b = 1, len(coef), 0.0
    for k, c in enumerate(coef):
        j.coef[k] = float(c)
    return j


def backward(dp: DeviceProblem, coef, gV2, gh1, gE0, prec="fp64", chunk_rows=None, device="cuda"):
    """dL/dc for L = gE0 E0 + <gh1, h1> + <gV2, V2> (device tensors or None), power Jastrow."""
    import torch
    p = (PRECISIONS[prec] if isinstance(prec, str) else prec) | XTC_WITH_BACKWARD
    chunk = auto_chunk(dp, p, chunk_rows)
    ws = torch.empty(xtc_workspace_size(dp, p, chunk), dtype=torch.uint8, device=device)
    xtc_prepare(dp, p, chunk, ws)
    g = torch.empty(len(coef), dtype=torch.float64, device=device)
    xtc_backward(dp, power_jastrow(coef), p, gV2, gh1, gE0, g, ws)
    return g


class XtcFunction:
    """torch.autograd.Function over the power-Jastrow coefficients:
    (V2, h1, E0) = XtcFunction.apply(coef, problem_on_device, prec, chunk_rows).
    The backward calls xtc_backward with the incoming output gradients as seeds
    (K is recomputed there, never stored)."""

    _F = None         # the torch.autograd.Function subclass, made on first use

    @classmethod
    def _cls(cls):
        if cls._F is not None:
            return cls._F
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, coef, dp, prec, chunk_rows):
                ps = Pass(dp, PRECISIONS[prec] if isinstance(prec, str) else prec, chunk_rows)
                V2, h1, E0 = ps.run(power_jastrow(coef.detach().cpu().tolist()))
                ctx.dp, ctx.prec, ctx.chunk = dp, prec, chunk_rows
                ctx.save_for_backward(coef)
                return V2.clone(), h1.clone(), E0.clone()

            @staticmethod
            def backward(ctx, gV2, gh1, gE0):
                (coef,) = ctx.saved_tensors
                gE = float(gE0.detach().cpu().reshape(-1)[0]) if gE0 is not None else 0.0
                g = backward(ctx.dp, coef.detach().cpu().tolist(),
                             gV2.contiguous() if gV2 is not None else None,
                             gh1.contiguous() if gh1 is not None else None, gE, ctx.prec, ctx.chunk)
                return g.to(coef.dtype).to(coef.device), None, None, None

        cls._F = _F
        return _F

    @classmethod
    def apply(cls, coef, dp, prec="fp64", chunk_rows=None):
        return cls._cls().apply(coef, dp, prec, chunk_rows)
