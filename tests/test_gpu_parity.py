"""GPU parity: the HIP path (through the C ABI) against the CPU oracle."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu

TOL_ABS = 1e-11      # FP64 summation-order noise on outputs of size <= ~1


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _run(problem, prec="fp64", chunk_rows=None):
    from paper_2304_07006_amd import xtc
    V2, h1, E0 = xtc.forward(problem, prec=prec, chunk_rows=chunk_rows)
    return V2.cpu().numpy(), h1.cpu().numpy(), float(E0.cpu().numpy()[0])


def _K(problem, g0, g1, chunk_rows=None, prec=None, kflags=0):
    """Grid intermediate of rows [g0,g1) through xtc_prepare + xtc_build_K."""
    import torch
    from paper_2304_07006_amd import xtc
    prec = xtc.XTC_FP64 if prec is None else xtc.PRECISIONS[prec]
    dp = xtc.device_problem(problem.xyz, problem.w, problem.phi, problem.occ)
    ps = xtc.Pass(dp, prec, chunk_rows or (g1 - g0))
    xtc.xtc_prepare(dp, prec, ps.chunk, ps.ws)
    K = ps.K_view(g0, g1)
    xtc.xtc_build_K(dp, xtc.make_jastrow(problem.jastrow), g0, g1, prec | kflags, K, ps.ws)
    torch.cuda.synchronize()
    return K.cpu().numpy()


def _unpack(Kp, N):
    """[3][rows][ldP] packed pairs -> [3][rows][N][N]."""
    out = np.zeros(Kp.shape[:2] + (N, N))
    P = 0
    for p in range(N):
        for q in range(p, N):
            out[:, :, p, q] = Kp[:, :, P]
            out[:, :, q, p] = Kp[:, :, P]
            P += 1
    return out


def test_tiny_against_explicit_L(torch_cuda):
    """N=8, 2 occupied, Ng=2000 against the explicit six-index L (tier A)."""
    from oracle import explicit as ex
    p = inputs.make_workload("N8-occ2-Ng2k")
    _note("case: N8-occ2-Ng2k fp64 vs explicit L")
    A = ex.tier_a(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    V2, h1, E0 = _run(p)
    assert np.abs(V2 - A["V2"]).max() < TOL_ABS
    assert np.abs(h1 - A["h1"]).max() < TOL_ABS
    assert abs(E0 - A["E0"]) < TOL_ABS


def test_tiny_K_entries(torch_cuda):
    from oracle import explicit as ex
    p = inputs.make_workload("N8-occ2-Ng2k")
    _note("case: N8-occ2-Ng2k K rows [100,1700)")
    K = _K(p, 100, 1700)
    N = p.N
    rng = np.random.default_rng(0)
    Ku = _unpack(K, N)
    for _ in range(40):
        g = int(rng.integers(0, 1600))
        a, b = sorted(int(x) for x in rng.integers(0, N, size=2))
        e = ex.exact_K_entry(p.xyz, p.w, p.phi, p.jastrow, 100 + g, a, b)
        assert np.abs(Ku[:, g, a, b] - e).max() < 1e-14
    ldP = K.shape[2]
    assert np.all(K[:, :, N * (N + 1) // 2:ldP] == 0.0)


def test_reduced_occ_option(torch_cuda):
    """xtc_build_K in split BF16 with XTC_K_REDUCED_OCC, XTC_K_OCC_FP64 and
    neither: the pairs outside the occupied-occupied block are bitwise the
    same; the block is the FP64 build to summation noise with XTC_K_OCC_FP64,
    within the integer block's 2^-30 of max|K| by default (its own tests
    hold it there against exact sums), and in the reduced arithmetic only
    with XTC_K_REDUCED_OCC."""
    from paper_2304_07006_amd import xtc
    p = inputs.make_workload("N64-occ8-Ng50k", Ng=3001)
    _note("case: N64-occ8-Ng3001 K rows [500,1800) bf16x3 default / XTC_K_OCC_FP64 / XTC_K_REDUCED_OCC")
    K64 = _K(p, 500, 1800)
    Kf = _K(p, 500, 1800, prec="bf16x3")
    K8 = _K(p, 500, 1800, prec="bf16x3", kflags=xtc.XTC_K_OCC_FP64)
    Kr = _K(p, 500, 1800, prec="bf16x3", kflags=xtc.XTC_K_REDUCED_OCC)
    N = p.N
    occ = sorted(int(k) for k in p.occ)
    cols = [a * N - a * (a - 1) // 2 + (b - a) for i, a in enumerate(occ) for b in occ[i:]]
    other = np.setdiff1d(np.arange(K64.shape[2]), cols)
    assert np.array_equal(Kf[:, :, other], Kr[:, :, other])
    assert np.array_equal(K8[:, :, other], Kr[:, :, other])
    scale = np.abs(K64).max()
    assert np.abs(K8[:, :, cols] - K64[:, :, cols]).max() < 1e-13 * scale
    assert np.abs(Kf[:, :, cols] - K64[:, :, cols]).max() < 2.0**-30 * scale
    er = np.abs(Kr[:, :, cols] - K64[:, :, cols]).max()
    _note(f"  reduced occupied block: max |dK| {er:.2e} (max |K| {scale:.2e})")
    assert 0 < er < 2.0**-16 * scale


@pytest.mark.parametrize("chunk_rows", [None, 1000])
def test_mid_against_factorised(torch_cuda, chunk_rows):
    """N=64, 8 occupied on a 3001-point grid (ragged in rows, pairs, chunks)."""
    from oracle import factorised as fb
    p = inputs.make_workload("N64-occ8-Ng50k", Ng=3001)
    _note(f"case: N64-occ8-Ng3001 fp64 chunk={chunk_rows}")
    V2o, h1o, E0o = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    V2, h1, E0 = _run(p, chunk_rows=chunk_rows)
    assert np.abs(V2 - V2o).max() < TOL_ABS
    assert np.abs(h1 - h1o).max() < TOL_ABS
    assert abs(E0 - E0o) < TOL_ABS


def test_power_jastrow_random_occ(torch_cuda):
    """16-term power Jastrow, seeded random occupied set, N=24."""
    from oracle import factorised as fb
    occ = inputs.random_occ(24, 5, seed=3)
    p = inputs.make_problem(24, 5, 1500, 6, "chain", "power16", seed=21, occ=occ)
    _note("case: N24 power16 random occ")
    V2o, h1o, E0o = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    V2, h1, E0 = _run(p, chunk_rows=700)
    assert np.abs(V2 - V2o).max() < TOL_ABS
    assert np.abs(h1 - h1o).max() < TOL_ABS
    assert abs(E0 - E0o) < TOL_ABS


def test_symmetry_and_determinism(torch_cuda):
    p = inputs.make_workload("N64-occ8-Ng50k", Ng=2500)
    _note("case: N64-occ8-Ng2500 symmetry + determinism")
    V2, h1, E0 = _run(p, chunk_rows=900)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(V2, V2.transpose(perm))
    assert np.array_equal(h1, h1.T)
    V2b, h1b, E0b = _run(p, chunk_rows=900)
    assert np.array_equal(V2, V2b) and np.array_equal(h1, h1b) and E0 == E0b


def test_single_occupied_E0_zero(torch_cuda):
    p = inputs.make_problem(8, 1, 700, 2, "pair", "pade", seed=4)
    _note("case: N8 n=1")
    V2, h1, E0 = _run(p)
    assert abs(E0) < 1e-15


# ----------------------------------------------------------- reduced forms --
TOL_2BODY_LP = 1e-6      # two-body bar of the reduced-precision forms (Eh)
TOL_1BODY_LP = 1e-6      # one-body (the paper is silent; same bar as two-body)
TOL_0BODY_LP = 1e-8      # zero-body bar: met by the FP64 occupied-occupied block


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_reduced_forms_against_factorised(torch_cuda, prec):
    from oracle import factorised as fb
    p = inputs.make_workload("N64-occ8-Ng50k", Ng=3001)
    _note(f"case: N64-occ8-Ng3001 {prec} chunk=1000")
    V2o, h1o, E0o = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    V2, h1, E0 = _run(p, prec=prec, chunk_rows=1000)
    eV, eh, eE = np.abs(V2 - V2o).max(), np.abs(h1 - h1o).max(), abs(E0 - E0o)
    _note(f"  {prec}: |dV2| {eV:.2e} |dh1| {eh:.2e} |dE0| {eE:.2e}")
    assert eV < TOL_2BODY_LP and eh < TOL_1BODY_LP and eE < TOL_0BODY_LP
    for perm in [(1, 0, 2, 3), (2, 3, 0, 1)]:
        assert np.array_equal(V2, V2.transpose(perm))
    assert np.array_equal(h1, h1.T)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_reduced_forms_power_jastrow(torch_cuda, prec):
    from oracle import factorised as fb
    occ = inputs.random_occ(24, 5, seed=3)
    p = inputs.make_problem(24, 5, 1500, 6, "chain", "power16", seed=21, occ=occ)
    _note(f"case: N24 power16 random occ {prec}")
    V2o, h1o, E0o = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    V2, h1, E0 = _run(p, prec=prec, chunk_rows=700)
    assert np.abs(V2 - V2o).max() < TOL_2BODY_LP
    assert np.abs(h1 - h1o).max() < TOL_1BODY_LP
    assert abs(E0 - E0o) < TOL_0BODY_LP


def test_reduced_form_occ_block_is_fp64_and_deterministic(torch_cuda):
    """In the reduced forms the occupied-occupied K columns are FP64 (summed in
    segments), so E0 agrees with the FP64 path to rounding; repeated runs are
    bitwise identical."""
    p = inputs.make_workload("N64-occ8-Ng50k", Ng=2200)
    _note("case: N64-occ8-Ng2200 bf16x3 vs fp64 E0, determinism")
    _, _, E64 = _run(p, prec="fp64", chunk_rows=800)
    V2a, h1a, Ea = _run(p, prec="bf16x3", chunk_rows=800)
    V2b, h1b, Eb = _run(p, prec="bf16x3", chunk_rows=800)
    assert abs(Ea - E64) < 1e-12 * max(1.0, abs(E64))
    assert np.array_equal(V2a, V2b) and np.array_equal(h1a, h1b) and Ea == Eb


# ----------------------------------------------------------------- Loewdin --
@pytest.mark.parametrize("name,Ng", [("N8-occ2-Ng2k", None), ("N64-occ8-Ng50k", 3001), ("N128-occ16-Ng150k", 6000)])
def test_lowdin_against_oracle(torch_cuda, name, Ng):
    """GPU Loewdin vs the oracle's (eigh-based) one; both are exact up to
    eps * cond(S), which sets the tolerance."""
    from oracle import lowdin as ol
    from paper_2304_07006_amd import xtc
    p = inputs.make_workload(name, Ng=Ng)
    _note(f"case: lowdin {name} Ng={p.Ng}")
    phi_o, C, lam_o = ol.lowdin(p.chi, p.w)
    phi_g, lam_g = xtc.lowdin(p.chi, p.w)
    phi_g = phi_g.cpu().numpy()
    cond = lam_o.max() / lam_o.min()
    tol = 50 * np.finfo(float).eps * cond * np.abs(phi_o).max()
    err = np.abs(phi_g - phi_o).max()
    _note(f"  cond(S) {cond:.2e}  max|dphi| {err:.2e}  tol {tol:.2e}")
    assert err < tol
    S = (phi_g * p.w) @ phi_g.T
    assert np.abs(S - np.eye(p.N)).max() < 50 * np.finfo(float).eps * cond
    assert np.allclose(np.sort(lam_g.cpu().numpy()), np.sort(lam_o), rtol=1e-9, atol=1e-14 * lam_o.max())


# ------------------------------------------------- intermediates reuse flag --
@pytest.mark.parametrize("case", ["closed-fp64", "closed-bf16x3", "open-bf16x3"])
def test_reuse_intermediates_is_bitwise_recompute(torch_cuda, case):
    """xtc_contract_1body_0body with XTC_REUSE_INTERMEDIATES right after
    xtc_contract_2body (what the forward pass does) gives bitwise the h1 and
    E0 of the same call recomputing the intermediates from K, over several
    ragged chunks; open shell: both spin channels' intermediates are kept."""
    import torch
    from paper_2304_07006_amd import xtc
    shell, prec = case.split("-")
    if shell == "open":
        k, na, nb = inputs.open_shell_occupations(3, 2)
        p = inputs.make_problem(24, 5, 1900, 6, "chain", "pade", seed=71, occ=k)
        p.occ_n, p.occ_n_beta = na, nb
    else:
        p = inputs.make_problem(24, 4, 1900, 6, "chain", "pade", seed=71)
    _note(f"case: N24 Ng1900 {case} reuse vs recompute, chunks of 700")
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ, occ_n=getattr(p, "occ_n", None),
                            occ_n_beta=getattr(p, "occ_n_beta", None))
    jas = xtc.make_jastrow(p.jastrow)
    out = {}
    for reuse in (0, xtc.XTC_REUSE_INTERMEDIATES):
        ps = xtc.Pass(dp, xtc.PRECISIONS[prec], 700)
        xtc.xtc_prepare(dp, ps.prec, ps.chunk, ps.ws)
        ch = ps.chunks()
        for i, (g0, g1) in enumerate(ch):
            flags = (xtc.XTC_RESET if i == 0 else 0) | (xtc.XTC_FINALIZE if i == len(ch) - 1 else 0)
            K = ps.K_view(g0, g1)
            xtc.xtc_build_K(dp, jas, g0, g1, ps.prec, K, ps.ws)
            xtc.xtc_contract_2body(dp, K, g0, g1, ps.prec, flags, ps.V2, ps.ws)
            xtc.xtc_contract_1body_0body(dp, K, g0, g1, ps.prec, flags | reuse, ps.h1, ps.E0, ps.ws)
        torch.cuda.synchronize()
        out[reuse] = (ps.V2.cpu().numpy(), ps.h1.cpu().numpy(), ps.E0.cpu().numpy())
    (Va, ha, Ea), (Vb, hb, Eb) = out[0], out[xtc.XTC_REUSE_INTERMEDIATES]
    assert np.array_equal(Va, Vb) and np.array_equal(ha, hb) and np.array_equal(Ea, Eb)
    assert np.abs(ha).max() > 0
