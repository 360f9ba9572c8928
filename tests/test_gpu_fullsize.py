"""The hot path at the full sizes of the measured workloads, in the launch
configuration bench.py times (N=128, 16 occupied, Ng=150 000, 20 chunks of
7500 rows in the reduced forms, 10 in FP64): sampled K entries against their
exact grid sums, the antisymmetry of the pair contraction of K, every form's
outputs against the oracle's values on an orbital subset (written by
tests/golden/make_subset_golden.py, which calls only the oracle) and the
reduced forms against the FP64 path, bitwise symmetry and determinism; the
adjoint at N=96, Ng=100 000 (closed and open shell) through the Euler
identity of the quadratic loss and central differences of the FP64 forward;
and forward + adjoint at N=160, Ng=250 000 with its peak device memory."""
import os

import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu

WORKLOAD = "N128-occ16-Ng150k"
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BARS = (1e-6, 1e-6, 1e-8)


def _load_golden(workload):
    g = np.load(os.path.join(GOLDEN_DIR, f"{workload}_subset.npz"), allow_pickle=False)
    return {k: g[k] for k in g.files}


def _regenerate(workload, golden):
    """The workload with the stored orthonormalisation matrix; its drawn
    inputs must reproduce the stored fingerprint."""
    p = inputs.make_workload(workload, lowdin=golden["X"])
    fp = inputs.input_fingerprint(p)
    dev = np.abs(fp - golden["fingerprint"]) / np.maximum(np.abs(golden["fingerprint"]), 1e-300)
    assert dev.max() < 1e-12, f"regenerated inputs differ from the stored ones: {dev.max():.2e}"
    return p


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def golden():
    """The oracle's subset values of the headline workload."""
    return _load_golden(WORKLOAD)


@pytest.fixture(scope="module")
def problem(golden):
    return _regenerate(WORKLOAD, golden)


def _against_golden(golden, V2, h1, E0, prec):
    """Max-abs differences of the subset outputs from the stored oracle values
    (V2 over its unique entries), checked against the bars."""
    S, idx = golden["S"], golden["idx"].astype(np.int64)
    Sv = S[idx]
    eV = float(np.abs(V2[Sv[:, 0], Sv[:, 1], Sv[:, 2], Sv[:, 3]] - golden["V2u"]).max())
    eh = float(np.abs(h1[np.ix_(S, S)] - golden["h1"]).max())
    E0o = float(golden["E0"][0])
    eE = abs(E0 - E0o)
    _note(f"  {prec} vs oracle on {len(S)} orbitals: |dV2| {eV:.2e} |dh1| {eh:.2e} |dE0| {eE:.2e} (E0 {E0o:.10f})")
    if prec == "fp64":
        assert eV < 1e-11 and eh < 1e-11 and eE < max(1e-11, 1e-12 * abs(E0o)), (eV, eh, eE)
    else:
        assert eV < BARS[0] and eh < BARS[1] and eE < BARS[2], (prec, eV, eh, eE)


def _chunk(prec, Ng):
    return -(-Ng // (10 if prec == "fp64" else 20))


def _pair(a, b, N):
    a, b = min(a, b), max(a, b)
    return a * N - a * (a - 1) // 2 + (b - a)


def test_full_size_K_entries(torch_cuda, problem):
    """One bench-sized chunk of K in FP64 and split BF16 x3 against exact grid
    sums (math.fsum over all 150 000 g') of sampled entries: FP64 to summation
    noise, the split form's BF16 pairs to 2^-15 of the sum of |terms|, its
    occupied-occupied pairs to the integer-sliced block's worst-case bound."""
    from oracle import explicit as ex
    from paper_2304_07006_amd import xtc
    p = problem
    N, Ng = p.N, p.Ng
    g0 = 10 * _chunk("bf16x3", Ng)
    g1 = g0 + _chunk("bf16x3", Ng)
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    jas = xtc.make_jastrow(p.jastrow)
    Ks = {}
    for prec in ("fp64", "bf16x3"):
        _note(f"case: {WORKLOAD} K rows [{g0},{g1}) {prec}")
        ps = xtc.Pass(dp, xtc.PRECISIONS[prec], g1 - g0)
        xtc.xtc_prepare(dp, ps.prec, ps.chunk, ps.ws)
        K = ps.K_view(g0, g1)
        xtc.xtc_build_K(dp, jas, g0, g1, ps.prec, K, ps.ws)
        torch_cuda.cuda.synchronize()
        Ks[prec] = K.cpu().numpy()
        del ps, K
        torch_cuda.cuda.empty_cache()
    occ = [int(k) for k in p.occ]
    rng = np.random.default_rng(11)
    samples = [(int(rng.integers(0, g1 - g0)), *sorted(int(x) for x in rng.integers(0, N, 2))) for _ in range(20)]
    samples += [(int(rng.integers(0, g1 - g0)), *sorted(int(x) for x in rng.choice(occ, 2))) for _ in range(8)]
    worst = {"fp64": 0.0, "bf16x3": 0.0}
    assert p.jastrow.kind == "pade"     # |d^x| <= |u'| <= 1/2: the integer block's d scale is 1
    for g, a, b in samples:
        e = ex.exact_K_entry(p.xyz, p.w, p.phi, p.jastrow, g0 + g, a, b)
        d = ex.grad1(p.xyz[g0 + g:g0 + g + 1], p.xyz, p.jastrow)[:, 0, :]
        rho = p.w * p.phi[a] * p.phi[b]
        bound = np.abs(d * rho).sum(axis=1)        # sum of |terms|
        P = _pair(a, b, N)
        both_occ = a in occ and b in occ
        for prec, K in Ks.items():
            err = np.abs(K[:, g, P] - e)
            if prec == "fp64":                     # summation noise
                tol = 1e-13 * (1.0 + bound)
            elif both_occ:
                # integer-sliced block: d and rho as six digits against the scales
                # S_d = 1 and S_P = the power of two above 2 max|rho_P|, each
                # within 2^-43 of its scale, and the left-out digit products
                # (order >= 8, digits <= 64 in magnitude) below 2.87e-13 S_d S_P
                # per point; plus summation noise
                S_P = np.ldexp(1.0, np.frexp(np.abs(rho).max())[1] + 1)
                tol = (1e-13 * (1.0 + bound) + 2.0**-43 * (np.abs(rho).sum() + S_P * np.abs(d).sum(axis=1))
                       + 2.87e-13 * S_P * np.count_nonzero(rho))
            else:                                  # split BF16 x3: 2^-16 per product
                tol = 2.0**-15 * bound + 1e-15
            assert np.all(err <= tol), (prec, g, a, b, err, tol)
            worst[prec] = max(worst[prec], float((err / (bound + 1e-300)).max()))
    _note(f"  max |dK| / sum|terms|: fp64 {worst['fp64']:.2e}, bf16x3 {worst['bf16x3']:.2e}")


def test_full_size_pair_antisymmetry(torch_cuda, problem):
    """sum_g rho_P(g) K^x_R(g) = -sum_g rho_R(g) K^x_P(g) (d^x is antisymmetric
    in g, g'), over all 20 split-BF16 chunks, on 192 sampled pairs."""
    import torch
    from paper_2304_07006_amd import xtc
    p = problem
    N, Ng = p.N, p.Ng
    chunk = _chunk("bf16x3", Ng)
    _note(f"case: {WORKLOAD} pair antisymmetry, bf16x3, chunks of {chunk}")
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    ps = xtc.Pass(dp, xtc.XTC_BF16X3, chunk)
    xtc.xtc_prepare(dp, ps.prec, ps.chunk, ps.ws)
    jas = xtc.make_jastrow(p.jastrow)
    rng = np.random.default_rng(12)
    ab = [tuple(sorted(int(x) for x in rng.integers(0, N, 2))) for _ in range(192)]
    cols = torch.tensor([_pair(a, b, N) for a, b in ab], device="cuda")
    ia = torch.tensor([a for a, _ in ab], device="cuda")
    ib = torch.tensor([b for _, b in ab], device="cuda")
    phi = torch.as_tensor(p.phi, device="cuda")
    w = torch.as_tensor(p.w, device="cuda")
    S = torch.zeros((3, len(ab), len(ab)), dtype=torch.float64, device="cuda")
    A = torch.zeros_like(S)
    for g0, g1 in ps.chunks():
        K = ps.K_view(g0, g1)
        xtc.xtc_build_K(dp, jas, g0, g1, ps.prec, K, ps.ws)
        rho = (w[g0:g1, None] * phi[ia, g0:g1].T * phi[ib, g0:g1].T)      # [rows][pairs]
        Kc = K.view(3, g1 - g0, -1)[:, :, cols]                              # [3][rows][pairs]
        for x in range(3):
            S[x] += rho.T @ Kc[x]
            A[x] += rho.abs().T @ Kc[x].abs()
    torch.cuda.synchronize()
    S, A = S.cpu().numpy(), A.cpu().numpy()
    asym = np.abs(S + S.transpose(0, 2, 1))
    bound = A + A.transpose(0, 2, 1)
    _note(f"  max |S + S^T| / bound {(asym / (bound + 1e-300)).max():.2e}; max |S| {np.abs(S).max():.2e}")
    assert np.all(asym <= 2.0**-15 * bound + 1e-15)


def test_full_size_forward_against_oracle_and_fp64(torch_cuda, problem, golden):
    """Every form at the bench configuration against the oracle's values on
    the 24-orbital subset (FP64: 1e-11; reduced forms: the 1e-6 Eh two-body,
    1e-6 one-body and 1e-8 zero-body bars), the reduced forms also against the
    FP64 path over all N^4 entries; bitwise symmetry of V2 and h1, bitwise
    determinism of two split-BF16 runs."""
    from paper_2304_07006_amd import xtc
    p = problem
    _note(f"case: {WORKLOAD} forward bf16x3 (x2), bf16x6, fp32, fp64 vs oracle subset and fp64")
    out = {}
    for prec, tag in (("bf16x3", "a"), ("bf16x3", "b"), ("bf16x6", "s"), ("fp32", "f"), ("fp64", "r")):
        V2, h1, E0 = xtc.forward(p, prec=prec, chunk_rows=_chunk(prec, p.Ng))
        out[tag] = (V2.cpu().numpy(), h1.cpu().numpy(), float(E0.cpu()[0]))
        del V2, h1, E0
        torch_cuda.cuda.empty_cache()
        if tag != "b":
            _against_golden(golden, *out[tag], prec)
    (Va, ha, Ea), (Vb, hb, Eb), (Vr, hr, Er) = out["a"], out["b"], out["r"]
    for tag, prec in (("a", "bf16x3"), ("s", "bf16x6"), ("f", "fp32")):
        V, h, E = out[tag]
        eV, eh, eE = np.abs(V - Vr).max(), np.abs(h - hr).max(), abs(E - Er)
        _note(f"  {prec} vs fp64: |dV2| {eV:.2e} |dh1| {eh:.2e} |dE0| {eE:.2e} (E0 = {Er:.10f})")
        assert eV < 1e-6 and eh < 1e-6 and eE < 1e-8, tag
    assert np.array_equal(Va, Vb) and np.array_equal(ha, hb) and Ea == Eb
    for V in (Va, Vr):
        for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
            assert np.array_equal(V, V.transpose(perm))
    assert np.array_equal(ha, ha.T) and np.array_equal(hr, hr.T)


def test_full_size_default_chunking(torch_cuda, problem):
    """Without chunk_rows the binding picks the largest halving of Ng whose
    workspace fits 40% of the free device memory.  The two-body term's FP32
    segments follow the chunk rows, so V2 changes within the reduced form's
    error (bar 1e-6); h1 and E0 are FP64 reductions."""
    from paper_2304_07006_amd import xtc
    p = problem
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    chunk = xtc.auto_chunk(dp, xtc.XTC_BF16X3, None)
    _note(f"case: {WORKLOAD} bf16x3 default chunk = {chunk} rows")
    del dp
    Va, ha, Ea = (t.cpu().numpy() for t in xtc.forward(p, prec="bf16x3"))
    torch_cuda.cuda.empty_cache()
    Vb, hb, Eb = (t.cpu().numpy() for t in xtc.forward(p, prec="bf16x3", chunk_rows=_chunk("bf16x3", p.Ng)))
    _note(f"  |dV2| {np.abs(Va - Vb).max():.2e} |dh1| {np.abs(ha - hb).max():.2e} |dE0| {abs(Ea[0] - Eb[0]):.2e}")
    assert 32 <= chunk <= p.Ng
    assert np.abs(Va - Vb).max() < 1e-6 and np.abs(ha - hb).max() < 1e-10 and abs(Ea[0] - Eb[0]) < 1e-12


def test_full_size_adjoint_euler(torch_cuda):
    """The loss E0 + <h1,D> + <V2,G> is homogeneous of degree 2 in the
    power-Jastrow coefficients, so c . dL/dc = 2L at any size; N=96,
    Ng=100 000, split BF16 x3 in 20 chunks (bench.py --backward)."""
    import bench
    wl = inputs.WORKLOADS["N96-occ12-Ng100k"]
    gold = _load_golden(wl.name)
    p = _regenerate(wl.name, gold)
    _note("case: N96-occ12-Ng100k adjoint bf16x3, Euler identity; forward vs the stored oracle values")
    keep = {}
    tf, tb, g, euler, _ = bench.run_backward(p, "bf16x3", _chunk("bf16x3", p.Ng), wl.aux_seed, 1, 0, keep)
    _note(f"  |c.g - 2L| / |2L| = {euler:.2e}; forward {tf:.2f} s, adjoint {tb:.2f} s")
    assert np.all(np.isfinite(g)) and euler < 1e-5
    _against_golden(gold, keep["V2"], keep["h1"], keep["E0"], "bf16x3")


def test_full_size_open_shell_adjoint_euler(torch_cuda):
    """The open-shell adjoint at N=96, Ng=100 000 (10 doubly and 4 singly
    occupied orbitals, spin-blocked seeds), split BF16 x3 in 20 chunks:
    c . dL/dc = 2L (bench.py --backward --density open:10,4)."""
    import bench
    wl = inputs.WORKLOADS["N96-occ12-Ng100k"]
    p = inputs.make_workload(wl.name)
    bench.apply_density(p, "open:10,4")
    _note("case: N96-occ12-Ng100k open shell 10+4 adjoint bf16x3, Euler identity")
    tf, tb, g, euler, _ = bench.run_backward(p, "bf16x3", _chunk("bf16x3", p.Ng), wl.aux_seed, 1, 0)
    _note(f"  |c.g - 2L| / |2L| = {euler:.2e}; forward {tf:.2f} s, adjoint {tb:.2f} s")
    assert np.all(np.isfinite(g)) and euler < 1e-5


def test_full_size_adjoint_central_differences(torch_cuda):
    """N=96, Ng=100 000, FP64: the adjoint against central differences of the
    FP64 forward with step 1e-5 on two coefficients (the loss is quadratic in
    the coefficients, so the difference quotient is exact up to rounding),
    1e-8 relative."""
    import bench
    from paper_2304_07006_amd import xtc
    wl = inputs.WORKLOADS["N96-occ12-Ng100k"]
    gold = _load_golden(wl.name)
    p = _regenerate(wl.name, gold)
    _note("case: N96-occ12-Ng100k adjoint fp64 vs central differences (h = 1e-5, k = 0, 5); forward vs oracle")
    keep = {}
    _, _, g, euler, _ = bench.run_backward(p, "fp64", _chunk("fp64", p.Ng), wl.aux_seed, 1, 0, keep)
    _against_golden(gold, keep["V2"], keep["h1"], keep["E0"], "fp64")
    D, G = bench.loss_weights_device(p.N, wl.aux_seed)
    coef = np.array(p.jastrow.coef)
    h = 1e-5

    def loss(c):
        jas = inputs.Jastrow("power", coef=tuple(float(x) for x in c))
        V2, h1, E0 = xtc.forward(p, prec="fp64", chunk_rows=_chunk("fp64", p.Ng), jastrow=jas)
        L = bench.loss_value(V2, h1, E0, D, G)
        del V2, h1, E0
        return L

    _note(f"  L = {keep['L']:.12e}, |c.g - 2L|/|2L| = {euler:.2e}")
    assert euler < 1e-10
    for k in (0, 5):
        e = np.zeros_like(coef)
        e[k] = h
        fd = (loss(coef + e) - loss(coef - e)) / (2 * h)
        rel = abs(fd - g[k]) / max(abs(g[k]), 1e-300)
        _note(f"  k={k}: adjoint {g[k]:.12e}, central difference {fd:.12e}, relative {rel:.2e}")
        assert rel < 1e-8, (k, fd, g[k])


def test_largest_workload_forward_and_adjoint(torch_cuda):
    """N=160, 20 occupied, Ng=250 000, split BF16 x3 in 20 chunks (bench.py
    --backward --workload N160-occ20-Ng250k): forward outputs against the
    stored oracle values on occ + 8 virtual orbitals and the FP64 path to the
    bars (the FP64 path to the oracle's 1e-11), c . dL/dc = 2 L to 1e-5 with K recomputed in the
    adjoint, and the peak device memory of the split-BF16 forward + adjoint
    within its stated bound (the larger of the two workspaces plus the
    outputs, the loss weights and the K chunk, plus 2%)."""
    import bench
    from paper_2304_07006_amd import xtc
    wl = inputs.WORKLOADS["N160-occ20-Ng250k"]
    gold = _load_golden(wl.name)
    p = _regenerate(wl.name, gold)
    chunk = _chunk("bf16x3", p.Ng)
    _note(f"case: {wl.name} forward + adjoint bf16x3, chunk={chunk}; forward vs the stored oracle values")
    torch_cuda.cuda.reset_peak_memory_stats()
    keep = {}
    tf, tb, g, euler, peak = bench.run_backward(p, "bf16x3", chunk, wl.aux_seed, 1, 0, keep)
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    N, ldP = p.N, xtc.xtc_pair_ld(p.N)
    ws_f = xtc.xtc_workspace_size(dp, xtc.XTC_BF16X3, chunk)
    ws_b = xtc.xtc_workspace_size(dp, xtc.XTC_BF16X3 | xtc.XTC_WITH_BACKWARD, chunk)
    inputs_b = (p.Ng * 4 + N * p.Ng) * 8
    outs = (2 * N ** 4 + N * N + 1) * 8 + 3 * chunk * ldP * 8     # V2, G (seed), h1, D, E0; K chunk
    bound = 1.02 * (max(ws_f, ws_b) + outs + inputs_b)
    _note(f"  forward {tf:.2f} s, adjoint {tb:.2f} s, |c.g - 2L|/|2L| = {euler:.2e}, "
          f"peak {peak / 1e9:.1f} GB (bound {bound / 1e9:.1f} GB; workspaces {ws_f / 1e9:.1f} / {ws_b / 1e9:.1f} GB)")
    assert np.all(np.isfinite(g)) and euler < 1e-5
    assert peak <= bound
    del dp
    torch_cuda.cuda.empty_cache()
    _against_golden(gold, keep["V2"], keep["h1"], keep["E0"], "bf16x3")
    V2r, h1r, E0r = (t.cpu().numpy() for t in xtc.forward(p, prec="fp64", chunk_rows=_chunk("fp64", p.Ng)))
    _against_golden(gold, V2r, h1r, float(E0r[0]), "fp64")
    eV = np.abs(keep["V2"] - V2r).max()
    eh = np.abs(keep["h1"] - h1r).max()
    eE = abs(keep["E0"] - float(E0r[0]))
    _note(f"  bf16x3 vs fp64: |dV2| {eV:.2e} |dh1| {eh:.2e} |dE0| {eE:.2e} (E0 {float(E0r[0]):.10f})")
    assert eV < BARS[0] and eh < BARS[1] and eE < BARS[2]
