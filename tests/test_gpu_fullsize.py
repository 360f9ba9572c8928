"""The hot path at the full sizes of the measured workloads, in the launch
configuration bench.py times (N=128, 16 occupied, Ng=150 000, 20 chunks of
7500 rows in split BF16 x3, 10 in FP64): sampled K entries against their exact
grid sums, the antisymmetry of the pair contraction of K, the split-BF16
and FP32 outputs against the FP64 path to the bars, bitwise symmetry and determinism;
and the adjoint at N=96, Ng=100 000 (closed and open shell) through the
Euler identity of the quadratic loss."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu

WORKLOAD = "N128-occ16-Ng150k"


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def problem():
    return inputs.make_workload(WORKLOAD)


def _chunk(prec, Ng):
    return -(-Ng // (10 if prec == "fp64" else 20))


def _pair(a, b, N):
    a, b = min(a, b), max(a, b)
    return a * N - a * (a - 1) // 2 + (b - a)


def test_full_size_K_entries(torch_cuda, problem):
    """One bench-sized chunk of K in FP64 and split BF16 x3 against exact grid
    sums (math.fsum over all 150 000 g') of sampled entries."""
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
    for g, a, b in samples:
        e = ex.exact_K_entry(p.xyz, p.w, p.phi, p.jastrow, g0 + g, a, b)
        d = ex.grad1(p.xyz[g0 + g:g0 + g + 1], p.xyz, p.jastrow)[:, 0, :]
        bound = np.abs(d * (p.w * p.phi[a] * p.phi[b])).sum(axis=1)        # sum of |terms|
        P = _pair(a, b, N)
        both_occ = a in occ and b in occ
        for prec, K in Ks.items():
            err = np.abs(K[:, g, P] - e)
            # FP64 (and the FP64 occupied block of the split form): summation
            # noise; split BF16 x3: 2^-16 per product, bounded by 2^-15 sum|terms|
            tol = 1e-13 * (1.0 + bound) if (prec == "fp64" or both_occ) else 2.0**-15 * bound + 1e-15
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


def test_full_size_forward_against_fp64(torch_cuda, problem):
    """Split BF16 x3 at the bench configuration, and the FP32 form in the same
    chunks, against the FP64 path: the 1e-6 Eh two-body bar (one-body 1e-6,
    zero-body 1e-8); bitwise symmetry of V2 and h1, bitwise determinism of two
    split-BF16 runs."""
    from paper_2304_07006_amd import xtc
    p = problem
    _note(f"case: {WORKLOAD} forward bf16x3 (x2) and fp32 vs fp64")
    out = {}
    for prec, tag in (("bf16x3", "a"), ("bf16x3", "b"), ("fp32", "f"), ("fp64", "r")):
        V2, h1, E0 = xtc.forward(p, prec=prec, chunk_rows=_chunk(prec, p.Ng))
        out[tag] = (V2.cpu().numpy(), h1.cpu().numpy(), float(E0.cpu()[0]))
        del V2, h1, E0
        torch_cuda.cuda.empty_cache()
    (Va, ha, Ea), (Vb, hb, Eb), (Vr, hr, Er) = out["a"], out["b"], out["r"]
    for tag in ("a", "f"):
        V, h, E = out[tag]
        eV, eh, eE = np.abs(V - Vr).max(), np.abs(h - hr).max(), abs(E - Er)
        _note(f"  {'bf16x3' if tag == 'a' else 'fp32'}: |dV2| {eV:.2e} |dh1| {eh:.2e} |dE0| {eE:.2e} (E0 = {Er:.10f})")
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
    p = inputs.make_workload(wl.name)
    _note("case: N96-occ12-Ng100k adjoint bf16x3, Euler identity")
    tf, tb, g, euler, _ = bench.run_backward(p, "bf16x3", _chunk("bf16x3", p.Ng), wl.aux_seed, 1, 0)
    _note(f"  |c.g - 2L| / |2L| = {euler:.2e}; forward {tf:.2f} s, adjoint {tb:.2f} s")
    assert np.all(np.isfinite(g)) and euler < 1e-5


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
