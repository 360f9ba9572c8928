"""The occupied-occupied block of K in the reduced forms, computed by default
from exact integer products of six-digit fixed-point operands (int8 MFMA,
int32 sums; up to 144 occupied pairs, one column group): against the FP64
MFMA block (XTC_K_OCC_FP64), the FP64 build and exact sums of the
definition, over one to nine column tiles, one and many int32 segments,
ragged row ranges and both Jastrow forms; above 144 pairs the FP64 block.

Tolerance: each operand is within 2^-43 of its power-of-two scale, and the
digit products left out (order 8 and up) add about 2^-44 S_d S_P per grid
point with random sign, so the block differs from exact sums by about
sqrt(Ng) 2^-44 S_d S_P (4e-11 of max|K| measured and emulated at N=64 on
3001 points, and less on larger grids, where S_P shrinks with the weights).
2^-30 of max|K| holds that with a wide margin and is still 2^14 times
tighter than the split-BF16 block's error."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu

TOL_REL = 2.0**-30


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _K(problem, g0, g1, prec, kflags=0):
    import torch
    from paper_2304_07006_amd import xtc
    prec = xtc.PRECISIONS[prec]
    dp = xtc.device_problem(problem.xyz, problem.w, problem.phi, problem.occ)
    ps = xtc.Pass(dp, prec, g1 - g0)
    xtc.xtc_prepare(dp, prec, ps.chunk, ps.ws)
    K = ps.K_view(g0, g1)
    xtc.xtc_build_K(dp, xtc.make_jastrow(problem.jastrow), g0, g1, prec | kflags, K, ps.ws)
    torch.cuda.synchronize()
    return K.cpu().numpy()


def _occ_cols(p):
    N = p.N
    occ = sorted(int(k) for k in p.occ)
    return [a * N - a * (a - 1) // 2 + (b - a) for i, a in enumerate(occ) for b in occ[i:]]


# (N, nocc, Ng, centres, Jastrow, g0, g1): 36 pairs in 3 tiles; 91 pairs in
# 6 tiles (power Jastrow; an even tile count: stage blocks padded to 4 KB);
# 136 pairs in 9 tiles (the most one group holds, the N=128 tiling); 10 pairs
# on 300 000 points (5 int32 segments of at most 65 536 points)
CASES = [
    (64, 8, 3001, 8, "pade", 500, 1800),
    (24, 13, 2501, 6, "power16", 37, 1190),
    (40, 16, 2048, 5, "pade", 0, 2048),
    (16, 4, 300000, 4, "pade", 123457, 123532),
]


@pytest.mark.parametrize("case", CASES, ids=["N64-occ8", "N24-occ13-power", "N40-occ16", "N16-occ4-Ng300k"])
def test_integer_block_against_fp64_block(torch_cuda, case):
    from paper_2304_07006_amd import xtc
    N, nocc, Ng, nc, jk, g0, g1 = case
    p = inputs.make_problem(N, nocc, Ng, nc, "chain", jk, seed=61)
    _note(f"case: N{N} occ{nocc} Ng{Ng} {jk} K rows [{g0},{g1}) bf16x3 integer vs FP64 occupied block")
    Ki = _K(p, g0, g1, "bf16x3")
    Kf = _K(p, g0, g1, "bf16x3", kflags=xtc.XTC_K_OCC_FP64)
    cols = _occ_cols(p)
    other = np.setdiff1d(np.arange(Ki.shape[2]), cols)
    assert np.array_equal(Ki[:, :, other], Kf[:, :, other])
    scale = np.abs(Kf[:, :, cols]).max()
    e = np.abs(Ki[:, :, cols] - Kf[:, :, cols]).max()
    _note(f"  max |dK| {e:.2e} = {e / scale:.2e} of max |K_occ| {scale:.2e}")
    assert np.all(np.isfinite(Ki))
    assert e < TOL_REL * scale


def test_more_than_one_column_group_uses_the_fp64_block(torch_cuda):
    """Above 144 occupied pairs (17 occupied orbitals: 153) the reduced forms'
    occupied block is the FP64 one: the default K equals the XTC_K_OCC_FP64 K
    bitwise."""
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(24, 17, 1500, 6, "chain", "power16", seed=63)
    _note("case: N24 occ17 Ng1500 power: default occupied block = FP64 block")
    Ki = _K(p, 100, 900, "bf16x3")
    Kf = _K(p, 100, 900, "bf16x3", kflags=xtc.XTC_K_OCC_FP64)
    assert np.array_equal(Ki, Kf)


def test_power_jastrow_without_a_finite_scale_uses_the_fp64_block(torch_cuda):
    """A power Jastrow whose |u'| bound is not finite in FP64 (a coefficient
    of 1e300) gets no integer scale: its occupied pairs come from the FP64
    block, bitwise equal to the XTC_K_OCC_FP64 build."""
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(24, 4, 1200, 6, "chain", "power16", seed=64)
    p.jastrow = inputs.Jastrow("power", coef=(1e300,) + (0.0,) * 15)
    _note("case: N24 occ4 Ng1200 power Jastrow with a 1e300 coefficient: FP64 occupied block")
    cols = _occ_cols(p)
    Ki = _K(p, 0, 600, "bf16x3")[:, :, cols]
    Kf = _K(p, 0, 600, "bf16x3", kflags=xtc.XTC_K_OCC_FP64)[:, :, cols]
    assert np.all(np.isfinite(Kf)) and np.array_equal(Ki, Kf)


def test_integer_block_against_fp64_build_and_exact_sums(torch_cuda):
    """The block against the FP64 path's K (a separate kernel) and against
    exact (math.fsum) sums of the definition at sampled rows and pairs."""
    from oracle import explicit as ex
    p = inputs.make_workload("N64-occ8-Ng50k", Ng=3001)
    _note("case: N64-occ8-Ng3001 K rows [0,3001) integer block vs FP64 build and exact sums")
    Ki = _K(p, 0, 3001, "bf16x3")
    K64 = _K(p, 0, 3001, "fp64")
    cols = _occ_cols(p)
    scale = np.abs(K64[:, :, cols]).max()
    e = np.abs(Ki[:, :, cols] - K64[:, :, cols]).max()
    _note(f"  vs FP64 build: max |dK| {e:.2e} = {e / scale:.2e} of max |K_occ|")
    assert e < TOL_REL * scale
    occ = sorted(int(k) for k in p.occ)
    N = p.N
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(24):
        g = int(rng.integers(0, 3001))
        i, j = sorted(int(x) for x in rng.integers(0, len(occ), size=2))
        a, b = occ[i], occ[j]
        P = a * N - a * (a - 1) // 2 + (b - a)
        ref = ex.exact_K_entry(p.xyz, p.w, p.phi, p.jastrow, g, a, b)
        worst = max(worst, float(np.abs(Ki[:, g, P] - ref).max()))
    _note(f"  vs exact sums: max |dK| {worst:.2e}")
    assert worst < TOL_REL * scale


def test_integer_block_is_the_same_in_every_reduced_form(torch_cuda):
    """The block depends only on the FP64 pair densities and positions: the
    three reduced forms give it bitwise equal."""
    p = inputs.make_problem(32, 6, 2100, 4, "chain", "power16", seed=62)
    _note("case: N32-occ6-Ng2100 power: integer block in fp32, bf16x3, bf16x6")
    cols = _occ_cols(p)
    Ks = [_K(p, 100, 1333, f)[:, :, cols] for f in ("fp32", "bf16x3", "bf16x6")]
    assert np.array_equal(Ks[0], Ks[1]) and np.array_equal(Ks[1], Ks[2])


def test_forward_with_either_occupied_block(torch_cuda):
    """xtc.forward in split BF16 x3 with the integer (default) and the FP64
    occupied block: both within the bars of the oracle, and within FP64-class
    noise of each other (only the occupied block differs between them)."""
    from oracle import factorised as fb
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(24, 5, 1500, 6, "chain", "pade", seed=65)
    _note("case: N24 occ5 Ng1500 forward bf16x3 with the integer and the FP64 occupied block")
    V2o, h1o, E0o = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    outs = []
    for occ_fp64 in (False, True):
        V2, h1, E0 = (t.cpu().numpy() for t in xtc.forward(p, prec="bf16x3", chunk_rows=600, occ_fp64=occ_fp64))
        assert np.abs(V2 - V2o).max() < 1e-6 and np.abs(h1 - h1o).max() < 1e-6 and abs(E0[0] - E0o) < 1e-8
        outs.append((V2, h1, float(E0[0])))
    (Vi, hi, Ei), (Vf, hf, Ef) = outs
    _note(f"  integer vs FP64 block: |dV2| {np.abs(Vi - Vf).max():.2e} |dh1| {np.abs(hi - hf).max():.2e} "
          f"|dE0| {abs(Ei - Ef):.2e}")
    assert np.abs(Vi - Vf).max() < 1e-9 and np.abs(hi - hf).max() < 1e-10 and abs(Ei - Ef) < 1e-10
