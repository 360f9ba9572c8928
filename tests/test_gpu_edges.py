"""Edge cases of the HIP path against the oracle: the largest supported N
(256) with the largest occupied set the on-chip staging of the intermediates
takes (19: nocc N 32 B within 159 KB), checked on an orbital subset; a
single orbital; every orbital occupied; a grid smaller than one tile; a
single grid point."""
import numpy as np
import pytest

from paper_2304_07006_amd import inputs

pytestmark = pytest.mark.gpu

TOL_ABS = 1e-11
BARS = (1e-6, 1e-6, 1e-8)   # two-, one-, zero-body bars of the reduced forms (Eh)


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _check(V2, h1, E0, ref, prec):
    V2o, h1o, E0o = ref
    scale = max(1.0, float(np.abs(V2o).max()))
    e = (np.abs(V2 - V2o).max(), np.abs(h1 - h1o).max(), abs(E0 - E0o))
    _note(f"  {prec}: |dV2| {e[0]:.2e} |dh1| {e[1]:.2e} |dE0| {e[2]:.2e} (max |V2| {scale:.2e})")
    if prec == "fp64":
        assert max(e) < TOL_ABS * scale
    else:
        assert e[0] < BARS[0] and e[1] < BARS[1] and e[2] < BARS[2]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_largest_N_on_an_orbital_subset(torch_cuda, prec):
    """N=256, 19 occupied, Ng=1500 in chunks of 700 rows.  The closed-shell
    outputs restricted to orbitals that include every occupied one equal the
    outputs of the problem built on that subset alone (the sums over k run
    over occupied orbitals only; pinned on the oracle), so the oracle runs on
    the 19 occupied plus 12 virtual orbitals."""
    import torch
    from oracle import factorised as fb
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(256, 19, 1500, 16, "chain", "pade", seed=61)
    _note(f"case: N=256 n=19 Ng=1500 chunk=700 {prec}")
    rng = np.random.default_rng(61)
    virt = np.sort(rng.choice(np.arange(19, 256), 12, replace=False))
    sub = np.concatenate([np.asarray(p.occ), virt])
    V2, h1, E0 = xtc.forward(p, prec=prec, chunk_rows=700)
    s = torch.as_tensor(sub, device=V2.device)
    V2s = V2[s][:, s][:, :, s][:, :, :, s].cpu().numpy()
    h1s = h1[s][:, s].cpu().numpy()
    E0v = float(E0.cpu()[0])
    del V2, h1, E0
    torch.cuda.empty_cache()
    ref = fb.closed_shell(p.xyz, p.w, p.phi[sub], np.arange(19), p.jastrow)
    _check(V2s, h1s, E0v, ref, prec)


def _single_orbital():
    p = inputs.make_problem(4, 1, 500, 1, "chain", "pade", seed=62)
    return inputs.Problem(p.xyz, p.w, p.chi[:1], p.phi[:1], np.array([0], dtype=np.int32), p.centres, p.jastrow)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_single_orbital(torch_cuda, prec):
    """N = n = 1: one pair; E0 vanishes (a single occupied orbital has no
    three-body energy)."""
    from oracle import factorised as fb
    from paper_2304_07006_amd import xtc
    p = _single_orbital()
    _note(f"case: N=1 n=1 Ng=500 {prec}")
    V2, h1, E0 = xtc.forward(p, prec=prec, chunk_rows=160)
    ref = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    _check(V2.cpu().numpy(), h1.cpu().numpy(), float(E0.cpu()[0]), ref, prec)
    assert abs(float(E0.cpu()[0])) < 1e-15


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_every_orbital_occupied(torch_cuda, prec):
    """n = N = 4: no virtual orbital; the occupied block is the whole pair set."""
    from oracle import factorised as fb
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(4, 4, 500, 1, "chain", "power16", seed=63)
    _note(f"case: N=4 n=4 Ng=500 power16 {prec}")
    V2, h1, E0 = xtc.forward(p, prec=prec, chunk_rows=192)
    ref = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    _check(V2.cpu().numpy(), h1.cpu().numpy(), float(E0.cpu()[0]), ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_grid_smaller_than_one_tile(torch_cuda, prec):
    """Ng=40 (one padded 128-point block, ragged 32-row chunks: 32 + 8)."""
    from oracle import factorised as fb
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(8, 2, 40, 2, "pair", "pade", seed=64)
    _note(f"case: N=8 n=2 Ng=40 chunk=32 {prec}")
    V2, h1, E0 = xtc.forward(p, prec=prec, chunk_rows=32)
    ref = fb.closed_shell(p.xyz, p.w, p.phi, p.occ, p.jastrow)
    _check(V2.cpu().numpy(), h1.cpu().numpy(), float(E0.cpu()[0]), ref,
           "fp64" if prec == "fp64" else prec)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_single_grid_point(torch_cuda, prec):
    """Ng=1: the only pair of points is the point with itself, where the
    Jastrow gradient is 0, so K = 0 and every output vanishes exactly."""
    from paper_2304_07006_amd import xtc
    p = inputs.make_problem(8, 2, 40, 2, "pair", "pade", seed=65)
    q = inputs.Problem(p.xyz[:1], p.w[:1], p.chi[:, :1], p.phi[:, :1], p.occ, p.centres, p.jastrow)
    _note(f"case: N=8 n=2 Ng=1 {prec}")
    V2, h1, E0 = xtc.forward(q, prec=prec)
    assert not V2.any() and not h1.any() and float(E0.cpu()[0]) == 0.0
