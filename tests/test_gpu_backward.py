"""GPU adjoint (xtc_backward) against the oracle's exact gradient and finite differences."""
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


def _case(N, nocc, Ng, nc, seed, occ=None, ncoef=16):
    p = inputs.make_problem(N, nocc, Ng, nc, "chain", "power16", seed=seed, occ=occ)
    coef = np.array(p.jastrow.coef[:ncoef])
    D, G = inputs.loss_weights(N, seed)
    return p, coef, D, G


def _gpu_grad(torch, p, coef, D, G, prec="fp64", chunk_rows=None):
    from paper_2304_07006_amd import xtc
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    g = xtc.backward(dp, list(coef), torch.as_tensor(G).cuda(), torch.as_tensor(D).cuda(), 1.0, prec, chunk_rows)
    return g.cpu().numpy()


def _gpu_loss(torch, p, coef, D, G, prec="fp64"):
    from paper_2304_07006_amd import xtc
    jas = inputs.Jastrow("power", coef=tuple(float(c) for c in coef))
    V2, h1, E0 = xtc.forward(p, prec=prec, jastrow=jas)
    return float(E0.cpu()[0]) + float((h1.cpu().numpy() * D).sum()) + float((V2.cpu().numpy() * G).sum())


@pytest.mark.parametrize("N,nocc,Ng,nc,seed,chunk", [(8, 2, 600, 2, 31, None), (12, 3, 900, 3, 32, 256)])
def test_gradient_matches_oracle(torch_cuda, N, nocc, Ng, nc, seed, chunk):
    from oracle import gradient as og
    p, coef, D, G = _case(N, nocc, Ng, nc, seed)
    _note(f"case: backward N={N} n={nocc} Ng={Ng} chunk={chunk}")
    go = og.exact_gradient(p.xyz, p.w, p.phi, p.occ, coef, D, G)
    gg = _gpu_grad(torch_cuda, p, coef, D, G, chunk_rows=chunk)
    scale = np.abs(go).max()
    _note(f"  max |dg| {np.abs(gg - go).max():.3e}  scale {scale:.3e}")
    assert np.abs(gg - go).max() < 1e-10 * max(1.0, scale)


def test_gradient_euler_and_fd(torch_cuda):
    """c . grad L = 2 L (homogeneous quadratic) and central FD on the GPU forward."""
    occ = inputs.random_occ(24, 5, seed=7)
    p, coef, D, G = _case(24, 5, 1500, 6, 33, occ=occ)
    _note("case: backward N=24 n=5 random occ, Euler + FD")
    g = _gpu_grad(torch_cuda, p, coef, D, G, chunk_rows=640)
    L = _gpu_loss(torch_cuda, p, coef, D, G)
    assert abs(np.dot(coef, g) - 2 * L) < 1e-9 * max(1.0, abs(L))
    h = 1e-5
    for k in (0, 1, 7):
        e = np.zeros_like(coef)
        e[k] = h
        fd = (_gpu_loss(torch_cuda, p, coef + e, D, G) - _gpu_loss(torch_cuda, p, coef - e, D, G)) / (2 * h)
        assert abs(fd - g[k]) < 1e-8 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_gradient_with_more_occupied_than_one_register_group(torch_cuda):
    """nocc = 32: the adjoint's local kernel takes the occupied columns in two
    groups (24 + 8): Euler identity and GPU central differences (N=40,
    ragged chunks)."""
    occ = inputs.random_occ(40, 32, seed=9)
    p, coef, D, G = _case(40, 32, 900, 5, 37, occ=occ)
    _note("case: backward N=40 n=32 chunk=320")
    g = _gpu_grad(torch_cuda, p, coef, D, G, chunk_rows=320)
    L = _gpu_loss(torch_cuda, p, coef, D, G)
    assert abs(np.dot(coef, g) - 2 * L) < 1e-9 * max(1.0, abs(L))
    h = 1e-5
    for k in (0, 3):
        e = np.zeros_like(coef)
        e[k] = h
        fd = (_gpu_loss(torch_cuda, p, coef + e, D, G) - _gpu_loss(torch_cuda, p, coef - e, D, G)) / (2 * h)
        assert abs(fd - g[k]) < 1e-8 * max(1.0, abs(g[k])), (k, fd, g[k])


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_gradient_matches_oracle_with_32_occupied(torch_cuda, prec):
    """nocc = 32 against the oracle's exact gradient (4 coefficients, N=40): FP64
    1e-10 relative, split BF16 x3 1e-5 of max|g|."""
    from oracle import gradient as og
    occ = inputs.random_occ(40, 32, seed=10)
    p, coef, D, G = _case(40, 32, 500, 5, 38, occ=occ, ncoef=4)
    _note(f"case: backward N=40 n=32 Ng=500 chunk=256 {prec} vs oracle")
    go = og.exact_gradient(p.xyz, p.w, p.phi, p.occ, coef, D, G)
    gg = _gpu_grad(torch_cuda, p, coef, D, G, prec=prec, chunk_rows=256)
    scale = np.abs(go).max()
    _note(f"  max |dg| {np.abs(gg - go).max():.3e}  scale {scale:.3e}")
    assert np.abs(gg - go).max() < (1e-10 * max(1.0, scale) if prec == "fp64" else 1e-5 * scale)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6", "fp32"])
@pytest.mark.parametrize("N,nocc,Ng,nc,seed,chunk", [(12, 3, 900, 3, 34, None), (24, 5, 1500, 6, 36, 640)])
def test_gradient_reduced_precision_close(torch_cuda, prec, N, nocc, Ng, nc, seed, chunk):
    """The reduced forms (K recompute and Pi contraction) change the gradient
    only at the level of their FP32 accumulation; the second case spans
    several pair k-steps, three g' tiles and a ragged last chunk."""
    p, coef, D, G = _case(N, nocc, Ng, nc, seed)
    _note(f"case: backward {prec} vs fp64 N={N} Ng={Ng} chunk={chunk}")
    g64 = _gpu_grad(torch_cuda, p, coef, D, G, chunk_rows=chunk)
    gr = _gpu_grad(torch_cuda, p, coef, D, G, prec=prec, chunk_rows=chunk)
    _note(f"  max |dg| {np.abs(gr - g64).max():.3e}  scale {np.abs(g64).max():.3e}")
    assert np.abs(gr - g64).max() < 1e-5 * max(1.0, np.abs(g64).max())


def test_autograd_function(torch_cuda):
    import torch
    from paper_2304_07006_amd import xtc
    p, coef, D, G = _case(8, 2, 500, 2, 35)
    _note("case: autograd.Function")
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ)
    c = torch.tensor(coef, dtype=torch.float64, device="cuda", requires_grad=True)
    V2, h1, E0 = xtc.XtcFunction.apply(c, dp)
    loss = E0.sum() + (h1 * torch.as_tensor(D).cuda()).sum() + (V2 * torch.as_tensor(G).cuda()).sum()
    loss.backward()
    g = _gpu_grad(torch, p, coef, D, G)
    assert np.abs(c.grad.cpu().numpy() - g).max() < 1e-12 * max(1.0, np.abs(g).max())


# ------------------------------------------------------------- open shell --
def _open_case(N, nd, ns, Ng, nc, seed):
    k, na, nb = inputs.open_shell_occupations(nd, ns)
    p = inputs.make_problem(N, nd + ns, Ng, nc, "chain", "power16", seed=seed, occ=k)
    p.occ_n, p.occ_n_beta = na, nb
    ga = np.zeros((N, N)); ga[k, k] = na
    gb = np.zeros((N, N)); gb[k, k] = nb
    coef = np.array(p.jastrow.coef[:16])
    D1, G1 = inputs.loss_weights(N, seed)
    D2, G2 = inputs.loss_weights(N, seed + 1)
    _, G3 = inputs.loss_weights(N, seed + 2)
    return p, ga, gb, coef, (D1, D2), (G1, G2, G3)


def _gpu_grad_open(torch, p, coef, D, G, prec="fp64", chunk_rows=None):
    from paper_2304_07006_amd import xtc
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ, occ_n=p.occ_n, occ_n_beta=p.occ_n_beta)
    gV2 = torch.as_tensor(np.stack(G)).cuda()
    gh1 = torch.as_tensor(np.stack(D)).cuda()
    return xtc.backward(dp, list(coef), gV2, gh1, 1.0, prec, chunk_rows).cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_open_shell_gradient_matches_oracle(torch_cuda, prec):
    """Restricted open shell (2 doubly, 2 singly occupied): the adjoint of the
    spin-blocked loss against the oracle's exact gradient of Appendix A's
    outputs (FP64 1e-10 relative; the reduced forms 1e-5 of max|g|, as in the
    closed shell), ragged chunks."""
    from oracle import gradient as og
    p, ga, gb, coef, D, G = _open_case(12, 2, 2, 900, 3, 41)
    _note(f"case: open-shell backward N=12 2+2 Ng=900 chunk=256 {prec}")
    go = og.exact_gradient_open(p.xyz, p.w, p.phi, ga, gb, coef, D, G)
    gg = _gpu_grad_open(torch_cuda, p, coef, D, G, prec, chunk_rows=256)
    scale = np.abs(go).max()
    err = np.abs(gg - go).max()
    _note(f"  max |dg| {err:.3e}  scale {scale:.3e}")
    assert err < (1e-10 * max(1.0, scale) if prec == "fp64" else 1e-5 * scale)


def test_open_shell_gradient_equal_spins_and_spin_exchange(torch_cuda):
    """Equal spin densities with the seeds split evenly over the spin blocks
    give the closed-shell adjoint; exchanging the spins (densities, one-body
    seeds, aa <-> bb and the ab block's pair indices) leaves the gradient
    unchanged.  FP64."""
    from paper_2304_07006_amd import xtc
    p, coef, D, G = _case(12, 3, 700, 3, 43)
    _note("case: open-shell backward N=12, equal spins vs closed shell; spin exchange")
    gc = _gpu_grad(torch_cuda, p, coef, D, G, chunk_rows=256)
    q = inputs.Problem(p.xyz, p.w, p.chi, p.phi, p.occ, p.centres, p.jastrow)
    q.occ_n = np.ones(len(p.occ)); q.occ_n_beta = np.ones(len(p.occ))
    ge = _gpu_grad_open(torch_cuda, q, coef, (D / 2, D / 2), (G / 3, G / 3, G / 3), chunk_rows=256)
    _note(f"  |g_open(equal) - g_closed| {np.abs(ge - gc).max():.3e} of {np.abs(gc).max():.3e}")
    assert np.abs(ge - gc).max() < 1e-11 * max(1.0, np.abs(gc).max())
    r, ga, gb, coef, Do, Go = _open_case(12, 1, 2, 700, 3, 44)
    g1 = _gpu_grad_open(torch_cuda, r, coef, Do, Go, chunk_rows=256)
    s = inputs.Problem(r.xyz, r.w, r.chi, r.phi, r.occ, r.centres, r.jastrow)
    s.occ_n, s.occ_n_beta = r.occ_n_beta, r.occ_n
    g2 = _gpu_grad_open(torch_cuda, s, coef, (Do[1], Do[0]),
                        (Go[2], np.ascontiguousarray(Go[1].transpose(2, 3, 0, 1)), Go[0]), chunk_rows=256)
    _note(f"  |g - g(spins exchanged)| {np.abs(g1 - g2).max():.3e} of {np.abs(g1).max():.3e}")
    assert np.abs(g1 - g2).max() < 1e-11 * max(1.0, np.abs(g1).max())


def test_open_shell_autograd_function(torch_cuda):
    """XtcFunction on an open-shell problem: the spin-blocked outputs' gradients
    flow back as the spin-blocked seeds of xtc_backward."""
    import torch
    from paper_2304_07006_amd import xtc
    p, ga, gb, coef, D, G = _open_case(8, 1, 1, 500, 2, 45)
    _note("case: autograd.Function, open shell")
    dp = xtc.device_problem(p.xyz, p.w, p.phi, p.occ, occ_n=p.occ_n, occ_n_beta=p.occ_n_beta)
    c = torch.tensor(coef, dtype=torch.float64, device="cuda", requires_grad=True)
    V2, h1, E0 = xtc.XtcFunction.apply(c, dp)
    assert tuple(V2.shape) == (3, 8, 8, 8, 8) and tuple(h1.shape) == (2, 8, 8)
    loss = (E0.sum() + (h1 * torch.as_tensor(np.stack(D)).cuda()).sum()
            + (V2 * torch.as_tensor(np.stack(G)).cuda()).sum())
    loss.backward()
    g = _gpu_grad_open(torch, p, coef, D, G)
    assert np.abs(c.grad.cpu().numpy() - g).max() < 1e-12 * max(1.0, np.abs(g).max())
