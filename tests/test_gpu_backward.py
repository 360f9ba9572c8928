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


def test_gradient_at_the_largest_occupied_set(torch_cuda):
    """nocc = 24, the most the adjoint's local kernels hold in registers:
    Euler identity and GPU central differences (N=32, ragged chunks)."""
    occ = inputs.random_occ(32, 24, seed=9)
    p, coef, D, G = _case(32, 24, 900, 4, 37, occ=occ)
    _note("case: backward N=32 n=24 (largest supported) chunk=320")
    g = _gpu_grad(torch_cuda, p, coef, D, G, chunk_rows=320)
    L = _gpu_loss(torch_cuda, p, coef, D, G)
    assert abs(np.dot(coef, g) - 2 * L) < 1e-9 * max(1.0, abs(L))
    h = 1e-5
    for k in (0, 3):
        e = np.zeros_like(coef)
        e[k] = h
        fd = (_gpu_loss(torch_cuda, p, coef + e, D, G) - _gpu_loss(torch_cuda, p, coef - e, D, G)) / (2 * h)
        assert abs(fd - g[k]) < 1e-8 * max(1.0, abs(g[k])), (k, fd, g[k])


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
