"""Pins for the seeded input generator (CPU only)."""
import math

import numpy as np
import pytest

from paper_2304_07006_amd import inputs


def _rows(problem):
    """(kind, centre, alpha, axis) for every raw function, in chi's row order."""
    out = []
    shells = problem.meta["shells"]
    for kind, c, a in shells:
        if kind == "s":
            out.append(("s", c, a, None))
        else:
            out.extend(("p", c, a, ax) for ax in range(3))
    # the generator emits, per centre, all s functions before the p shells
    by_centre = {}
    for r in out:
        by_centre.setdefault(r[1], []).append(r)
    ordered = []
    for c in sorted(by_centre):
        ordered += [r for r in by_centre[c] if r[0] == "s"] + [r for r in by_centre[c] if r[0] == "p"]
    return ordered


def _analytic_overlap(fa, fb, centres):
    """Gaussian product theorem for normalised s / p Cartesian Gaussians."""
    ka, ca, a, xa = fa
    kb, cb, b, xb = fb
    A, B = centres[ca], centres[cb]
    c = a + b
    P = (a * A + b * B) / c
    K = math.exp(-a * b / c * float(np.sum((A - B) ** 2))) * (math.pi / c) ** 1.5
    na = (2 * a / math.pi) ** 0.75 if ka == "s" else (128 * a ** 5 / math.pi ** 3) ** 0.25
    nb = (2 * b / math.pi) ** 0.75 if kb == "s" else (128 * b ** 5 / math.pi ** 3) ** 0.25
    if ka == "s" and kb == "s":
        poly = 1.0
    elif ka == "s":
        poly = P[xb] - B[xb]
    elif kb == "s":
        poly = P[xa] - A[xa]
    elif xa == xb:
        poly = (P[xa] - A[xa]) * (P[xa] - B[xa]) + 0.5 / c
    else:
        poly = (P[xa] - A[xa]) * (P[xb] - B[xb])
    return na * nb * K * poly


def test_weights_are_inverse_density():
    p = inputs.make_workload("N8-occ2-Ng2k")
    pdf = inputs.mixture_pdf(p.xyz, p.centres)
    # w_g p(r_g) = 1/Ng for every point, hence sum_g w_g p(r_g) = 1
    assert np.allclose(p.w * pdf * p.Ng, 1.0, rtol=1e-13, atol=0)
    assert abs(np.sum(p.w * pdf) - 1.0) < 1e-12


@pytest.mark.parametrize("name,Ng", [("N8-occ2-Ng2k", None), ("N64-occ8-Ng50k", 20000)])
def test_grid_quadrature_of_gaussian_overlaps(name, Ng):
    p = inputs.make_workload(name, Ng=Ng)
    rows = _rows(p)
    assert len(rows) == p.N
    rng = np.random.default_rng(5)
    pairs = [(i, j) for i in range(p.N) for j in range(i, p.N)]
    pick = [pairs[k] for k in rng.choice(len(pairs), size=min(60, len(pairs)), replace=False)]
    worst = 0.0
    for i, j in pick:
        f = p.chi[i] * p.chi[j] * p.w
        est = f.sum()
        sig = math.sqrt(np.sum((f - est / p.Ng) ** 2))
        exact = _analytic_overlap(rows[i], rows[j], p.centres)
        z = abs(est - exact) / max(sig, 1e-300)
        worst = max(worst, z)
    assert worst < 5.0, worst


def test_orbitals_orthonormal_under_weights():
    for name, Ng in [("N8-occ2-Ng2k", None), ("N64-occ8-Ng50k", 8000)]:
        p = inputs.make_workload(name, Ng=Ng)
        S = (p.phi * p.w) @ p.phi.T
        S0 = (p.chi * p.w) @ p.chi.T
        cond = np.linalg.cond(S0)
        assert np.abs(S - np.eye(p.N)).max() < 1e-15 * max(cond, 10.0) * 10


def test_seeds_reproduce_bitwise():
    a = inputs.make_workload("N8-occ2-Ng2k")
    b = inputs.make_workload("N8-occ2-Ng2k")
    for k in ("xyz", "w", "chi", "phi", "occ"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = inputs.make_problem(8, 2, 2000, 2, "pair", "pade", seed=7)
    assert not np.array_equal(a.xyz, c.xyz)


def test_workload_shapes():
    wl = inputs.WORKLOADS
    assert [w.N for w in wl.values()] == [8, 64, 128, 96, 160]
    assert [w.nocc for w in wl.values()] == [2, 8, 16, 12, 20]
    assert [w.Ng for w in wl.values()] == [2000, 50000, 150000, 100000, 250000]
    for w in wl.values():
        assert (w.N // w.n_centres) % 4 == 0
    p = inputs.make_workload("N96-occ12-Ng100k", Ng=500)
    assert p.jastrow.kind == "power" and p.jastrow.ncoef == 16 and p.jastrow.coef[0] == 0.5
    assert abs(np.std(p.jastrow.coef[1:]) - 0.05) < 0.03


def test_chain_spacing():
    rng = np.random.default_rng(3)
    R = inputs.chain_centres(6, rng)
    assert np.allclose(np.linalg.norm(np.diff(R, axis=0), axis=1), 2.0)
    assert np.allclose(R.mean(axis=0), 0.0, atol=1e-14)


def test_loss_weights_symmetry():
    D, G = inputs.loss_weights(5, 11)
    assert np.array_equal(D, D.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.allclose(G, G.transpose(perm), atol=1e-15)


def test_occupation_generators():
    k, n = inputs.sa_occupations(3, 2)
    assert list(k) == [0, 1, 2, 3, 4] and list(n) == [1.0, 1.0, 1.0, 0.5, 0.5]
    m = inputs.natural_occupations(9, 5)
    assert m.shape == (9,) and np.all(m > 0) and np.all(m < 1) and np.all(np.diff(m) <= 0)
    assert np.array_equal(m, inputs.natural_occupations(9, 5))


def test_orbital_gradients_match_finite_differences():
    p = inputs.make_problem(8, 2, 40, 2, "pair", "pade", seed=3)
    dchi = inputs.basis_gradients(p.xyz, p.centres, p.meta["shells"])
    h = 1e-5
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        fd = (inputs.eval_shells(p.xyz + e, p.centres, p.meta["shells"])
              - inputs.eval_shells(p.xyz - e, p.centres, p.meta["shells"])) / (2 * h)
        assert np.abs(fd - dchi[ax]).max() < 1e-8
    dphi = inputs.orbital_gradients(p)
    X = inputs.lowdin_matrix(p.chi, p.w)
    assert np.abs(X @ p.chi - p.phi).max() < 1e-13
    assert np.abs(dphi - np.einsum("ij,xjg->xig", X, dchi)).max() == 0.0
