"""Seeded synthetic inputs for the xTC three-body folding.

This module only *draws* inputs: atom centres, a Monte-Carlo quadrature grid
with importance weights, orthonormal s/p Gaussian orbitals tabulated on that
grid, the occupied set, Jastrow parameters and the fixed weights of the
differentiation loss.  It holds none of the xTC arithmetic (no Jastrow
gradient, no grid intermediate, no contraction); both the HIP path and the
CPU oracle receive exactly the arrays produced here.

The paper evaluates the method on the HEAT molecules with Dunning basis sets
on Treutler-Ahlrichs/Lebedev grids and optimised Drummond-Towler-Needs
Jastrows (Results section, computational details).  None of those are
available here; the workloads below stand in for them with small-molecule
shaped synthetic problems:

* grid points drawn i.i.d. from an equal-weight mixture of isotropic Gaussians
  (sigma = 1.5 bohr) around the atom centres, weights w_g = 1/(Ng p(r_g)), so
  that sum_g w_g f(r_g) is an unbiased estimate of the integral of f;
* per centre m = N/n_centres functions: m/4 normalised s Gaussians and m/4 p
  shells (x, y, z), exponents log-uniform in [0.2, 5];
* the orbitals are the symmetric (Loewdin) orthonormalisation of those
  functions under the grid weights, in FP64, so that sum_g w_g phi_p phi_q is
  the identity to rounding;
* electron-electron Jastrow: Pade u = r/(2(1+b r)) with b = 1, or the
  16-term power series u = sum_k c_k (r/(1+r))^k with c_1 = 1/2 (the cusp)
  and c_2..c_16 ~ N(0, 0.05^2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SIGMA_BOHR = 1.5
ALPHA_RANGE = (0.2, 5.0)


@dataclass(frozen=True)
class Jastrow:
    """Electron-electron Jastrow u(r12) parameters (passed to both sides).

    kind "pade":  u = r / (2 (1 + b r))
    kind "power": u = sum_{k=1..ncoef} coef[k-1] * (r/(1+r))^k
    """
    kind: str
    b: float = 1.0
    coef: tuple = ()

    @property
    def ncoef(self) -> int:
        return len(self.coef)


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    nocc: int
    Ng: int
    n_centres: int
    layout: str          # "pair": two centres at (0,0,+-0.7); "chain": 2-bohr random chain
    jastrow_kind: str    # "pade" or "power16"
    seed: int            # generator seed
    aux_seed: int        # seed for Jastrow coefficients and loss weights


# The five synthetic workloads: a tiny one the explicit six-index oracle handles,
# a mid-size FP64 one, the N=128 precision workload, the N=96 differentiation
# workload and the N=160 forward+backward workload.
WORKLOADS = {
    "N8-occ2-Ng2k": Workload("N8-occ2-Ng2k", 8, 2, 2000, 2, "pair", "pade", 1000, 2000),
    "N64-occ8-Ng50k": Workload("N64-occ8-Ng50k", 64, 8, 50000, 4, "chain", "pade", 1001, 2001),
    "N128-occ16-Ng150k": Workload("N128-occ16-Ng150k", 128, 16, 150000, 8, "chain", "pade", 1002, 2002),
    "N96-occ12-Ng100k": Workload("N96-occ12-Ng100k", 96, 12, 100000, 6, "chain", "power16", 1003, 2003),
    "N160-occ20-Ng250k": Workload("N160-occ20-Ng250k", 160, 20, 250000, 10, "chain", "power16", 1004, 2004),
}


@dataclass
class Problem:
    """Host (numpy, FP64) arrays of one problem instance."""
    xyz: np.ndarray      # [Ng][3]
    w: np.ndarray        # [Ng]
    chi: np.ndarray      # [N][Ng] raw normalised primitives
    phi: np.ndarray      # [N][Ng] orthonormal orbitals under w
    occ: np.ndarray      # [nocc] int32
    centres: np.ndarray  # [n_centres][3]
    jastrow: Jastrow
    meta: dict = field(default_factory=dict)
    occ_n: np.ndarray | None = None       # per-spin occupations of occ (None: 1 each)
    occ_n_beta: np.ndarray | None = None  # open shell: beta occupations (occ_n is then alpha)

    @property
    def N(self) -> int:
        return self.phi.shape[0]

    @property
    def Ng(self) -> int:
        return self.phi.shape[1]

    @property
    def nocc(self) -> int:
        return len(self.occ)


def chain_centres(n_centres: int, rng: np.random.Generator, spacing: float = 2.0) -> np.ndarray:
    """R_0 = 0, R_{c+1} = R_c + spacing * u_c with u_c uniform on the sphere, recentred."""
    R = np.zeros((n_centres, 3))
    for c in range(1, n_centres):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        R[c] = R[c - 1] + spacing * v
    return R - R.mean(axis=0)


def pair_centres() -> np.ndarray:
    return np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])


def mixture_pdf(xyz: np.ndarray, centres: np.ndarray, sigma: float = SIGMA_BOHR) -> np.ndarray:
    norm = (2.0 * math.pi * sigma * sigma) ** -1.5
    acc = np.zeros(xyz.shape[0])
    for R in centres:
        d2 = np.sum((xyz - R) ** 2, axis=1)
        acc += norm * np.exp(-d2 / (2.0 * sigma * sigma))
    return acc / len(centres)


def sample_grid(centres: np.ndarray, Ng: int, rng: np.random.Generator,
                sigma: float = SIGMA_BOHR):
    """Points from the equal-weight Gaussian mixture; weights 1/(Ng p(r))."""
    which = rng.integers(0, len(centres), size=Ng)
    xyz = centres[which] + sigma * rng.standard_normal((Ng, 3))
    w = 1.0 / (Ng * mixture_pdf(xyz, centres, sigma))
    return np.ascontiguousarray(xyz), w


def basis_values(xyz: np.ndarray, centres: np.ndarray, per_centre: int,
                 rng: np.random.Generator):
    """Normalised s and p Gaussians on the grid, [N][Ng]; also returns the shell list."""
    if per_centre % 4 != 0:
        raise ValueError("functions per centre must be a multiple of 4 (m/4 s + m/4 p shells)")
    ns = per_centre // 4
    lo, hi = math.log(ALPHA_RANGE[0]), math.log(ALPHA_RANGE[1])
    shells = []
    for c in range(len(centres)):
        for _ in range(ns):
            shells.append(("s", c, math.exp(rng.uniform(lo, hi))))
        for _ in range(ns):
            shells.append(("p", c, math.exp(rng.uniform(lo, hi))))
    return eval_shells(xyz, centres, shells), shells


def eval_shells(xyz: np.ndarray, centres: np.ndarray, shells) -> np.ndarray:
    """Values of the shells' functions at xyz, [N][len(xyz)] (s: one function,
    p: x, y, z)."""
    rows = []
    for kind, c, a in shells:
        d = xyz - centres[c]
        r2 = np.sum(d * d, axis=1)
        if kind == "s":
            rows.append((2.0 * a / math.pi) ** 0.75 * np.exp(-a * r2))
        else:
            g = (128.0 * a ** 5 / math.pi ** 3) ** 0.25 * np.exp(-a * r2)
            for ax in range(3):
                rows.append(d[:, ax] * g)
    return np.ascontiguousarray(np.array(rows))


def lowdin_matrix(chi: np.ndarray, w: np.ndarray) -> np.ndarray:
    """X = S^{-1/2} with S = chi diag(w) chi^T (FP64, input preparation)."""
    S = (chi * w) @ chi.T
    S = 0.5 * (S + S.T)
    lam, U = np.linalg.eigh(S)
    if lam[0] <= 0:
        raise ValueError("grid overlap matrix is not positive definite")
    return (U * lam ** -0.5) @ U.T


def orthonormalise_inputs(chi: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Symmetric orthonormalisation of the raw functions under the grid weights.

    Input preparation only: phi = S^{-1/2} chi with S = chi diag(w) chi^T, in FP64.
    """
    return np.ascontiguousarray(lowdin_matrix(chi, w) @ chi)


def basis_gradients(xyz: np.ndarray, centres: np.ndarray, shells) -> np.ndarray:
    """Analytic gradients of the raw functions of basis_values, [3][N][Ng]
    (same order: per shell one s function or the x, y, z components of a p shell)."""
    out = []
    for kind, c, a in shells:
        d = xyz - centres[c]
        e = np.exp(-a * np.sum(d * d, axis=1))
        if kind == "s":
            g = (2.0 * a / math.pi) ** 0.75 * e
            out.append(-2.0 * a * d.T * g)                      # grad of N e^{-a r^2}
        else:
            g = (128.0 * a ** 5 / math.pi ** 3) ** 0.25 * e
            for ax in range(3):
                gr = -2.0 * a * d[:, ax] * d.T * g              # d_ax * grad(e) part
                gr[ax] += g                                     # grad(d_ax) e part
                out.append(gr)
    return np.ascontiguousarray(np.moveaxis(np.array(out), 1, 0))


def orbital_gradients(p: "Problem") -> np.ndarray:
    """grad phi on the grid, [3][N][Ng]: the Loewdin transform of the analytic
    basis gradients (phi = X chi, so grad phi = X grad chi)."""
    X = p.meta.get("lowdin")
    if X is None:
        X = lowdin_matrix(p.chi, p.w)
    dchi = basis_gradients(p.xyz, p.centres, p.meta["shells"])
    return np.ascontiguousarray(np.einsum("ij,xjg->xig", X, dchi))


def make_jastrow(kind: str, aux_seed: int) -> Jastrow:
    if kind == "pade":
        return Jastrow("pade", b=1.0)
    if kind == "power16":
        rng = np.random.default_rng(aux_seed)
        c = np.empty(16)
        c[0] = 0.5
        c[1:] = 0.05 * rng.standard_normal(15)
        return Jastrow("power", coef=tuple(float(x) for x in c))
    raise ValueError(kind)


def make_problem(N: int, nocc: int, Ng: int, n_centres: int, layout: str = "chain",
                 jastrow_kind: str = "pade", seed: int = 0, aux_seed: int | None = None,
                 occ: np.ndarray | None = None, lowdin: np.ndarray | None = None) -> Problem:
    """One seeded problem.  ``lowdin``: a stored orthonormalisation matrix X
    (phi = X chi) to use instead of computing S^{-1/2} here.  S^{-1/2} is
    ill-conditioned (cond(S) reaches 2e8 at N=128), so eigen-solvers on
    different hosts give orbitals that differ by about cond(S) x 1e-16; a
    stored X reproduces stored oracle values to about 1e-12 on any host."""
    if N % n_centres != 0:
        raise ValueError("N must be a multiple of the number of centres")
    if not (1 <= nocc <= N):
        raise ValueError("nocc must lie in [1, N]")
    rng = np.random.default_rng(seed)
    centres = pair_centres() if layout == "pair" else chain_centres(n_centres, rng)
    if len(centres) != n_centres:
        raise ValueError("layout 'pair' has exactly two centres")
    xyz, w = sample_grid(centres, Ng, rng)
    chi, shells = basis_values(xyz, centres, N // n_centres, rng)
    if lowdin is None:
        phi = orthonormalise_inputs(chi, w)
    else:
        if np.shape(lowdin) != (N, N):
            raise ValueError(f"lowdin matrix must be [{N}][{N}]")
        phi = np.ascontiguousarray(np.asarray(lowdin, dtype=np.float64) @ chi)
    if occ is None:
        occ = np.arange(nocc, dtype=np.int32)
    occ = np.asarray(occ, dtype=np.int32)
    jas = make_jastrow(jastrow_kind, 2000 + seed if aux_seed is None else aux_seed)
    return Problem(xyz=xyz, w=w, chi=chi, phi=phi, occ=occ, centres=centres, jastrow=jas,
                   meta=dict(seed=seed, shells=shells, layout=layout, lowdin=lowdin))


def make_workload(name: str, Ng: int | None = None, lowdin: np.ndarray | None = None) -> Problem:
    """One of WORKLOADS, optionally on a smaller grid (same generator, same
    seed) or with a stored orthonormalisation matrix (see make_problem)."""
    wl = WORKLOADS[name]
    p = make_problem(wl.N, wl.nocc, wl.Ng if Ng is None else Ng, wl.n_centres, wl.layout,
                     wl.jastrow_kind, wl.seed, wl.aux_seed, lowdin=lowdin)
    p.meta["workload"] = name
    return p


def input_fingerprint(p: Problem) -> np.ndarray:
    """Checksums of the drawn inputs (positions, weights, raw functions), to
    check that a host regenerates the inputs a stored result was computed
    from.  Compared to a relative tolerance: the exponentials may differ in
    the last bit between hosts, which moves these sums by about 1e-16."""
    u = np.random.default_rng(12345).standard_normal(p.Ng)
    return np.concatenate([p.xyz.sum(axis=0), [p.w.sum(), (p.w * np.sum(p.xyz ** 2, axis=1)).sum()],
                           p.chi.sum(axis=1), (p.chi * p.chi * p.w).sum(axis=1), p.chi @ u])


def random_occ(N: int, nocc: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=nocc, replace=False)).astype(np.int32)


def sa_occupations(n_double: int, n_single: int) -> tuple[np.ndarray, np.ndarray]:
    """Spin-averaged density of a high-spin open-shell determinant in its
    orbital basis: n_double doubly occupied orbitals (1 per spin) followed by
    n_single singly occupied ones (1/2 per spin).  Returns (orbitals, n)."""
    k = np.arange(n_double + n_single, dtype=np.int32)
    n = np.concatenate([np.ones(n_double), np.full(n_single, 0.5)])
    return k, n


def open_shell_occupations(n_double: int, n_single: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """High-spin open-shell determinant in its orbital basis: n_double doubly
    occupied orbitals then n_single alpha-only ones.  Returns (orbitals,
    alpha occupations, beta occupations)."""
    k = np.arange(n_double + n_single, dtype=np.int32)
    na = np.ones(n_double + n_single)
    nb = np.concatenate([np.ones(n_double), np.zeros(n_single)])
    return k, na, nb


def natural_occupations(nact: int, seed: int) -> np.ndarray:
    """Per-spin natural occupation numbers of a weakly correlated closed-shell
    density: nact orbitals, the first half near 1 (1 - 10^U(-3,-1)), the
    rest small (10^U(-4,-1.5)), in decreasing order."""
    rng = np.random.default_rng(seed)
    h = (nact + 1) // 2
    hi = 1.0 - 10.0 ** rng.uniform(-3.0, -1.0, h)
    lo = 10.0 ** rng.uniform(-4.0, -1.5, nact - h)
    return np.concatenate([np.sort(hi)[::-1], np.sort(lo)[::-1]])


def loss_weights(N: int, aux_seed: int):
    """Fixed symmetric one-body weights D [N][N] and 8-fold symmetric two-body
    weights G [N][N][N][N] (chemist order) for the differentiation loss
    E0 + <h1, D> + <V2, G>."""
    rng = np.random.default_rng(aux_seed + 7)
    X = rng.standard_normal((N, N))
    D = 0.5 * (X + X.T)
    Y = rng.standard_normal((N, N, N, N))
    G = (Y + Y.transpose(1, 0, 2, 3) + Y.transpose(0, 1, 3, 2) + Y.transpose(1, 0, 3, 2)
         + Y.transpose(2, 3, 0, 1) + Y.transpose(3, 2, 0, 1) + Y.transpose(2, 3, 1, 0)
         + Y.transpose(3, 2, 1, 0)) / 8.0
    return np.ascontiguousarray(D), np.ascontiguousarray(G)
