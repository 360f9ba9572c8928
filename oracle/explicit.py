"""Tier A oracle: the explicit six-index three-body integrals and their
normal ordering (small inputs only).

Steps, in the paper's order and notation:

1. grid intermediate V_R^S(i) = sum_j w_j phi_R(j) grad_1 u(r_i, r_j) phi_S(j)
   (Theory, "Decomposition of two-body correction", definition under eq. Ldecomp);
2. L_{prt}^{qsu} on the grid (eq. Ldecomp).  The permutation operator in that
   equation is read as the three-term sum over which electron pair sits on the
   centre point i, which is what the symmetric operator P^1_{2,3} in the
   definition of L produces;
3. cross-check of (2) against the literal triple grid sum of the definition of L
   (Theory, "Transcorrelation") on micro grids;
4. spin-orbital L (spin-free Jastrow: L is diagonal in the spin of each pair);
5. Delta U by eq. dU, Delta h by eq. tcmf:1el (both forms) and by the general
   expression with the two-body density of a determinant, the zero-body term
   <Phi0|L|Phi0> = -(1/6) L gamma^3 and = -(1/3) Delta h gamma (eq. tcmf:0el);
6. brute-force check in determinant space: the three-body operator
   T3 = -(1/6) L a^{PRT}_{QSU} minus the folded operator
   E0 + Delta h a^P_Q + (1/2) Delta U a^{PR}_{QS} equals the normal-ordered L_N,
   so its matrix elements between Phi0 and any determinant up to doubles vanish
   (Theory, "Generalized normal ordering" and "The xTC approximation").

Index conventions: spin-orbital arrays store lower indices first, then upper:
L_so[P,R,T,Q,S,U] = L_{PRT}^{QSU}, dU_so[P,R,Q,S] = Delta U_{PR}^{QS}.
Spin orbital P = sigma*N + p.  The closed-shell outputs are returned as
V2[p,q,r,s] = Delta U_{pr}^{qs} (chemist order (pq|rs)), h1[p,q] = Delta h_p^q.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .jastrow import grad1


# ---------------------------------------------------------------- step 1 --
def grid_intermediate(xyz, w, phi, jas):
    """V[x][i][r][s] = sum_j w_j grad_1 u(r_i, r_j)_x phi_r(j) phi_s(j)."""
    d = grad1(xyz, xyz, jas)                       # [3][i][j]
    pw = phi * w                                   # [N][j]
    return np.einsum("xij,rj,sj->xirs", d, pw, phi, optimize=True)


# ---------------------------------------------------------------- step 2 --
def L_spatial(xyz, w, phi, jas, V=None):
    """L_sp[p,q,r,s,t,u] = L_{prt}^{qsu}: pairs (p,q), (r,s), (t,u) belong to
    electrons 1, 2, 3.  Three-term grid decomposition (eq. Ldecomp)."""
    if V is None:
        V = grid_intermediate(xyz, w, phi, jas)
    rho = np.einsum("i,pi,qi->ipq", w, phi, phi)
    N = phi.shape[0]
    VV = np.einsum("xirs,xitu->irstu", V, V, optimize=True)       # V_rs . V_tu
    # centre on electron 1, 2 and 3 respectively
    L1 = np.einsum("ipq,irstu->pqrstu", rho, VV, optimize=True)
    L2 = np.einsum("irs,ipqtu->pqrstu", rho, VV, optimize=True)
    L3 = np.einsum("itu,ipqrs->pqrstu", rho, VV, optimize=True)
    L = L1 + L2 + L3
    assert L.shape == (N,) * 6
    return L


# ---------------------------------------------------------------- step 3 --
def L_triple_sum(xyz, w, phi, jas):
    """Literal definition: L = <prt| P^1_{2,3} grad_1 u_12 . grad_1 u_13 |qsu>
    with every integral replaced by the grid quadrature (micro inputs only)."""
    g = grad1(xyz, xyz, jas)                       # g[x][a][b] = grad_a u(r_a, r_b)
    # f(1,2,3) = g(i,j).g(i,k); f(2,1,3) = g(j,i).g(j,k); f(3,2,1) = g(k,j).g(k,i)
    F = (np.einsum("xij,xik->ijk", g, g)
         + np.einsum("xji,xjk->ijk", g, g)
         + np.einsum("xkj,xki->ijk", g, g))
    pw = phi * w
    return np.einsum("ijk,pi,qi,rj,sj,tk,uk->pqrstu", F, pw, phi, pw, phi, pw, phi,
                     optimize=True)


# ---------------------------------------------------------------- step 4 --
def spin_orbital_L(L_sp):
    """L_so[P,R,T,Q,S,U] = L_{prt}^{qsu} delta(sP,sQ) delta(sR,sS) delta(sT,sU)."""
    N = L_sp.shape[0]
    M = 2 * N
    L = np.zeros((M,) * 6)
    Lprt = L_sp.transpose(0, 2, 4, 1, 3, 5)        # [p,r,t,q,s,u]
    for s1, s2, s3 in itertools.product((0, 1), repeat=3):
        a, b, c = s1 * N, s2 * N, s3 * N
        L[a:a + N, b:b + N, c:c + N, a:a + N, b:b + N, c:c + N] = Lprt
    return L


def spin_orbital_gamma(N, occ):
    g = np.zeros((2 * N, 2 * N))
    for k in occ:
        g[k, k] = 1.0
        g[N + k, N + k] = 1.0
    return g


# ---------------------------------------------------------------- step 5 --
def delta_U_so(L, g):
    """eq. dU: Delta U_{PR}^{QS} = -(L_{PRT}^{QSU} - L_{PRT}^{QUS} - L_{PRT}^{USQ}) gamma^T_U."""
    return -(np.einsum("prtqsu,tu->prqs", L, g, optimize=True)
             - np.einsum("prtqus,tu->prqs", L, g, optimize=True)
             - np.einsum("prtusq,tu->prqs", L, g, optimize=True))


def delta_h_so_from_L(L, g):
    """eq. tcmf:1el, first form:
    1/2 (L_{PRT}^{QSU} - L_{PRT}^{SQU} - L_{PRT}^{USQ}) (g^R_S g^T_U - g^R_U g^T_S)."""
    G2 = np.einsum("rs,tu->rtsu", g, g) - np.einsum("ru,ts->rtsu", g, g)
    return 0.5 * (np.einsum("prtqsu,rtsu->pq", L, G2, optimize=True)
                  - np.einsum("prtsqu,rtsu->pq", L, G2, optimize=True)
                  - np.einsum("prtusq,rtsu->pq", L, G2, optimize=True))


def delta_h_so_general(L, g):
    """The general one-body correction with an arbitrary reference, evaluated
    with the determinant's two-body density gamma^{RT}_{SU} = g^R_S g^T_U - g^R_U g^T_S:
    (L - L^{SQU} - L^{USQ}) (g^R_S g^T_U - g^R_U g^T_S - 1/2 gamma^{RT}_{SU})."""
    G2 = np.einsum("rs,tu->rtsu", g, g) - np.einsum("ru,ts->rtsu", g, g)
    Gw = np.einsum("rs,tu->rtsu", g, g) - np.einsum("ru,ts->rtsu", g, g) - 0.5 * G2
    return (np.einsum("prtqsu,rtsu->pq", L, Gw, optimize=True)
            - np.einsum("prtsqu,rtsu->pq", L, Gw, optimize=True)
            - np.einsum("prtusq,rtsu->pq", L, Gw, optimize=True))


def delta_h_so_from_dU(dU, g):
    """eq. tcmf:1el, second form: -1/2 (Delta U_{PR}^{QS} - Delta U_{PR}^{SQ}) gamma^R_S."""
    return -0.5 * (np.einsum("prqs,rs->pq", dU, g) - np.einsum("prsq,rs->pq", dU, g))


def zero_body_so(L, g):
    """<Phi0|L|Phi0> = -(1/6) L_{PRT}^{QSU} gamma^{PRT}_{QSU}; the three-body density
    of a determinant is the 3x3 determinant of one-body densities (eq. 1Ddens)."""
    terms = [("prtqsu,pq,rs,tu->", +1), ("prtqsu,pq,ru,ts->", -1),
             ("prtqsu,ps,rq,tu->", -1), ("prtqsu,ps,ru,tq->", +1),
             ("prtqsu,pu,rq,ts->", +1), ("prtqsu,pu,rs,tq->", -1)]
    acc = 0.0
    for spec, sgn in terms:
        acc += sgn * np.einsum(spec, L, g, g, g, optimize=True)
    return -acc / 6.0


def tier_a(xyz, w, phi, occ, jas):
    """All tier-A quantities for a closed-shell determinant on spatial orbitals phi.

    Returns a dict with the spin-orbital objects and the closed-shell outputs
    V2 [N]^4 (chemist), h1 [N]^2, E0."""
    N = phi.shape[0]
    V = grid_intermediate(xyz, w, phi, jas)
    Lsp = L_spatial(xyz, w, phi, jas, V)
    L = spin_orbital_L(Lsp)
    g = spin_orbital_gamma(N, occ)
    dU = delta_U_so(L, g)
    dh = delta_h_so_from_L(L, g)
    E0 = zero_body_so(L, g)
    V2 = np.ascontiguousarray(dU[:N, :N, :N, :N].transpose(0, 2, 1, 3))
    return dict(V=V, L_sp=Lsp, L_so=L, gamma_so=g, dU_so=dU, dh_so=dh, E0=E0,
                V2=V2, h1=dh[:N, :N].copy())


def spin_orbital_gamma_general(gamma):
    """Per-spin spatial density gamma [N][N] (the same for both spins, as in the
    closed-shell and spin-averaged equations) as a spin-orbital matrix."""
    N = gamma.shape[0]
    g = np.zeros((2 * N, 2 * N))
    g[:N, :N] = gamma
    g[N:, N:] = gamma
    return g


def tier_a_density(xyz, w, phi, gamma, jas):
    """Tier A for a general (not necessarily idempotent) per-spin density gamma:
    eq. dU for Delta U, the first form of eq. tcmf:1el for Delta h and
    eq. tcmf:0el for the zero-body term, all on the explicit six-index L.  For a
    correlated density the paper uses these single-determinant expressions as
    an approximation (higher cumulants neglected); they are its definition of
    the folded terms for such densities."""
    N = phi.shape[0]
    V = grid_intermediate(xyz, w, phi, jas)
    L = spin_orbital_L(L_spatial(xyz, w, phi, jas, V))
    g = spin_orbital_gamma_general(np.asarray(gamma, dtype=np.float64))
    dU = delta_U_so(L, g)
    dh = delta_h_so_from_L(L, g)
    E0 = -float(np.sum(dh * g)) / 3.0
    V2 = np.ascontiguousarray(dU[:N, :N, :N, :N].transpose(0, 2, 1, 3))
    return dict(L_so=L, gamma_so=g, dU_so=dU, dh_so=dh, E0=E0, V2=V2, h1=dh[:N, :N].copy())


def tier_a_open_shell(xyz, w, phi, occ_a, occ_b, jas):
    """Tier A for an open-shell determinant: alpha orbitals occ_a, beta occ_b
    (same spatial orbitals), on the explicit spin-orbital L.  Spin blocks
    V2[s][t][p,q,r,u] = Delta U_so[(p s),(r t),(q s),(u t)], h1[s] the
    (s, s) block of Delta h_so, and the zero-body term."""
    N = phi.shape[0]
    V = grid_intermediate(xyz, w, phi, jas)
    L = spin_orbital_L(L_spatial(xyz, w, phi, jas, V))
    g = np.zeros((2 * N, 2 * N))
    for k in occ_a:
        g[k, k] = 1.0
    for k in occ_b:
        g[N + k, N + k] = 1.0
    dU = delta_U_so(L, g)
    dh = delta_h_so_from_L(L, g)
    E0 = zero_body_so(L, g)
    sl = (slice(0, N), slice(N, 2 * N))
    V2 = [[np.ascontiguousarray(dU[sl[s], sl[t], sl[s], sl[t]].transpose(0, 2, 1, 3)) for t in range(2)]
          for s in range(2)]
    h1 = [dh[sl[s], sl[s]].copy() for s in range(2)]
    occ_so = [int(k) for k in occ_a] + [N + int(k) for k in occ_b]
    return dict(L_so=L, gamma_so=g, dU_so=dU, dh_so=dh, E0=E0, V2=V2, h1=h1, occ_so=occ_so)


# ---------------------------------------------------------------- step 6 --
def _apply(det: int, creators, annihilators):
    """Apply a^P1 a^P2 ... a_Qk ... a_Q1 (creators listed left to right,
    annihilators listed in the order they act) to the bit-string determinant."""
    sign = 1
    for q in annihilators:
        if not (det >> q) & 1:
            return 0, 0
        if bin(det & ((1 << q) - 1)).count("1") & 1:
            sign = -sign
        det &= ~(1 << q)
    for p in reversed(creators):
        if (det >> p) & 1:
            return 0, 0
        if bin(det & ((1 << p) - 1)).count("1") & 1:
            sign = -sign
        det |= 1 << p
    return sign, det


def _three_body_on(det, L, M, transpose=False, tol=0.0):
    """-(1/6) sum L_{PRT}^{QSU} a^P a^R a^T a_U a_S a_Q |det>  (or with L^T)."""
    occ = [k for k in range(M) if (det >> k) & 1]
    out = {}
    for Q, S, U in itertools.permutations(occ, 3):
        for P, R, T in itertools.permutations(range(M), 3):
            val = L[Q, S, U, P, R, T] if transpose else L[P, R, T, Q, S, U]
            if val == 0.0:
                continue
            sgn, d2 = _apply(det, (P, R, T), (Q, S, U))
            if sgn:
                out[d2] = out.get(d2, 0.0) - sgn * val / 6.0
    return out


def _folded_on(det, E0, dh, dU, M, transpose=False):
    """(E0 + dh_{PQ} a^P a_Q + 1/2 dU_{PR}^{QS} a^P a^R a_S a_Q) |det>  (or transposed)."""
    out = {det: E0}
    occ = [k for k in range(M) if (det >> k) & 1]
    for Q in occ:
        for P in range(M):
            val = dh[Q, P] if transpose else dh[P, Q]
            sgn, d2 = _apply(det, (P,), (Q,))
            if sgn:
                out[d2] = out.get(d2, 0.0) + sgn * val
    for Q, S in itertools.permutations(occ, 2):
        for P, R in itertools.permutations(range(M), 2):
            val = dU[Q, S, P, R] if transpose else dU[P, R, Q, S]
            sgn, d2 = _apply(det, (P, R), (Q, S))
            if sgn:
                out[d2] = out.get(d2, 0.0) + 0.5 * sgn * val
    return out


def determinant_check(L, dU, dh, E0, occ_so):
    """Matrix elements of T3 - (E0 + dh + dU) between the reference determinant and
    every determinant, grouped by excitation level: returns
    {level: max |<X|T3 - Tx|Phi0>|} and the same for <Phi0|T3 - Tx|X>."""
    M = L.shape[0]
    ref = 0
    for k in occ_so:
        ref |= 1 << int(k)
    res = {}
    for transpose in (False, True):
        a = _three_body_on(ref, L, M, transpose)
        b = _folded_on(ref, E0, dh, dU, M, transpose)
        diff = {}
        for d in set(a) | set(b):
            diff[d] = a.get(d, 0.0) - b.get(d, 0.0)
        worst = {}
        for d, v in diff.items():
            lvl = bin(d & ~ref).count("1")
            worst[lvl] = max(worst.get(lvl, 0.0), abs(v))
        res["ket" if not transpose else "bra"] = worst
    return res


def occ_spin_orbitals(N, occ):
    return [int(k) for k in occ] + [N + int(k) for k in occ]


def exact_K_entry(xyz, w, phi, jas, g, p, q):
    """One entry triple K^x_pq(g), x = 0..2, summed exactly (math.fsum) over g'."""
    d = grad1(xyz[g:g + 1], xyz, jas)[:, 0, :]     # [3][Ng]
    terms = w * phi[p] * phi[q]
    return np.array([math.fsum(d[x] * terms) for x in range(3)])
