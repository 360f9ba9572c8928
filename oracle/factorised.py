"""Tier B oracle: the closed-shell working equations (Appendix B), any size.

Literal transcription, in FP64 numpy on full (unpacked) N x N orbital pairs,
of the restricted closed-shell equations: the factor of two of spin
integration is written into W, W~, Delta h and the zero-body term, and gamma is
the per-spin one-body density (here a real symmetric N x N matrix; for a
closed-shell determinant the projector onto the occupied orbitals).

Grid sums are implicit in the paper (Einstein convention over the grid index i
in eq. tcmf:2el); the permutation operator P^{(pq)}_{(rs)} there is read as
f(pq, rs) + f(rs, pq).

Orbital-subset restriction: Delta U[pq, rs] only involves grid intermediates
of pairs inside {p, q, r, s} and the occupied orbitals, so calling ``closed_shell``
with phi restricted to S = occ + any other orbitals returns the exact S-blocks
of V2 and h1 and the exact E0.
"""
from __future__ import annotations

import os
from collections import deque
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .jastrow import grad1


def grid_K(xyz, w, phi, jas, rows):
    """V_r^s(i) for the grid rows ``rows`` (a slice), [3][len][N][N]:
    sum_j w_j phi_r(j) grad_1 u(r_i, r_j) phi_s(j)."""
    d = grad1(xyz[rows], xyz, jas)
    N = phi.shape[0]
    rho_j = ((phi * w)[:, None, :] * phi[None, :, :]).reshape(N * N, -1)   # [rs][j]
    K = np.einsum("xij,aj->xia", d, rho_j, optimize=True)
    return K.reshape(3, -1, N, N)


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def grid_K_blocks(xyz, w, phi, jas, block):
    """(rows, V) for the successive row blocks [i0, i0 + block) of the grid, V
    as in grid_K.  Only the evaluation order differs: the Jastrow gradients of
    the next blocks are computed ahead on a thread pool (numpy's array loops
    release the interpreter lock), and the sums over j run in block order.
    Blocks shrink on large grids so that the gradients in flight stay within
    a few GB."""
    N, Ng = phi.shape
    block = max(16, min(block, (1 << 25) // max(1, Ng)))
    rho_j = ((phi * w)[:, None, :] * phi[None, :, :]).reshape(N * N, -1)   # [rs][j]
    starts = iter(range(0, Ng, block))
    nt = _threads()
    with ThreadPoolExecutor(nt) as pool:
        pending = deque()

        def submit():
            i0 = next(starts, None)
            if i0 is not None:
                rows = slice(i0, min(Ng, i0 + block))
                pending.append((rows, pool.submit(grad1, xyz[rows], xyz, jas)))

        for _ in range(nt + 1):
            submit()
        while pending:
            rows, fut = pending.popleft()
            d = fut.result()
            submit()
            nb = d.shape[1]
            yield rows, (d.reshape(3 * nb, Ng) @ rho_j.T).reshape(3, nb, N, N)


def intermediates(rho, K, gamma):
    """eq. tcmf:inter (closed shell) for a block of grid points.

    rho [i][r][s], K [3][i][r][s] (V in the paper), gamma [N][N].
    Returns A [i][r][s] and B [3][i][r][s]."""
    W = 2.0 * np.einsum("xitu,tu->xi", K, gamma)                  # W = 2 V_t^u g^t_u
    X = np.einsum("xits,tu->xius", K, gamma)                       # X_u^s = V_t^s g^t_u
    Zt = np.einsum("xiru,xius->irs", K, X)                         # Z~ = V_r^u . X_u^s
    Vt = np.einsum("xi,xirs->irs", W, K)                           # V~ = W . V
    A = Vt - Zt
    Wt = 2.0 * np.einsum("itu,tu->i", rho, gamma)                  # W~ = 2 rho_t^u g^t_u
    Y = np.einsum("xiru,tu->xirt", K, gamma)                       # Y_r^t = V_r^u g^t_u
    Z = (np.einsum("iru,xius->xirs", rho, X)
         + np.einsum("xirt,its->xirs", Y, rho))                    # Z = rho X + Y rho
    B = 0.5 * Wt[None, :, None, None] * K - Z
    return A, B


def closed_shell(xyz, w, phi, gamma, jas, block=512, return_f=False):
    """V2 [N]^4 (V2[p,q,r,s] = Delta U_{pr}^{qs}), h1 [N][N] and E0.

    ``gamma`` may be an (N x N) matrix or an index array of occupied orbitals."""
    N, Ng = phi.shape
    gamma = _as_gamma(gamma, N)
    f = np.zeros((N * N, N * N))
    for rows, K in grid_K_blocks(xyz, w, phi, jas, block):
        rho = w[rows, None, None] * phi[:, rows].T[:, :, None] * phi[:, rows].T[:, None, :]
        A, B = intermediates(rho, K, gamma)
        nb = rho.shape[0]
        # f(pq, rs) = sum_i rho_pq(i) A_rs(i) + V_pq(i) . B_rs(i)
        f += rho.reshape(nb, -1).T @ A.reshape(nb, -1)
        for x in range(3):
            f += K[x].reshape(nb, -1).T @ B[x].reshape(nb, -1)
    # eq. tcmf:2el: Delta U_pr^qs = -(f(pq, rs) + f(rs, pq))
    V2 = -(f + f.T).reshape(N, N, N, N)
    h1 = one_body_from_V2(V2, gamma)
    E0 = zero_body_from_h1(h1, gamma)
    if return_f:
        return V2, h1, E0, f.reshape(N, N, N, N)
    return V2, h1, E0


def intermediates_spin(rho, K, g_tau, g_tot):
    """Appendix A (restricted open shell) intermediates of spin tau:
    W = V_t^u sum_rho gamma^rho, W~ = rho_t^u sum_rho gamma^rho (total density, no
    factor two), X^tau, Y^tau, Z~^tau, Z^tau with the density of spin tau."""
    W = np.einsum("xitu,tu->xi", K, g_tot)
    X = np.einsum("xits,tu->xius", K, g_tau)
    Zt = np.einsum("xiru,xius->irs", K, X)
    A = np.einsum("xi,xirs->irs", W, K) - Zt
    Wt = np.einsum("itu,tu->i", rho, g_tot)
    Y = np.einsum("xiru,tu->xirt", K, g_tau)
    Z = np.einsum("iru,xius->xirs", rho, X) + np.einsum("xirt,its->xirs", Y, rho)
    B = 0.5 * Wt[None, :, None, None] * K - Z
    return A, B


def open_shell(xyz, w, phi, gamma_a, gamma_b, jas, block=512):
    """Restricted open-shell working equations (Appendix A): same spatial
    orbitals and Jastrow for both spins, spin-specific densities.

    Returns V2[s][t] [N]^4 for (s, t) in {a, b}^2 (V2[s][t][p,q,r,s'] =
    [Delta U_pr^qs']^{st}), h1[s] [N][N] and E0, with
      [Delta U]^{st}[pq, rs] = -(f^t(pq, rs) + f^s(rs, pq)),
      f^t(pq, rs) = sum_i rho_pq A^t_rs + V_pq . B^t_rs,
      [Delta h]^s = -1/2 (sum_t [Delta U_pr^qs]^{st} g^t_rs - [Delta U_pr^sq]^{ss} g^s_rs),
      E0 = -1/3 sum_s [Delta h]^s . g^s."""
    N, Ng = phi.shape
    ga, gb = _as_gamma(gamma_a, N), _as_gamma(gamma_b, N)
    gs = (ga, gb)
    gtot = ga + gb
    f = [np.zeros((N * N, N * N)), np.zeros((N * N, N * N))]
    for rows, K in grid_K_blocks(xyz, w, phi, jas, block):
        rho = w[rows, None, None] * phi[:, rows].T[:, :, None] * phi[:, rows].T[:, None, :]
        nb = rho.shape[0]
        for t in range(2):
            A, B = intermediates_spin(rho, K, gs[t], gtot)
            f[t] += rho.reshape(nb, -1).T @ A.reshape(nb, -1)
            for x in range(3):
                f[t] += K[x].reshape(nb, -1).T @ B[x].reshape(nb, -1)
    V2 = [[-(f[t] + f[s].T).reshape(N, N, N, N) for t in range(2)] for s in range(2)]
    h1 = []
    for s in range(2):
        h = sum(np.einsum("pqrs,rs->pq", V2[s][t], gs[t]) for t in range(2))
        h = h - np.einsum("psrq,rs->pq", V2[s][s], gs[s])
        h1.append(-0.5 * h)
    E0 = -sum(float(np.einsum("pq,pq->", h1[s], gs[s])) for s in range(2)) / 3.0
    return V2, h1, E0


def frozen_core(V2, h1, E0, core, active):
    """Closed-shell frozen-core folding of a zero-, one- and two-body operator
    (the xTC-FC scheme of the results section: the corrections are computed
    with all electrons, then the standard frozen-core equations are applied),
    with V2[p,q,r,s] = (pq|rs) and a doubly occupied core:
      E  = E0 + 2 sum_c h1[c,c] + sum_{c,d} (2 (cc|dd) - (cd|dc)),
      h[p,q] = h1[p,q] + sum_c (2 (pq|cc) - (pc|cq)),   p, q active,
      V = V2 restricted to the active orbitals."""
    c = np.asarray(core, dtype=int)
    a = np.asarray(active, dtype=int)
    E = E0 + 2.0 * float(np.trace(h1[np.ix_(c, c)]))
    E += float(np.sum(2.0 * np.einsum("ccdd->cd", V2[np.ix_(c, c, c, c)]) - np.einsum("cddc->cd", V2[np.ix_(c, c, c, c)])))
    h = h1[np.ix_(a, a)].copy()
    h += 2.0 * np.einsum("pqcc->pq", V2[np.ix_(a, a, c, c)]) - np.einsum("pccq->pq", V2[np.ix_(a, c, c, a)])
    return V2[np.ix_(a, a, a, a)].copy(), h, E


def one_body_from_V2(V2, gamma):
    """Appendix B: Delta h_p^q = -1/2 (2 Delta U_pr^qs g^r_s - Delta U_pr^sq g^r_s),
    with Delta U_pr^qs = V2[p,q,r,s] and Delta U_pr^sq = V2[p,s,r,q]."""
    return -0.5 * (2.0 * np.einsum("pqrs,rs->pq", V2, gamma)
                   - np.einsum("psrq,rs->pq", V2, gamma))


def zero_body_from_h1(h1, gamma):
    """Appendix B: <Psi0|L|Psi0> = -(2/3) Delta h_p^q g^p_q."""
    return -(2.0 / 3.0) * float(np.einsum("pq,pq->", h1, gamma))


def _as_gamma(gamma, N):
    g = np.asarray(gamma)
    if g.ndim == 2:
        return g.astype(np.float64)
    G = np.zeros((N, N))
    for k in g:
        G[int(k), int(k)] = 1.0
    return G


def subset(phi, occ, extra):
    """Orbital subset S = occ + extra (in that order) and occ's positions in S."""
    S = [int(k) for k in occ] + [int(k) for k in extra if int(k) not in set(map(int, occ))]
    return np.array(S), np.arange(len(occ))

