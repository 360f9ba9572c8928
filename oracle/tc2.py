"""Two-body transcorrelated integrals on the grid (oracle; test infrastructure only).

Theory, definition of K:
  K_pr^qs = 1/2 <pr| P^1_2 ( lap_1 u + (grad_1 u)^2 + 2 grad_1 u . grad_1 ) |qs>,
  P^1_2 f(1,2) = f(1,2) + f(2,1),
with p, q on electron 1 and r, s on electron 2, evaluated with both electrons
on the same weighted grid.  Output K2[p][q][r][s] = K_pr^qs (the order of V2).
At coincident points both the gradient and S = lap_1 u + |grad_1 u|^2 are
taken as zero.  Needs the orbital gradients on the grid, dphi [3][N][Ng].
"""
from __future__ import annotations

import numpy as np

from .factorised import grid_K
from .jastrow import grad1, scalar_kernel


def tc_two_body_explicit(xyz, w, phi, dphi, jas):
    """The definition written out as one double grid sum per term (tiny inputs)."""
    S = scalar_kernel(xyz, xyz, jas)                  # S(g,g') = S(g',g)
    G = grad1(xyz, xyz, jas)                           # grad_1 u(r_g, r_g'), [3][g][g']
    wphi = w * phi
    # f(1,2) on phi_q(1) phi_s(2): (lap_1 u + |grad_1 u|^2) phi_q phi_s + 2 grad_1 u . grad phi_q phi_s
    t1 = np.einsum("pg,qg,gh,rh,sh->pqrs", wphi, phi, S, wphi, phi, optimize=True)
    t2 = 2.0 * np.einsum("pg,xqg,xgh,rh,sh->pqrs", wphi, dphi, G, wphi, phi, optimize=True)
    # f(2,1): the same operator acting on electron 2 (u(r2, r1) = u(r1, r2))
    t3 = np.einsum("pg,qg,hg,rh,sh->pqrs", wphi, phi, S, wphi, phi, optimize=True)
    t4 = 2.0 * np.einsum("pg,qg,xhg,rh,xsh->pqrs", wphi, phi, G, wphi, dphi, optimize=True)
    return 0.5 * (t1 + t2 + t3 + t4)


def tc_two_body(xyz, w, phi, dphi, jas, block=512):
    """Factorised on the grid: with rho_pq = w phi_p phi_q, F_rs(g) = sum_g' S(g,g') rho_rs(g'),
    K_rs(g) = sum_g' grad_1 u(g,g') rho_rs(g') (the xTC grid intermediate) and
    rhog_pq(g) = w phi_p grad phi_q (not symmetric in p, q):
      K2[pq,rs] = A[pq,rs] + B[pq,rs] + B[rs,pq],
      A = sum_g rho_pq F_rs,  B = sum_g rhog_pq . K_rs."""
    N, Ng = phi.shape
    rho_j = ((phi * w)[:, None, :] * phi[None, :, :]).reshape(N * N, -1)
    A = np.zeros((N * N, N * N))
    B = np.zeros((N * N, N * N))
    for i0 in range(0, Ng, block):
        rows = slice(i0, min(Ng, i0 + block))
        F = scalar_kernel(xyz[rows], xyz, jas) @ rho_j.T                       # [nb][N^2]
        K = grid_K(xyz, w, phi, jas, rows).reshape(3, -1, N * N)             # [3][nb][N^2]
        nb = F.shape[0]
        rho = rho_j[:, rows].T                                                 # [nb][N^2]
        rhog = (w[rows] * phi[:, rows])[None, :, None, :] * dphi[:, None, :, rows]   # [3][p][q][g]
        rhog = rhog.reshape(3, N * N, nb)
        A += rho.T @ F
        for x in range(3):
            B += rhog[x] @ K[x]
    return (A + B + B.T).reshape(N, N, N, N)


def quadratic_part(xyz, w, phi, jas):
    """The part of K2 that is quadratic in u: sum_{g,g'} rho_pq(g) |grad_1 u|^2 rho_rs(g')."""
    G = grad1(xyz, xyz, jas)
    g2 = np.sum(G * G, axis=0)
    rho = ((phi * w)[:, None, :] * phi[None, :, :]).reshape(phi.shape[0] ** 2, -1)
    N = phi.shape[0]
    return (rho @ g2 @ rho.T).reshape(N, N, N, N)
