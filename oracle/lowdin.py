"""Symmetric (Loewdin) orthonormalisation under the grid weights (oracle).

S_mn = sum_g w_g chi_m(g) chi_n(g);  phi = S^{-1/2} chi, with S^{-1/2} the
symmetric inverse square root (eigen-decomposition of S).  Among all sets
phi = C chi that are orthonormal under w, this one minimises
sum_m ||phi_m - chi_m||_w^2, and C is symmetric positive definite.
"""
from __future__ import annotations

import numpy as np


def overlap(chi, w):
    return (chi * w) @ chi.T


def lowdin(chi, w):
    S = overlap(chi, w)
    S = 0.5 * (S + S.T)
    lam, U = np.linalg.eigh(S)
    C = (U / np.sqrt(lam)) @ U.T
    return C @ chi, C, lam
