"""Differentiation oracle: the loss E0 + <h1, D> + <V2, G> and its gradient
with respect to the power-Jastrow coefficients c_k; for the restricted
open-shell equations (Appendix A) the loss
E0 + sum_s <h1^s, D^s> + sum over the blocks (aa, ab, bb) of <V2^st, G^st>.

The grid intermediate V is linear in u, hence in c; L on the grid (eq. Ldecomp)
is quadratic in V, and so are Delta U, Delta h and the zero-body term.  The
loss is therefore an exact homogeneous quadratic form c^T Q c, and the central
difference with unit step, [loss(c + e_k) - loss(c - e_k)] / 2 = 2 (Q c)_k, is
its exact gradient (up to rounding): no step-size truncation error.
"""
from __future__ import annotations

from collections import namedtuple

import numpy as np

from .factorised import closed_shell, open_shell

PowerJastrow = namedtuple("PowerJastrow", "kind b coef")


def loss(xyz, w, phi, occ, coef, D, G):
    jas = PowerJastrow("power", 0.0, tuple(float(c) for c in coef))
    V2, h1, E0 = closed_shell(xyz, w, phi, occ, jas)
    return E0 + float(np.sum(h1 * D)) + float(np.sum(V2 * G))


def exact_gradient(xyz, w, phi, occ, coef, D, G):
    coef = np.asarray(coef, dtype=np.float64)
    g = np.zeros_like(coef)
    for k in range(len(coef)):
        e = np.zeros_like(coef)
        e[k] = 1.0
        g[k] = 0.5 * (loss(xyz, w, phi, occ, coef + e, D, G)
                      - loss(xyz, w, phi, occ, coef - e, D, G))
    return g


def loss_open(xyz, w, phi, gamma_a, gamma_b, coef, D, G):
    """D = (D^a, D^b) [N][N] each; G = (G^aa, G^ab, G^bb) [N]^4 each, the
    blocks V2^st of the spin-resolved two-body term."""
    jas = PowerJastrow("power", 0.0, tuple(float(c) for c in coef))
    V2, h1, E0 = open_shell(xyz, w, phi, gamma_a, gamma_b, jas)
    blocks = (V2[0][0], V2[0][1], V2[1][1])
    return (E0 + sum(float(np.sum(h1[s] * D[s])) for s in range(2))
            + sum(float(np.sum(b * g)) for b, g in zip(blocks, G)))


def exact_gradient_open(xyz, w, phi, gamma_a, gamma_b, coef, D, G):
    coef = np.asarray(coef, dtype=np.float64)
    g = np.zeros_like(coef)
    for k in range(len(coef)):
        e = np.zeros_like(coef)
        e[k] = 1.0
        g[k] = 0.5 * (loss_open(xyz, w, phi, gamma_a, gamma_b, coef + e, D, G)
                      - loss_open(xyz, w, phi, gamma_a, gamma_b, coef - e, D, G))
    return g
