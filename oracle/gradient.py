"""Differentiation oracle: the loss E0 + <h1, D> + <V2, G> and its gradient
with respect to the power-Jastrow coefficients c_k.

The grid intermediate V is linear in u, hence in c; L on the grid (eq. Ldecomp)
is quadratic in V, and so are Delta U, Delta h and the zero-body term.  The
loss is therefore an exact homogeneous quadratic form c^T Q c, and the central
difference with unit step, [loss(c + e_k) - loss(c - e_k)] / 2 = 2 (Q c)_k, is
its exact gradient (up to rounding): no step-size truncation error.
"""
from __future__ import annotations

from collections import namedtuple

import numpy as np

from .factorised import closed_shell

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
