"""Electron-electron Jastrow u(r12) and its first-argument gradient (oracle).

The three-body integrals contain grad_1 u(r1, r2) (Theory, definition of L);
for u depending only on r12 = |r1 - r2| this is u'(r12) (r1 - r2)/r12.
At coincident points (r12 == 0 exactly) the paper is silent; the gradient of
an isotropic function is taken as zero there (it is bounded by max u').

Supported forms (parameters are plain Python values):
* Pade:  u = r / (2 (1 + b r)),        u' = 1 / (2 (1 + b r)^2),  u'' = -b / (1 + b r)^3
* power: u = sum_k c_k t^k, t = r/(1+r), u' = sum_k k c_k t^(k-1) / (1 + r)^2,
         u'' = sum_k k (k-1) c_k t^(k-2) / (1 + r)^4 - 2 sum_k k c_k t^(k-1) / (1 + r)^3

The two-body TC integrals (Theory, definition of K) need the scalar
  S(r1, r2) = laplacian_1 u + |grad_1 u|^2 = u'' + 2 u'/r + u'^2,
which is symmetric in the two points; at coincident points it is taken as
zero, like the gradient (the 2u'/r term is integrable but not finite there).
"""
from __future__ import annotations

import numpy as np


def u_of_r(r, kind: str, b: float = 1.0, coef=()):
    r = np.asarray(r, dtype=np.float64)
    if kind == "pade":
        return r / (2.0 * (1.0 + b * r))
    if kind == "power":
        t = r / (1.0 + r)
        return sum(c * t ** (k + 1) for k, c in enumerate(coef))
    raise ValueError(kind)


def du_dr(r, kind: str, b: float = 1.0, coef=()):
    r = np.asarray(r, dtype=np.float64)
    if kind == "pade":
        return 1.0 / (2.0 * (1.0 + b * r) ** 2)
    if kind == "power":
        t = r / (1.0 + r)
        s = sum((k + 1) * c * t ** k for k, c in enumerate(coef))
        return s / (1.0 + r) ** 2
    raise ValueError(kind)


def grad1(xa: np.ndarray, xb: np.ndarray, jas) -> np.ndarray:
    """grad_1 u(r_a, r_b) for all pairs: array [3][len(xa)][len(xb)].

    ``jas`` has attributes kind, b, coef.  Zero where r_a == r_b exactly.
    """
    d = np.empty((3, len(xa), len(xb)))            # [3][na][nb], C order
    np.subtract(np.ascontiguousarray(xa.T)[:, :, None], np.ascontiguousarray(xb.T)[:, None, :], out=d)
    r = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    up = du_dr(r, jas.kind, jas.b, jas.coef)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(r > 0.0, up / np.where(r > 0.0, r, 1.0), 0.0)
    d *= f
    return d


def d2u_dr2(r, kind: str, b: float = 1.0, coef=()):
    r = np.asarray(r, dtype=np.float64)
    if kind == "pade":
        return -b / (1.0 + b * r) ** 3
    if kind == "power":
        t = r / (1.0 + r)
        s2 = sum((k + 1) * k * c * t ** (k - 1) for k, c in enumerate(coef) if k >= 1)
        s1 = sum((k + 1) * c * t ** k for k, c in enumerate(coef))
        return s2 / (1.0 + r) ** 4 - 2.0 * s1 / (1.0 + r) ** 3
    raise ValueError(kind)


def scalar_kernel(xa: np.ndarray, xb: np.ndarray, jas) -> np.ndarray:
    """S = laplacian_1 u + |grad_1 u|^2 for all pairs, [len(xa)][len(xb)]; 0 at r == 0."""
    d = xa[:, None, :] - xb[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    up = du_dr(r, jas.kind, jas.b, jas.coef)
    upp = d2u_dr2(r, jas.kind, jas.b, jas.coef)
    with np.errstate(divide="ignore", invalid="ignore"):
        S = np.where(r > 0.0, upp + 2.0 * up / np.where(r > 0.0, r, 1.0) + up * up, 0.0)
    return S
