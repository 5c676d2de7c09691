"""Gauss-Legendre product rules collapsed onto the unit simplex (Duffy map).

Used to pin the closed-form element matrices and to compute L2 error norms.
The reference simplex is {xi_i >= 0, sum xi_i <= 1}; a rule with n points per
axis integrates polynomials of total degree <= 2n - 1 - (d - 1) exactly.
"""
from __future__ import annotations

import numpy as np


def simplex_rule(d: int, n: int):
    """Return (points [Q, d], weights [Q]) on the unit reference simplex."""
    t, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    if d == 2:
        U, V = np.meshgrid(t, t, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        x = U
        y = V * (1.0 - U)
        wt = WU * WV * (1.0 - U)
        return np.stack([x.ravel(), y.ravel()], axis=1), wt.ravel()
    if d == 3:
        U, V, W = np.meshgrid(t, t, t, indexing="ij")
        WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
        x = U
        y = V * (1.0 - U)
        z = W * (1.0 - U) * (1.0 - V)
        wt = WU * WV * WW * (1.0 - U) ** 2 * (1.0 - V)
        return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), wt.ravel()
    raise ValueError("dim must be 2 or 3")


def barycentric(points: np.ndarray) -> np.ndarray:
    """[Q, d] reference points -> [Q, d+1] barycentric coordinates."""
    return np.concatenate([1.0 - points.sum(axis=1, keepdims=True), points], axis=1)
