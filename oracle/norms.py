"""L2 error norms of P1 fields against closed-form functions.

The Taylor-Green errors of the paper (Sec. 6.1, Table 1) are L2 norms.
Reading: ||u_h - u_e|| = sqrt(sum_k ||u_h,k - u_e,k||^2_{L2(Omega)}) with a
per-cell collapsed Gauss-Legendre rule (5 points per axis, exact to degree
>= 8); for the pressure both fields have their domain mean removed first.
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature


def _quad_points(mesh, n=5):
    pts, wts = quadrature.simplex_rule(mesh.dim, n)
    lam = quadrature.barycentric(pts)                        # [Q, d+1]
    X = mesh.coords[mesh.cells]                              # [E, d+1, dim]
    xq = np.einsum("qi,eid->eqd", lam, X)                    # [E, Q, dim]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    detJ = np.abs(np.linalg.det(J))                          # = d! vol
    w = detJ[:, None] * wts[None, :]                         # [E, Q]
    return lam, xq, w


def l2_error(mesh, values, exact, n=5, remove_mean=False):
    """values: [N] dof values of a P1 field; exact: callable (x[..., dim]) -> f."""
    lam, xq, w = _quad_points(mesh, n)
    dofs = mesh.vert2dof[mesh.cells]
    uh = np.einsum("qi,ei->eq", lam, values[dofs])
    ue = exact(xq)
    e = uh - ue
    if remove_mean:
        vol = w.sum()
        e = e - (w * e).sum() / vol
    return math.sqrt(float((w * e * e).sum()))


def vector_l2_error(mesh, values, exact_list, n=5):
    return math.sqrt(sum(l2_error(mesh, values[k], exact_list[k], n) ** 2
                         for k in range(len(exact_list))))
