"""Naive reassembly of the tentative-velocity system by quadrature.

The paper's naive solver (Sec. 4, the solvers submodule: the tentative form
F[ui] with the Crank-Nicolson velocity U_CN = (u + u^{n-1})/2 and convecting
velocity U_AB = 1.5 u^{n-1} - 0.5 u^{n-2}) reassembles the whole system
every step; the paper uses it to verify the optimised solver, which is "the
same" scheme.  Here the bilinear and linear forms are integrated cell by cell
with a collapsed Gauss-Legendre rule, evaluating the P1 basis and the known
fields at the quadrature points, without the closed-form element matrices.

  a(u, v) = (1/dt) u v + (1/2)(u_bar . grad u) v + (nu/2) grad u . grad v
  L(v)    = (1/dt) u1 v - (1/2)(u_bar . grad u1) v - (nu/2) grad u1 . grad v
            - (d_k p*) v + f_k v
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import quadrature


def _basis(mesh, nq):
    pts, wts = quadrature.simplex_rule(mesh.dim, nq)
    lam = quadrature.barycentric(pts)                      # [Q, n] basis values
    X = mesh.coords[mesh.cells]                            # [E, n, dim]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    detJ = np.abs(np.linalg.det(J))
    d = mesh.dim
    dref = np.vstack([-np.ones((1, d)), np.eye(d)])        # reference gradients [n, d]
    JinvT = np.transpose(np.linalg.inv(J), (0, 2, 1))
    grad = np.einsum("eab,ib->eia", JinvT, dref)           # physical gradients [E, n, d]
    w = detJ[:, None] * wts[None, :]                       # [E, Q]
    return lam, grad, w


def tentative_system(mesh, nu, dt, f, U1, U2, p_star, k, nq=3):
    """Return (A_k, b_k) for component k, before Dirichlet rows."""
    lam, grad, w = _basis(mesh, nq)
    dofs = mesh.vert2dof[mesh.cells]
    ubar = 1.5 * U1 - 0.5 * U2
    ubar_q = np.einsum("qi,cei->eqc", lam, ubar[:, dofs])            # [E, Q, d]
    adv = np.einsum("eqc,ejc->eqj", ubar_q, grad)                    # u_bar . grad phi_j
    mass = np.einsum("eq,qi,qj->eij", w, lam, lam)
    conv = np.einsum("eq,qi,eqj->eij", w, lam, adv)
    stiff = np.einsum("eq,eic,ejc->eij", w, grad, grad)
    Aloc = mass / dt + 0.5 * conv + 0.5 * nu * stiff
    u1_loc = U1[k][dofs]                                             # [E, n]
    u1_q = np.einsum("qi,ei->eq", lam, u1_loc)
    gu1 = np.einsum("ei,eic->ec", u1_loc, grad)                      # constant per cell
    adv_u1 = np.einsum("eqc,ec->eq", ubar_q, gu1)
    dkp = np.einsum("ei,ei->e", p_star[dofs], grad[:, :, k])
    integrand = (u1_q / dt - 0.5 * adv_u1 - dkp[:, None] + f[k])     # [E, Q] times v
    bloc = np.einsum("eq,qi,eq->ei", w, lam, integrand)
    bloc -= 0.5 * nu * np.einsum("ec,eic,eq->ei", gu1, grad, w)
    n = mesh.dim + 1
    rows = np.repeat(dofs, n, axis=1).ravel()
    cols = np.tile(dofs, (1, n)).ravel()
    A = sp.coo_matrix((Aloc.ravel(), (rows, cols)), shape=(mesh.n_dof,) * 2).tocsr()
    b = np.zeros(mesh.n_dof)
    np.add.at(b, dofs.ravel(), bloc.ravel())
    return A, b
