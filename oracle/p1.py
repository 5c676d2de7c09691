"""P1 element matrices in closed form and their global assembly (FP64).

Paper passages: the matrices M, K (Sec. 5, definitions after the discrete
tentative-velocity expansion), the convection matrix C(u_bar) (Sec. 5, the
ABCN convection form eq:convection_ABCN with u_bar = 1.5 u^{n-1} - 0.5 u^{n-2}),
the pressure-gradient matrices dP^k (eq:dp_matrix).

For a simplex T with vertices x_0..x_d, J = [x_1-x_0, ..., x_d-x_0],
vol_T = |det J| / d!, and the barycentric gradients g_i (i >= 1) are the
columns of J^{-T}, g_0 = -sum_i g_i.  Every P1 integrand below is a
polynomial of degree <= 2, integrated exactly with the simplex monomial
formula  int_T l_i l_j = vol_T (1 + delta_ij) / ((d+1)(d+2)),
int_T l_i = vol_T / (d+1):

  M_T[i,j]   = vol_T (1 + delta_ij) / ((d+1)(d+2))
  K_T[i,j]   = vol_T g_i . g_j
  dP^k_T[i,j]= int_T (d_k phi_j) phi_i = vol_T g_j[k] / (d+1)
  C_T[i,j]   = int_T (u_bar . grad phi_j) phi_i
             = vol_T / ((d+1)(d+2)) * g_j . (S + u_bar_i),  S = sum_m u_bar_m

Row index i is the test function, column j the trial function.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def element_geometry(mesh):
    """Return (vol [E], grads [E, d+1, d]) for every cell."""
    d = mesh.dim
    X = mesh.coords[mesh.cells]                 # [E, d+1, d]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))   # columns x_i - x_0
    det = np.linalg.det(J)
    vol = np.abs(det) / math.factorial(d)
    JinvT = np.transpose(np.linalg.inv(J), (0, 2, 1))        # [E, d, d]
    g = np.empty((X.shape[0], d + 1, d))
    g[:, 1:, :] = np.transpose(JinvT, (0, 2, 1))             # g_i = column i of J^{-T}
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    return vol, g


def local_mass(vol, d):
    n = d + 1
    base = (np.ones((n, n)) + np.eye(n)) / ((d + 1) * (d + 2))
    return vol[:, None, None] * base[None]


def local_stiffness(vol, g):
    return vol[:, None, None] * np.einsum("eik,ejk->eij", g, g)


def local_gradient(vol, g, k):
    d = g.shape[2]
    # row i (test), column j (trial): vol * g_j[k] / (d+1), independent of i
    col = vol[:, None] * g[:, :, k] / (d + 1)
    return np.broadcast_to(col[:, None, :], (g.shape[0], d + 1, d + 1)).copy()


def local_convection(vol, g, ubar_cell):
    """ubar_cell: [E, d+1, d] nodal convecting velocity at the cell's vertices."""
    d = g.shape[2]
    S = ubar_cell.sum(axis=1)                                  # [E, d]
    w = S[:, None, :] + ubar_cell                              # [E, d+1(i), d]
    return (vol / ((d + 1) * (d + 2)))[:, None, None] * np.einsum("eid,ejd->eij", w, g)


def assemble(mesh, local):
    """Sum local [E, d+1, d+1] matrices into a global CSR over dofs."""
    dofs = mesh.vert2dof[mesh.cells]                           # [E, d+1]
    n = mesh.dim + 1
    rows = np.repeat(dofs, n, axis=1).ravel()
    cols = np.tile(dofs, (1, n)).ravel()
    A = sp.coo_matrix((local.ravel(), (rows, cols)), shape=(mesh.n_dof, mesh.n_dof)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def cell_ubar(mesh, ubar):
    """Gather the nodal convecting velocity [d, n_dof] onto cells: [E, d+1, d]."""
    dofs = mesh.vert2dof[mesh.cells]
    return np.transpose(ubar[:, dofs], (1, 2, 0))


def mass_matrix(mesh, geo=None):
    vol, g = geo if geo is not None else element_geometry(mesh)
    return assemble(mesh, local_mass(vol, mesh.dim))


def stiffness_matrix(mesh, geo=None):
    vol, g = geo if geo is not None else element_geometry(mesh)
    return assemble(mesh, local_stiffness(vol, g))


def gradient_matrix(mesh, k, geo=None):
    vol, g = geo if geo is not None else element_geometry(mesh)
    return assemble(mesh, local_gradient(vol, g, k))


def convection_matrix(mesh, ubar, geo=None):
    vol, g = geo if geo is not None else element_geometry(mesh)
    return assemble(mesh, local_convection(vol, g, cell_ubar(mesh, ubar)))


def on_pattern(A, pattern):
    """Values of A laid out on the CSR pattern `pattern` (same shape, superset)."""
    P = pattern.tocsr()
    out = np.zeros(P.nnz)
    rows = np.repeat(np.arange(P.shape[0]), np.diff(P.indptr))
    vals = np.asarray(A[rows, P.indices]).ravel()
    out[:] = vals
    return out
