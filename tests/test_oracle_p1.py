"""Pins for the oracle's element matrices and global matrix invariants.

The element matrices are checked against brute-force quadrature in which the
barycentric coordinates are obtained by solving the affine system of each
simplex and their gradients by finite differences, so a wrong factor, sign,
index or transpose in the closed forms fails here.
"""
import math

import numpy as np
import pytest

import synth
from oracle import graph, ipcs, p1, quadrature


def _random_simplices(d, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        X = rng.normal(size=(d + 1, d))
        J = (X[1:] - X[0]).T
        if abs(np.linalg.det(J)) > 0.05:
            out.append(X)
    return out


def _bary_solve(X, pts):
    """Barycentric coordinates of physical points by solving [X^T; 1] l = [x; 1]."""
    d = X.shape[1]
    Amat = np.vstack([X.T, np.ones(d + 1)])
    rhs = np.vstack([pts.T, np.ones(pts.shape[0])])
    return np.linalg.solve(Amat, rhs).T             # [Q, d+1]


@pytest.mark.parametrize("d", [2, 3])
def test_element_matrices_vs_quadrature(d):
    pts_ref, w_ref = quadrature.simplex_rule(d, 6)
    rng = np.random.default_rng(11)
    for X in _random_simplices(d, 100, seed=d):
        class _M:  # one-cell mesh
            pass
        m = _M()
        m.dim = d
        m.coords = X
        m.cells = np.arange(d + 1, dtype=np.int32)[None]
        vol, g = p1.element_geometry(m)
        # physical quadrature points through the affine map, weights scaled by |det J|
        J = (X[1:] - X[0]).T
        xq = X[0] + pts_ref @ J.T
        wq = w_ref * abs(np.linalg.det(J))
        assert np.isclose(wq.sum(), vol[0], rtol=1e-13)
        lam = _bary_solve(X, xq)
        # gradients by central differences of the barycentric map (exact for affine maps)
        eps = 1e-3
        gfd = np.zeros((d + 1, d))
        x0 = X.mean(axis=0)
        for k in range(d):
            e = np.zeros(d)
            e[k] = eps
            gfd[:, k] = (_bary_solve(X, (x0 + e)[None])[0] - _bary_solve(X, (x0 - e)[None])[0]) / (2 * eps)
        np.testing.assert_allclose(g[0], gfd, rtol=1e-9, atol=1e-9)
        Mq = np.einsum("q,qi,qj->ij", wq, lam, lam)
        np.testing.assert_allclose(p1.local_mass(vol, d)[0], Mq, rtol=1e-12, atol=1e-14)
        Kq = np.einsum("q,ik,jk->ij", wq, gfd, gfd)
        np.testing.assert_allclose(p1.local_stiffness(vol, g)[0], Kq, rtol=1e-8, atol=1e-10)
        for k in range(d):
            Gq = np.einsum("q,qi,j->ij", wq, lam, gfd[:, k])
            np.testing.assert_allclose(p1.local_gradient(vol, g, k)[0], Gq, rtol=1e-8, atol=1e-10)
        ub = rng.normal(size=(d + 1, d))             # nodal convecting velocity
        uq = lam @ ub                                # [Q, d]
        Cq = np.einsum("q,qi,qk,jk->ij", wq, lam, uq, gfd)
        np.testing.assert_allclose(p1.local_convection(vol, g, ub[None])[0], Cq, rtol=1e-8, atol=1e-10)


def _meshes():
    return [synth.unit_square(7), synth.periodic_square(6),
            synth.channel(9, 9, 7), synth.channel(9, 9, 7, displace_seed=3)]


@pytest.mark.parametrize("mesh", _meshes(), ids=lambda m: m.name)
def test_global_invariants(mesh):
    S = ipcs.setup(mesh, 0.01, 1e-3, np.zeros(mesh.dim))
    N = mesh.n_dof
    one = np.ones(N)
    K, M = S.K, S.M
    scale = abs(K).max()
    assert abs(K - K.T).max() <= 1e-14 * scale
    assert np.abs(K @ one).max() <= 1e-12 * scale
    assert np.isclose(one @ (M @ one), mesh.volume, rtol=1e-12)
    rng = np.random.default_rng(0)
    ubar = rng.normal(size=(mesh.dim, N))
    C = p1.convection_matrix(mesh, ubar, S.geo)
    assert np.abs(C @ one).max() <= 1e-12 * abs(C).max()
    for k in range(mesh.dim):
        assert np.abs(S.dP[k] @ one).max() <= 1e-12 * abs(S.dP[k]).max()
    # coordinates that are globally linear (not wrapped by periodicity)
    nonper = {"unit_square_7": [0, 1], "periodic_square_6": [], "channel_9x9x7": [1],
              "channel_9x9x7_disp3": [1]}[mesh.name]
    for m_ in nonper:
        xm = mesh.dof_coords[:, m_]
        for k in range(mesh.dim):
            expect = S.ML if k == m_ else np.zeros(N)
            np.testing.assert_allclose(S.dP[k] @ xm, expect, atol=1e-12 * abs(S.dP[k]).max())
        np.testing.assert_allclose(C @ xm, M @ ubar[m_], atol=1e-12 * abs(C).max() * np.abs(ubar).max())
    # periodic directions: column sums of dP^k vanish
    per = {"unit_square_7": [], "periodic_square_6": [0, 1], "channel_9x9x7": [0, 2],
           "channel_9x9x7_disp3": [0, 2]}[mesh.name]
    for k in per:
        assert np.abs(one @ S.dP[k]).max() <= 1e-12 * abs(S.dP[k]).max()
    # Alg. 2 intermediate: A_rhs = M/dt - C/2 - nu K/2 maps 1 to M_L/dt
    Arhs = M / S.dt - 0.5 * C - 0.5 * S.nu * K
    np.testing.assert_allclose(Arhs @ one, S.ML / S.dt, rtol=1e-11)


def test_channel_pattern_counts():
    m = synth.channel(9, 9, 7)
    rp, ci = graph.csr_pattern(m)
    n_wall = m.bc_dofs.size
    assert rp[-1] == 15 * m.n_dof - 4 * n_wall
    S = ipcs.setup(m, 1.0, 1.0, np.zeros(3))
    M = S.M
    assert M.nnz == rp[-1]
    np.testing.assert_array_equal(M.indptr, rp)
    np.testing.assert_array_equal(M.indices, ci)
    # full-size counts quoted for the 129x129x97 workload
    nx, ny, nz = synth.CHANNEL_SIZES["c129"]
    N = (nx - 1) * ny * (nz - 1)
    assert N == 1_585_152
    assert 15 * N - 4 * 2 * (nx - 1) * (nz - 1) == 23_678_976
    assert 6 * (nx - 1) * (ny - 1) * (nz - 1) == 9_437_184


def test_channel_volume_and_stretching():
    m = synth.channel(17, 17, 13)
    assert math.isclose(m.volume, 32 * math.pi ** 2 / 3, rel_tol=1e-14)
    ys = np.unique(m.coords[:, 1])
    eta = -1 + 2 * np.arange(17) / 16
    np.testing.assert_allclose(ys, np.tanh(2 * eta) / np.tanh(2.0), atol=1e-15)
