"""Pins of the smoothed-aggregation oracle (oracle/amg.py) against what the
method and the mathematics fix independently of the code:

* strength of connection on an anisotropic 5-point Laplacian, where the
  strong couplings are known in closed form;
* the greedy aggregation of a path graph, whose aggregates are known in
  closed form, and the invariants of any aggregation (a partition into
  connected pieces of the strong graph);
* the tentative prolongator's orthonormal columns and exact reproduction
  of the near-null vector, and the energy decrease of prolongator smoothing;
* the Galerkin coarse operator's symmetry, semi-definiteness and null
  vector;
* the V-cycle as a symmetric positive definite preconditioner with a
  two-grid-like contraction on the 2D Poisson problem, and AMG-PCG
  reaching the tolerance with the solution of a direct solve;
* the regularised coarsest solve against the pseudo-inverse.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg, ipcs, krylov


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def lap2d(n, eps=1.0):
    """eps u_xx + u_yy, 5-point, Dirichlet, n x n interior nodes, x fastest."""
    I = sp.identity(n)
    return (eps * sp.kron(I, lap1d(n)) + sp.kron(lap1d(n), I)).tocsr()


def test_strength_on_anisotropic_laplacian():
    n = 6
    A = lap2d(n, eps=0.01)
    S = amg.strength(A, 0.25)
    # a_ij = -eps for x-neighbours, -1 for y-neighbours, a_ii = 2 + 2 eps:
    # only the y-neighbours pass |a_ij| >= 0.25 a_ii
    for i in range(n * n):
        strong = set(S.indices[S.indptr[i]:S.indptr[i + 1]][S.data[S.indptr[i]:S.indptr[i + 1]]])
        expect = {j for j in (i - n, i + n) if 0 <= j < n * n}
        assert strong == expect, (i, strong, expect)


def test_aggregation_of_a_path_is_known():
    n = 10
    A = lap1d(n)
    agg, na = amg.aggregate(A, amg.strength(A, 0.25))
    # pass (a) in index order takes {0,1}, {2,3,4}, {5,6,7}; node 8's left
    # neighbour is taken, node 9 starts {8, 9}
    assert na == 4
    assert list(agg) == [(i + 1) // 3 for i in range(n)]


@pytest.mark.parametrize("theta", [0.0, 0.25])
def test_aggregation_is_a_partition_into_connected_pieces(theta):
    pr = synth.channel_flow("tiny", seed=1)
    K = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f).K.tocsr()
    K.sort_indices()
    S = amg.strength(K, theta)
    agg, na = amg.aggregate(K, S)
    assert agg.min() == 0 and agg.max() == na - 1 and np.unique(agg).size == na
    G = sp.csr_matrix((S.data.astype(float), S.indices, S.indptr), shape=K.shape)
    for a in range(na):
        idx = np.flatnonzero(agg == a)
        sub = G[idx][:, idx]
        ncomp, _ = sp.csgraph.connected_components(sub + sub.T, directed=False)
        assert ncomp == 1, (a, idx)


def test_tentative_prolongator_orthonormal_and_exact_on_b():
    rng = np.random.default_rng(0)
    agg = rng.integers(0, 7, size=40)
    agg[:7] = np.arange(7)
    B = rng.uniform(0.5, 2.0, size=40)
    P, Bc = amg.tentative(agg, 7, B)
    np.testing.assert_allclose((P.T @ P).toarray(), np.eye(7), atol=1e-14)
    np.testing.assert_allclose(P @ Bc, B, rtol=1e-14)


def _channel_scaled(size="small"):
    pr = synth.channel_flow(size, seed=1)
    K = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f).K.tocsr()
    s = np.sqrt(K.diagonal())
    Ks = sp.csr_matrix(sp.diags(1 / s) @ K @ sp.diags(1 / s))
    Ks.sort_indices()
    return Ks, s


def test_smoothing_lowers_the_prolongator_energy_and_keeps_the_null_vector():
    Ks, s = _channel_scaled("tiny")
    S = amg.strength(Ks, 0.25)
    agg, na = amg.aggregate(Ks, S)
    P, Bc, Pt = amg.smoothed_prolongator(Ks, S, s, agg, na)
    # one damped Jacobi step with omega rho <= 4/3 < 2 lowers every
    # column's energy (a wrong sign raises it)
    eP = np.asarray((P.multiply(Ks @ P)).sum(axis=0)).ravel()
    eT = np.asarray((Pt.multiply(Ks @ Pt)).sum(axis=0)).ravel()
    assert np.all(eP < eT)
    # Ks s = 0 and the filtered matrix keeps it: P reproduces s exactly
    np.testing.assert_allclose(P @ Bc, s, rtol=1e-12)


def test_coarse_operators_symmetric_semidefinite_with_null_vector():
    Ks, s = _channel_scaled("tiny")
    H = amg.hierarchy(Ks, B=s, coarse_size=40, singular=True)
    assert len(H.levels) >= 3
    for lv in H.levels[1:]:
        Ac = lv.A.toarray()
        np.testing.assert_allclose(Ac, Ac.T, atol=1e-13 * np.abs(Ac).max())
        ev = np.linalg.eigvalsh(Ac)
        assert ev[0] > -1e-12 * ev[-1]
        assert np.linalg.norm(Ac @ lv.B) <= 1e-12 * np.abs(Ac).max() * np.linalg.norm(lv.B)


@pytest.mark.parametrize("case", ["poisson2d", "channel", "displaced"])
def test_rho_estimate_lies_between_the_spectral_radius_and_gershgorin(case):
    """The damping estimate never under-estimates rho(D^{-1} A) (so omega rho
    stays <= 4/3 < 2), is never above the Gershgorin bound, and is a real
    improvement on it where the off-diagonals have both signs."""
    if case == "poisson2d":
        A = lap2d(20)
    else:
        pr = synth.channel_flow("small", seed=0, displace_seed=5 if case == "displaced" else None)
        A = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f).K
    A = sp.csr_matrix(A)
    d = A.diagonal()
    M = (sp.diags(1 / np.sqrt(d)) @ A @ sp.diags(1 / np.sqrt(d))).toarray()
    rho = np.linalg.eigvalsh(M)[-1]
    est, g = amg.rho_estimate(A), amg.gershgorin(A)
    assert rho <= est <= g + 1e-15, (rho, est, g)
    if case == "displaced":
        assert est < 0.9 * g, (rho, est, g)           # mixed-sign rows: a looser bound
    # 1.1 times a Rayleigh quotient of an iterate: at most 10% above rho
    assert est <= 1.1 * rho * (1 + 1e-12)


def _vcycle_matrix(H, n):
    return np.column_stack([amg.vcycle(H, e) for e in np.eye(n)])


def test_vcycle_is_spd_and_contracts_on_poisson_2d():
    A = lap2d(24)
    H = amg.hierarchy(A, coarse_size=30)
    assert len(H.levels) >= 3
    Minv = _vcycle_matrix(H, A.shape[0])
    np.testing.assert_allclose(Minv, Minv.T, atol=1e-12 * np.abs(Minv).max())
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T))[0] > 0
    # error propagation of one cycle, I - M^{-1} A: smoothed aggregation
    # V(1,1) contracts the Poisson error by a small factor at every size
    E = np.eye(A.shape[0]) - Minv @ A.toarray()
    rho = np.max(np.abs(np.linalg.eigvals(E)))
    assert rho < 0.6, rho            # 0.55 here; without prolongator smoothing 0.87


def test_coarse_solve_is_the_pseudo_inverse_on_range():
    Ks, s = _channel_scaled("tiny")
    H = amg.hierarchy(Ks, B=s, coarse_size=10 ** 6, singular=True)
    assert len(H.levels) == 1
    rng = np.random.default_rng(5)
    r = rng.normal(size=Ks.shape[0])
    r -= (r @ s) / (s @ s) * s                     # consistent right-hand side
    x = H.coarse_inv @ r
    ref = np.linalg.pinv(Ks.toarray()) @ r
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("size", ["tiny", "small"])
def test_amg_pcg_reaches_tolerance_with_few_iterations(size):
    Ks, s = _channel_scaled(size)
    rng = np.random.default_rng(2)
    b = rng.normal(size=Ks.shape[0])
    b -= (b @ s) / (s @ s) * s
    H = amg.hierarchy(Ks, B=s, coarse_size=100, singular=True)
    r = amg.amg_pcg(Ks, b, np.zeros_like(b), H, rtol=1e-10)
    assert r.status == krylov.OK and r.rel_res <= 1e-10
    assert np.linalg.norm(b - Ks @ r.x) <= 1e-10 * np.linalg.norm(b)
    j = krylov.pcg(Ks, b, np.zeros_like(b), rtol=1e-10)
    assert r.iters * 5 < j.iters, (r.iters, j.iters)
    # same solution as a direct solve, up to the null vector
    ref = np.linalg.lstsq(Ks.toarray(), b, rcond=None)[0] if Ks.shape[0] < 4000 else j.x
    d = r.x - ref
    d -= (d @ s) / (s @ s) * s
    assert np.linalg.norm(d) <= 1e-7 * np.linalg.norm(ref)
