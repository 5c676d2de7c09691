"""Pins for the oracle's Krylov loops: direct solves, pseudo-inverse on the
singular pressure matrix, CG energy-norm monotonicity, finite termination,
and the failure paths (not converged, breakdown, NaN)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import ipcs, krylov, mixed


def _tent(problem):
    S = ipcs.setup(problem.mesh, problem.nu, problem.dt, problem.f)
    st = ipcs.initial_state(problem)
    A, b = ipcs.tentative_system(S, st, problem.t0 + problem.dt, problem.bc_values(problem.dt))
    return S, st, A, b


@pytest.mark.parametrize("prob", [synth.taylor_green(16), synth.channel_flow("tiny", displace_seed=1)],
                         ids=lambda p: p.name)
def test_bicgstab_matches_direct_solve(prob):
    S, st, A, b = _tent(prob)
    A = A.tocsc()
    for k in range(prob.mesh.dim):
        x_ref = spla.spsolve(A, b[k])
        r = krylov.bicgstab(A.tocsr(), b[k], st.U1[k], rtol=1e-12)
        assert r.status == krylov.OK
        assert r.rel_res <= 1e-12
        kappa = np.linalg.cond(A.toarray())
        assert np.linalg.norm(r.x - x_ref) <= 10 * kappa * 1e-12 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("prob", [synth.taylor_green(12), synth.channel_flow("tiny")], ids=lambda p: p.name)
def test_pcg_singular_pressure_matches_pseudoinverse(prob):
    S, st, A, b = _tent(prob)
    K = S.K
    rng = np.random.default_rng(3)
    bphi = rng.normal(size=K.shape[0])
    bphi -= bphi.mean()
    r = krylov.pcg(K, bphi, np.zeros_like(bphi), rtol=1e-13)
    assert r.status == krylov.OK
    x = r.x - r.x.mean()
    x_ref = np.linalg.lstsq(K.toarray(), bphi, rcond=None)[0]
    x_ref -= x_ref.mean()
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_pcg_energy_error_monotone_and_finite_termination():
    rng = np.random.default_rng(5)
    n = 24
    Q = rng.normal(size=(n, n))
    A = sp.csr_matrix(Q @ Q.T + n * np.eye(n))
    xs = rng.normal(size=n)
    b = A @ xs
    errs = []
    x = np.zeros(n)
    for it in range(1, n + 1):
        r = krylov.pcg(A, b, x * 0, rtol=1e-30, maxit=it)
        e = r.x - xs
        errs.append(float(e @ (A @ e)))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    r = krylov.pcg(A, b, np.zeros(n), rtol=1e-12, maxit=3 * n)
    assert r.status == krylov.OK and r.iters <= n + 5


def test_failure_paths():
    A = sp.csr_matrix(np.array([[4.0, 1.0], [1.0, 3.0]]))
    b = np.array([1.0, 2.0])
    r = krylov.pcg(A, b, np.zeros(2), rtol=1e-14, maxit=1)
    assert r.status == krylov.NOTCONV and r.iters == 1
    r = krylov.bicgstab(A, b, np.zeros(2), rtol=1e-14, maxit=1)
    assert r.status == krylov.NOTCONV
    # indefinite matrix with positive diagonal: p^T A p < 0 stops CG
    Ai = sp.csr_matrix(np.array([[1.0, 2.0], [2.0, 1.0]]))
    r = krylov.pcg(Ai, np.array([1.0, -1.0]), np.zeros(2), rtol=1e-12)
    assert r.status == krylov.BREAKDOWN
    # (r_hat, D^{-1} A r_hat) = 0 twice: BiCGStab breakdown after one restart
    Ab = sp.csr_matrix(np.array([[1.0, -2.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    r = krylov.bicgstab(Ab, np.array([1.0, 1.0, 0.0]), np.zeros(3), rtol=1e-12)
    assert r.status == krylov.BREAKDOWN
    bn = b.copy()
    bn[0] = np.nan
    assert krylov.pcg(A, bn, np.zeros(2)).status == krylov.NAN
    assert krylov.bicgstab(A, bn, np.zeros(2)).status == krylov.NAN


def test_mixed_refinement_reaches_fp64_tolerance():
    prob = synth.channel_flow("small")
    S, st, A, b = _tent(prob)
    rng = np.random.default_rng(9)
    bphi = rng.normal(size=S.K.shape[0])
    bphi -= bphi.mean()
    ref = krylov.pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-12)
    r = mixed.refine("cg", S.K, bphi, np.zeros_like(bphi), rtol=1e-8, inner_rtol=1e-4)
    assert r.status == krylov.OK and r.rel_res <= 1e-8
    assert len(r.history) >= 2          # more than one refinement step was needed
    rel = np.linalg.norm((r.x - r.x.mean()) - (ref.x - ref.x.mean())) / np.linalg.norm(ref.x - ref.x.mean())
    assert rel < 1e-5
    rb = mixed.refine("bicgstab", A, b[0], st.U1[0], rtol=1e-10, inner_rtol=1e-4)
    assert rb.status == krylov.OK and rb.rel_res <= 1e-10


def test_reliable_pcg_in_fp64_is_plain_pcg():
    """With FP64 recurrences the residual replacements change r only by
    rounding and keep the direction, so the iteration is Jacobi-PCG: the
    same iteration count (within one) and the same answer.  A restart of the
    direction at a replacement, or a wrong beta, costs many iterations."""
    prob = synth.channel_flow("small")
    S, st, A, b = _tent(prob)
    rng = np.random.default_rng(21)
    bphi = rng.normal(size=S.K.shape[0])
    bphi -= bphi.mean()
    x0 = rng.normal(size=bphi.size) * 0.1
    ref = krylov.pcg(S.K, bphi, x0, rtol=1e-8)
    r = mixed.reliable_pcg(S.K, bphi, x0, rtol=1e-8, delta=0.1, inner_dtype=np.float64)
    assert r.status == krylov.OK and r.rel_res <= 1e-8
    assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    assert len(r.history) >= 7                       # one replacement per decade of 1e-8
    assert np.linalg.norm(r.x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_reliable_pcg_fp32_reaches_fp64_tolerance():
    prob = synth.channel_flow("small")
    S, st, A, b = _tent(prob)
    rng = np.random.default_rng(22)
    bphi = rng.normal(size=S.K.shape[0])
    bphi -= bphi.mean()
    ref = krylov.pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-12)
    r64 = krylov.pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-8)
    r = mixed.reliable_pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-8)
    assert r.status == krylov.OK
    assert np.linalg.norm(bphi - S.K @ r.x) <= 1e-8 * np.linalg.norm(bphi)
    assert r.iters <= 1.3 * r64.iters, (r.iters, r64.iters)
    rel = np.linalg.norm((r.x - r.x.mean()) - (ref.x - ref.x.mean())) / np.linalg.norm(ref.x - ref.x.mean())
    assert rel < 1e-5
    # FP32 recurrences alone stall: without replacements the true residual
    # cannot reach 1e-8 even though the recursive one does
    rs = mixed.reliable_pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-8, delta=0.0, maxit=3 * r64.iters)
    assert rs.status == krylov.NOTCONV and rs.rel_res > 1e-7


def test_bicgstab_right_jacobi_is_plain_bicgstab_on_column_scaled_matrix():
    """Right Jacobi preconditioning means BiCGStab on A D^{-1} in y = D x:
    running the unpreconditioned method (diag = 1) on the explicitly
    column-scaled matrix must give the same iterations and, after x = y/d,
    the same solution.  Left preconditioning (D^{-1} A) fails this."""
    prob = synth.channel_flow("small", seed=5)
    S, st, A, b = _tent(prob)
    d = A.diagonal()
    Ac = (A @ sp.diags(1.0 / d)).tocsr()
    for k in range(3):
        r1 = krylov.bicgstab(A, b[k], st.U1[k], rtol=1e-10)
        r2 = krylov.bicgstab(Ac, b[k], d * st.U1[k], rtol=1e-10, diag=np.ones_like(d))
        assert r1.status == krylov.OK and r2.status == krylov.OK
        assert r1.iters == r2.iters
        assert np.linalg.norm(r1.x - r2.x / d) <= 1e-9 * np.linalg.norm(r1.x)
    Al = (sp.diags(1.0 / d) @ A).tocsr()
    x_left = krylov.bicgstab(Al, b[0] / d, st.U1[0], rtol=1e-10, maxit=3, diag=np.ones_like(d)).x
    x_right = krylov.bicgstab(A, b[0], st.U1[0], rtol=1e-10, maxit=3).x
    assert np.linalg.norm(x_left - x_right) > 1e-6 * np.linalg.norm(x_right)
