"""Pins of the oracle's options beyond the channel runs' configuration
(oracle/ipcs.py): Alg. 1's inner velocity-pressure iterations, the
consistent-mass velocity update (eq:velocity_update) and passive scalars
(eq:scalar_disc), against what the mathematics fixes:

* consistent update: the symmetric elimination of the Dirichlet dofs solved
  by CG equals a direct solve of the identity-row system (the reading's
  other form), with non-zero Dirichlet values (Taylor-Green);
* Poiseuille flow stays a discrete steady state with either update and any
  number of inner iterations;
* the inner iterations form a contracting fixed-point iteration: every
  pressure correction is smaller than the one before, the second less than
  half the first;
* a scalar that is constant, or linear across the channel under a flow
  along it, is a discrete steady state; a scalar with D = nu, source f_x,
  the same start and Dirichlet values as u_x solves the same linear system
  as the tentative u_x when p* = 0;
* the explicit Adams-Bashforth convection (eq:convection_ABE) and the ABCN
  form are two second-order discretisations of the same term, so their
  solutions differ by O(dt^2): halving dt divides the difference of both
  velocity and pressure by ~4 (periodic Taylor-Green).  A first-order
  convection (one explicit term at t^{n-1}) gives ~2 on the pressure, a
  wrong sign or weight a difference that does not vanish;
* the weighted gradient matrix G^k (read as the volume-weighted nodal
  average of cellwise gradients) equals that average computed cell by cell
  from the vertex coordinates, is exact for linear fields, and its update
  equals the lumped one.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import ipcs


def _poiseuille(size):
    pr = synth.channel_flow(size, noise=0.0)
    y = pr.mesh.dof_coords[:, 1]
    U = np.zeros((3, pr.mesh.n_dof))
    U[0] = (1.0 - y ** 2) / (2.0 * pr.nu)
    pr.U1, pr.U2 = U.copy(), U.copy()
    return pr, U


def test_consistent_update_equals_identity_row_direct_solve():
    pr = synth.taylor_green(8)
    m = pr.mesh
    S = ipcs.setup(m, pr.nu, pr.dt, pr.f)
    st = ipcs.initial_state(pr)
    out = ipcs.step(S, st, pr.bc_values, rtol_u=1e-14, rtol_p=1e-13, update="consistent")
    g = pr.bc_values(st.t + pr.dt)
    Mid = ipcs.apply_dirichlet_rows(S.M, m.bc_dofs)
    for k in range(2):
        rhs = S.M @ out.UI[k] - pr.dt * (S.dP[k] @ out.phi)
        rhs[m.bc_dofs] = g[k]
        ref = spla.spsolve(Mid.tocsc(), rhs)
        assert np.abs(out.state.U1[k] - ref).max() <= 1e-12 * np.abs(ref).max(), k
    assert all(i > 0 for i in out.iters_m)
    # and it differs from the lumped update by more than the tolerance
    lumped = ipcs.step(S, st, pr.bc_values, rtol_u=1e-14, rtol_p=1e-13)
    assert np.abs(lumped.state.U1 - out.state.U1).max() > 1e-9


@pytest.mark.parametrize("convection", ["abcn", "abe"])
@pytest.mark.parametrize("update", ["lumped", "consistent", "gradient"])
@pytest.mark.parametrize("inner", [1, 3])
def test_poiseuille_steady_with_options(update, inner, convection):
    pr, U = _poiseuille("tiny")
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, inner_iters=inner,
                    update=update, convection=convection)
    assert np.abs(out.state.U1 - U).max() <= 1e-12 * U.max()
    assert len(out.phis) == inner and all(np.abs(f).max() <= 1e-9 for f in out.phis)


@pytest.mark.parametrize("prob", [synth.taylor_green(16), synth.channel_flow("tiny", seed=3)],
                         ids=lambda p: p.name)
def test_inner_iterations_contract(prob):
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    out = ipcs.step(S, ipcs.initial_state(prob), prob.bc_values, rtol_u=1e-13, rtol_p=1e-13, inner_iters=4)
    norms = [np.linalg.norm(f) for f in out.phis]
    # monotone, with most of the correction in the first iteration (the
    # fixed point's contraction then slows: 0.7-0.95 per iteration here)
    assert all(b < a for a, b in zip(norms, norms[1:])), norms
    assert norms[1] < 0.5 * norms[0], norms
    # one inner iteration is the plain step, value for value
    one = ipcs.step(S, ipcs.initial_state(prob), prob.bc_values, rtol_u=1e-13, rtol_p=1e-13, inner_iters=1)
    assert np.array_equal(one.phis[0], out.phis[0])


def test_scalar_constant_and_linear_profiles_are_steady():
    pr, U = _poiseuille("small")
    m = pr.mesh
    y = m.dof_coords[:, 1]
    yb = y[m.bc_dofs]
    S = ipcs.setup(m, pr.nu, pr.dt, pr.f)
    scal = [ipcs.Scalar(D=0.3, bc=lambda t: np.full(yb.size, 2.5)),
            ipcs.Scalar(D=0.01, bc=lambda t: yb.copy())]
    C1 = np.stack([np.full(m.n_dof, 2.5), y.copy()])
    out = ipcs.step(S, ipcs.initial_state(pr, C1), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, scalars=scal)
    assert np.abs(out.state.C1[0] - 2.5).max() <= 1e-12
    assert np.abs(out.state.C1[1] - y).max() <= 1e-12
    assert len(out.iters_c) == 2


def test_scalar_with_viscosity_solves_the_tentative_system():
    pr = synth.channel_flow("small", seed=2)
    m = pr.mesh
    S = ipcs.setup(m, pr.nu, pr.dt, pr.f)
    st = ipcs.initial_state(pr, pr.U1[:1].copy())          # p* = 0 at the start of the channel run
    sc = ipcs.Scalar(D=pr.nu, f=pr.f[0], bc=lambda t: np.zeros(m.bc_dofs.size))
    out = ipcs.step(S, st, pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, scalars=[sc])
    assert np.abs(out.state.C1[0] - out.UI[0]).max() <= 1e-10 * np.abs(out.UI[0]).max()
    # a different diffusivity gives a different field
    sc2 = ipcs.Scalar(D=3 * pr.nu, f=pr.f[0], bc=sc.bc)
    out2 = ipcs.step(S, st, pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, scalars=[sc2])
    assert np.abs(out2.state.C1[0] - out.UI[0]).max() > 1e-6 * np.abs(out.UI[0]).max()


def _run_tg(convection, dt, T=0.4):
    pr = synth.taylor_green(12, periodic=True, nu=0.01, dt=dt)
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    st = ipcs.initial_state(pr)
    for _ in range(int(round(T / dt))):
        st = ipcs.step(S, st, pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, convection=convection).state
    return st


def test_abe_and_abcn_convection_agree_to_second_order():
    du, dp = [], []
    for dt in (0.04, 0.02, 0.01):
        a, b = _run_tg("abe", dt), _run_tg("abcn", dt)
        du.append(np.linalg.norm(a.U1 - b.U1) / np.linalg.norm(b.U1))
        dp.append(np.linalg.norm(a.p - b.p) / np.linalg.norm(b.p))
    for d in (du, dp):
        ratios = [d[i] / d[i + 1] for i in range(2)]
        assert all(3.3 <= r <= 4.7 for r in ratios), (du, dp)
    assert 0 < du[-1] < 1e-4


def test_abe_system_is_constant_and_symmetric():
    pr = synth.channel_flow("tiny", seed=5)
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    st = ipcs.initial_state(pr)
    g = pr.bc_values(pr.dt)
    A1, _ = ipcs.tentative_system(S, st, pr.dt, g, convection="abe")
    st.U1 = st.U1 + 0.3
    A2, b2 = ipcs.tentative_system(S, st, pr.dt, g, convection="abe")
    assert (A1 - A2).count_nonzero() == 0             # no convection in the matrix
    keep = np.ones(pr.mesh.n_dof, bool)
    keep[pr.mesh.bc_dofs] = False
    Ai = A2[keep][:, keep]
    assert abs(Ai - Ai.T).max() <= 1e-15 * abs(Ai).max()


def _cell_gradient_average(mesh, q):
    """sum_T |T| grad(q)|_T / sum_T |T| per dof, one cell at a time."""
    d = mesh.dim
    num = np.zeros((mesh.n_dof, d))
    den = np.zeros(mesh.n_dof)
    for cell in mesh.cells:
        X = mesh.coords[cell]
        dofs = mesh.vert2dof[cell]
        E = (X[1:] - X[0]).T                           # columns x_i - x_0
        vol = abs(np.linalg.det(E)) / (2.0 if d == 2 else 6.0)
        grad = np.linalg.solve(E.T, q[dofs[1:]] - q[dofs[0]])
        for v in dofs:
            num[v] += vol * grad
            den[v] += vol
    return num / den[:, None]


@pytest.mark.parametrize("mesh", [synth.unit_square(6), synth.channel(5, 5, 4, displace_seed=3)],
                         ids=lambda m: m.name)
def test_gradient_matrix_is_the_volume_weighted_cell_gradient(mesh):
    S = ipcs.setup(mesh, 0.01, 0.01, np.zeros(mesh.dim))
    G = ipcs.gradient_update_matrices(S)
    q = np.random.default_rng(7).standard_normal(mesh.n_dof)
    ref = _cell_gradient_average(mesh, q)
    for k in range(mesh.dim):
        assert np.abs(G[k] @ q - ref[:, k]).max() <= 1e-12 * np.abs(ref).max(), k
    if mesh.dim == 2:                                  # no periodic identification: linear fields are exact
        c = np.array([0.7, -1.3])
        lin = mesh.dof_coords @ c + 2.0
        for k in range(2):
            assert np.abs(G[k] @ lin - c[k]).max() <= 1e-12


def test_gradient_update_equals_lumped_update():
    pr = synth.channel_flow("tiny", seed=1)
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    a = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, update="gradient")
    b = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, update="lumped")
    assert np.abs(a.state.U1 - b.state.U1).max() <= 1e-13 * np.abs(b.state.U1).max()
