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
  as the tentative u_x when p* = 0.
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


@pytest.mark.parametrize("update", ["lumped", "consistent"])
@pytest.mark.parametrize("inner", [1, 3])
def test_poiseuille_steady_with_options(update, inner):
    pr, U = _poiseuille("tiny")
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13, inner_iters=inner,
                    update=update)
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
