"""Pins for the oracle's full time step.

* The paper's printed Taylor-Green errors (Sec. 6.1, Table 1, P1P1 rows) are
  reproduced from the golden fixture.  Reading of the paper's ||.||_h: the
  root mean square of the nodal errors over all nodes (and over both velocity
  components), pressure compared at t^n - dt/2 after removing means.
* The Dirichlet Taylor-Green workload on [0,1]^2 converges at rate ~2.
* Alg. 2 equals the naive per-cell quadrature reassembly.
* Laminar Poiseuille flow is a discrete steady state of the structured channel.
* The corrected velocity satisfies the discrete divergence identity of the
  lumped P1-P1 projection, and the global divergence vanishes in the channel.
"""
import os

import numpy as np
import pytest

import synth
from oracle import ipcs, naive, norms

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tg_p1p1_table1.txt")


def _table1():
    rows = []
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            n, h, eu, ku, ep, kp = line.split()
            rows.append((int(n), float(h), float(eu), float(ep)))
    return rows


def _tg_rms_errors(n, T=1.0, dt=1e-3):
    pr = synth.taylor_green(n, periodic=True, dt=dt, rtol=1e-12)
    S, st, _ = ipcs.run(pr, int(round(T / dt)))
    X, Y = pr.mesh.dof_coords[:, 0], pr.mesh.dof_coords[:, 1]
    du = st.U1 - synth.tg_exact_velocity(X, Y, st.t, pr.nu)
    pe = synth.tg_exact_pressure(X, Y, st.t - 0.5 * dt, pr.nu)
    dp = (st.p - st.p.mean()) - (pe - pe.mean())
    return float(np.sqrt(np.mean(du ** 2))), float(np.sqrt(np.mean(dp ** 2)))


@pytest.mark.parametrize("row", _table1(), ids=lambda r: "N%d" % r[0])
def test_taylor_green_table1(row):
    n, h, eu_paper, ep_paper = row
    assert abs(h - 2.0 / n * np.sqrt(2.0)) < 0.005 * h      # h = 2 x circumradius
    eu, ep = _tg_rms_errors(n)
    assert abs(eu / eu_paper - 1.0) < 0.01, (eu, eu_paper)
    assert abs(ep / ep_paper - 1.0) < 0.02, (ep, ep_paper)


def test_dirichlet_taylor_green_rate():
    """The [0,1]^2 workload with exact boundary velocity: L2 rate ~2 at t = 0.1."""
    errs = []
    hs = []
    for n in (8, 16, 32):
        pr = synth.taylor_green(n, periodic=False, rtol=1e-12)
        S, st, _ = ipcs.run(pr, 100)
        ex = [lambda x, k=k: synth.tg_exact_velocity(x[..., 0], x[..., 1], st.t, pr.nu)[k] for k in range(2)]
        errs.append(norms.vector_l2_error(pr.mesh, st.U1, ex))
        hs.append(1.0 / n)
    rates = [np.log(errs[i + 1] / errs[i]) / np.log(hs[i + 1] / hs[i]) for i in range(2)]
    assert all(1.8 <= k <= 2.2 for k in rates), rates


@pytest.mark.parametrize("prob", [synth.taylor_green(7), synth.channel_flow("tiny", displace_seed=4)],
                         ids=lambda p: p.name)
def test_alg2_equals_naive_reassembly(prob):
    m = prob.mesh
    S = ipcs.setup(m, prob.nu, prob.dt, prob.f)
    st = ipcs.initial_state(prob)
    rng = np.random.default_rng(2)
    st.U2 = st.U2 + 0.1 * rng.normal(size=st.U2.shape)
    st.p = rng.normal(size=m.n_dof)
    g = prob.bc_values(prob.t0 + prob.dt)
    A, b = ipcs.tentative_system(S, st, prob.t0 + prob.dt, g)
    for k in range(m.dim):
        An, bn = naive.tentative_system(m, prob.nu, prob.dt, prob.f, st.U1, st.U2, st.p, k)
        An = ipcs.apply_dirichlet_rows(An, m.bc_dofs)
        bn[m.bc_dofs] = g[k]
        assert abs(A - An).max() <= 1e-13 * abs(A).max()
        assert np.abs(b[k] - bn).max() <= 1e-13 * np.abs(b[k]).max()


@pytest.mark.parametrize("size", ["tiny", "small"])
def test_poiseuille_is_steady(size):
    pr = synth.channel_flow(size, noise=0.0)
    y = pr.mesh.dof_coords[:, 1]
    U = np.zeros((3, pr.mesh.n_dof))
    U[0] = (1.0 - y ** 2) / (2.0 * pr.nu)
    pr.U1, pr.U2 = U.copy(), U.copy()
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13)
    assert np.abs(out.state.U1 - U).max() <= 1e-12 * U.max()
    assert np.abs(out.phi).max() <= 1e-9


def test_divergence_identity_and_reduction():
    pr = synth.channel_flow("small", seed=1)
    m = pr.mesh
    S = ipcs.setup(m, pr.nu, pr.dt, pr.f)
    out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-13, rtol_p=1e-13)
    div = lambda U: sum(S.dP[k] @ U[k] for k in range(3))  # noqa: E731
    phi = out.phi
    mask = np.ones(m.n_dof)
    mask[m.bc_dofs] = 0.0
    op = S.K @ phi + sum(S.dP[k] @ (mask * (S.dP[k] @ phi) / S.ML) for k in range(3))
    lhs = div(out.state.U1)
    rhs = -pr.dt * op
    c = np.mean(lhs - rhs)          # the projected-out constant of b_phi
    assert np.linalg.norm(lhs - rhs - c) <= 1e-8 * np.linalg.norm(lhs)
    # global conservation in the periodic channel
    assert abs(lhs.sum()) <= 1e-11 * np.abs(lhs).sum()
    assert np.linalg.norm(lhs) < np.linalg.norm(div(out.UI))


def test_divergence_reduction_improves_under_refinement():
    """For a smooth divergent field ||D U^n|| / ||D U^I|| falls under refinement."""
    ratios = []
    for size in ["tiny", "small", (33, 33, 25)]:
        pr = synth.channel_flow(size, noise=0.0)
        m = pr.mesh
        x, y, z = m.dof_coords.T
        U = np.zeros((3, m.n_dof))
        U[0] = (1 - y ** 2) * (1 + 0.3 * np.sin(x / 2) * np.cos(1.5 * z))
        U[1] = 0.2 * (1 - y ** 2) * np.sin(x / 2)
        U[:, m.bc_dofs] = 0.0
        pr.U1, pr.U2 = U, U.copy()
        S = ipcs.setup(m, pr.nu, pr.dt, pr.f)
        out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-12, rtol_p=1e-12)
        div = lambda V: sum(S.dP[k] @ V[k] for k in range(3))  # noqa: E731
        ratios.append(np.linalg.norm(div(out.state.U1)) / np.linalg.norm(div(out.UI)))
    assert ratios[0] < 0.5 and ratios[1] < ratios[0] / 2 and ratios[2] < ratios[1] / 2, ratios


def test_step_outputs_have_zero_mean_pressure():
    pr = synth.channel_flow("tiny", seed=3)
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    st = ipcs.initial_state(pr)
    for _ in range(3):
        out = ipcs.step(S, st, pr.bc_values)
        st = out.state
        assert abs(st.p.mean()) < 1e-12 * (1 + np.abs(st.p).max())
        assert abs(out.phi.mean()) < 1e-12 * (1 + np.abs(out.phi).max())
        assert out.status == 0
        assert np.all(st.U1[:, pr.mesh.bc_dofs] == 0.0)


def test_pressure_start_changes_only_the_iterate():
    """phi_prev and phi_0 = 0 starts reach the same correction within the
    solver tolerance (the stopping test is relative to ||b_phi||, not to
    the initial residual), and a guess equal to phi_prev is the prev start."""
    prob = synth.channel_flow((9, 9, 7), seed=3)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    st = ipcs.step(S, ipcs.initial_state(prob), prob.bc_values, rtol_u=1e-12, rtol_p=1e-12).state
    assert np.linalg.norm(st.phi_prev) > 0
    a = ipcs.step(S, st, prob.bc_values, rtol_u=1e-12, rtol_p=1e-12, pressure_start="prev")
    b = ipcs.step(S, st, prob.bc_values, rtol_u=1e-12, rtol_p=1e-12, pressure_start="zero")
    c = ipcs.step(S, st, prob.bc_values, rtol_u=1e-12, rtol_p=1e-12, phi_guess=st.phi_prev)
    assert np.linalg.norm(a.phi - b.phi) <= 1e-8 * np.linalg.norm(a.phi)
    np.testing.assert_array_equal(a.phi, c.phi)
    assert a.iters_p == c.iters_p
    with pytest.raises(ValueError):
        ipcs.step(S, st, prob.bc_values, pressure_start="other")
