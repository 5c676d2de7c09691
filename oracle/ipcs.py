"""One IPCS_ABCN time step in FP64, following the paper step by step.

Passages: the generic fractional-step loop (Alg. 1, one inner iteration),
the high-performance assembly of the coefficient matrix (Alg. 2 and its
implementation figure: assemble C into A, scale by -1/2, add M/dt and
-nu K/2, form the partial right-hand side with A U^{n-1}, reset A to
-A + 2M/dt, apply Dirichlet rows), the pressure-gradient matrices
(eq:dp_matrix), the algebraic pressure-correction equation with
dU^k = dP^k for equal spaces, and the lumped-mass velocity update
(Sec. 5, last paragraphs; the channel runs of Sec. 6.2 use lumping).

Readings (where the paper is silent or inconsistent):
* Pressure sign: K phi = -(1/dt) sum_k dP^k U^{k,I}.  This is the algebraic
  form of Sec. 5 and the only sign consistent with the correction
  u^n = u^I - dt grad(phi) (eq:correction) making u^n divergence free;
  eq:pressure and eq:pressureVF print the opposite sign.
* The velocity update subtracts dt * M_L^{-1} dP^k phi (the correction phi,
  as in eq:correction), not the full pressure.
* By default one inner iteration (plain IPCS) and the lumped-mass update.
* Dirichlet rows of A become identity rows (columns kept); b_i = g_i there.
  All velocity components share the Dirichlet dof set, so one A serves all.
* No pressure boundary condition: b_phi is projected onto 1-perp before the
  solve, phi and p are shifted to zero arithmetic mean of their dof values.
* Initial guesses (the paper does not fix them): U^{k,n-1} for the
  tentative velocity; for the pressure correction the previous correction
  phi_prev (pressure_start="prev").  pressure_start="zero" starts from
  phi_0 = 0, i.e. solving for p from p*, as the pressure-solve routine of
  the naive solver (Sec. 4) would with an iterative solver.  A caller
  guess (phi_guess) replaces either.

Options beyond the channel runs' configuration (Alg. 1 in general, Sec. 5's
other update types, eq:scalar_disc):
* inner_iters > 1: Alg. 1's inner velocity-pressure loop.  The coefficient
  matrix and b_tmp are built on the first inner iteration only (Sec. 5:
  the convecting velocity holds only known velocities); every inner
  iteration subtracts the gradient of the current p* (eq:dp_matrix),
  solves the tentative velocity (from U^{n-1} on the first iteration, from
  the previous U^I after), the pressure correction (from the plain start
  on the first iteration, from 0 after: it corrects the p* just updated),
  and sets p* = p* + phi.  The velocity update uses the last correction,
  which also becomes phi_prev.
* update="consistent": eq:velocity_update, M U^n = M U^I - dt dP^k phi,
  solved by Jacobi-PCG from U^I to rtol_u.  Dirichlet values are imposed by
  symmetric elimination (rows and columns of the Dirichlet dofs removed,
  their known values moved to the right-hand side), which has the same
  solution as identity rows and keeps the matrix SPD for CG.
* convection="abe": eq:convection_ABE in place of eq:convection_ABCN.  The
  convection is fully explicit, so the coefficient matrix is the constant
  M/dt + nu K/2 (Dirichlet rows as above) and the right-hand side carries
  it: b_tmp = f M_L + (M/dt - nu K/2) U^{n-1} - 1.5 C(u^{n-1}) U^{n-1}
  + 0.5 C(u^{n-2}) U^{n-2}, with C(w) the convection matrix of the
  convecting field w.  Scalars keep the u_bar form (the paper's scalar
  discretisation is that form for either velocity convection).
* update="gradient": the direct update with the weighted gradient matrix
  G^k of Sec. 5 (last paragraphs).  The paper does not define its weights;
  it is read as the nodal average of the cellwise constant gradient,
  weighted by cell volume: (G^k q)_i = sum_{T ni i} |T| d_k q|_T /
  sum_{T ni i} |T|.  For P1 elements int_T phi_i = |T|/(d+1) for every
  vertex of T, so G^k = M_L^{-1} dP^k (the rows of dP^k over the lumped
  mass), and U^n = U^I - dt G^k phi with the Dirichlet values.
* scalars: eq:scalar_disc with the convection term of the paper's scalar
  discretisation, u_bar . grad(c~) with the same Adams-Bashforth u_bar and
  Crank-Nicolson c~, i.e. the tentative-velocity system with nu replaced
  by D_alpha and no pressure gradient, assembled in Alg. 2's order:
  (M/dt + C/2 + D K/2) c^n = (M/dt - C/2 - D K/2) c^{n-1} + f_alpha M_L,
  solved after the velocity update (Alg. 1) by BiCGStab + Jacobi from
  c^{n-1}.  Dirichlet values on the velocity's Dirichlet dofs.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import krylov, p1


@dataclasses.dataclass
class Setup:
    mesh: object
    nu: float
    dt: float
    f: np.ndarray
    M: sp.csr_matrix
    K: sp.csr_matrix
    dP: list
    ML: np.ndarray
    b0: np.ndarray          # [d, N]
    geo: tuple


@dataclasses.dataclass
class State:
    U1: np.ndarray          # [d, N]  U^{n-1}
    U2: np.ndarray          # [d, N]  U^{n-2}
    p: np.ndarray           # [N]     p* (pressure from the last step)
    phi_prev: np.ndarray    # [N]
    t: float
    C1: np.ndarray | None = None   # [n_scalars, N] c^{n-1}


@dataclasses.dataclass
class Scalar:
    """A passive scalar of eq:scalar: diffusivity D, constant source f and
    its Dirichlet values bc(t) -> [n_bc] on the velocity's Dirichlet dofs."""
    D: float
    f: float = 0.0
    bc: object = None


@dataclasses.dataclass
class StepOut:
    state: State
    A: sp.csr_matrix        # tentative-velocity matrix after Dirichlet rows
    b: np.ndarray           # [d, N] tentative right-hand sides after Dirichlet values
    UI: np.ndarray          # [d, N] tentative velocity
    b_phi: np.ndarray       # [N] projected pressure right-hand side
    phi: np.ndarray         # [N] pressure correction (zero mean)
    iters_u: list
    iters_p: int
    res_u: list
    res_p: float
    status: int
    phis: list = dataclasses.field(default_factory=list)    # phi of every inner iteration
    iters_m: list = dataclasses.field(default_factory=list)  # consistent-update CG iterations
    iters_c: list = dataclasses.field(default_factory=list)  # scalar BiCGStab iterations


def setup(mesh, nu, dt, f):
    """Preassemble the constant matrices (Sec. 5: M, K once; dP^k once)."""
    geo = p1.element_geometry(mesh)
    M = p1.mass_matrix(mesh, geo)
    K = p1.stiffness_matrix(mesh, geo)
    dP = [p1.gradient_matrix(mesh, k, geo) for k in range(mesh.dim)]
    ML = np.asarray(M.sum(axis=1)).ravel()
    b0 = np.stack([f[k] * ML for k in range(mesh.dim)])
    return Setup(mesh, float(nu), float(dt), np.asarray(f, float), M, K, dP, ML, b0, geo)


def apply_dirichlet_rows(A, rows):
    """Replace the given rows of a CSR matrix by identity rows (in a copy)."""
    A = A.tocsr(copy=True)
    is_bc = np.zeros(A.shape[0], bool)
    is_bc[rows] = True
    row_of = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    m = is_bc[row_of]
    A.data[m] = 0.0
    A.data[m & (A.indices == row_of)] = 1.0
    return A


def tentative_system(S: Setup, st: State, t_new: float, bc_vals, with_tmp=False, convection="abcn"):
    """Alg. 2 literal: returns (A after BC rows, b [d, N] after BC values),
    and b_tmp with with_tmp.  convection="abe" builds the explicit form
    instead (tentative_system_abe)."""
    if convection == "abe":
        return tentative_system_abe(S, st, bc_vals, with_tmp)
    if convection != "abcn":
        raise ValueError(convection)
    mesh = S.mesh
    d = mesh.dim
    ubar = 1.5 * st.U1 - 0.5 * st.U2
    A = p1.convection_matrix(mesh, ubar, S.geo)          # A <- C
    A = -0.5 * A                                         # A._scale(-0.5)
    A = A + (1.0 / S.dt) * S.M                           # A.axpy(1/dt, M)
    A = A + (-0.5 * S.nu) * S.K                          # A.axpy(-nu/2, K)
    b_tmp = np.stack([S.b0[k] + A @ st.U1[k] for k in range(d)])
    A = -1.0 * A                                         # A._scale(-1)
    A = A + (2.0 / S.dt) * S.M                           # A.axpy(2/dt, M)
    A = apply_dirichlet_rows(A, mesh.bc_dofs)
    b = tentative_rhs(S, b_tmp, st.p, bc_vals)
    if with_tmp:
        return A.tocsr(), b, b_tmp
    return A.tocsr(), b


def tentative_system_abe(S: Setup, st: State, bc_vals, with_tmp=False):
    """eq:NStentative with eq:convection_ABE in matrix form:
    (M/dt + nu K/2) U^I = f M_L + (M/dt - nu K/2) U^{n-1}
                          - 1.5 C(u^{n-1}) U^{n-1} + 0.5 C(u^{n-2}) U^{n-2} - dP^k p*."""
    mesh = S.mesh
    d = mesh.dim
    C1 = p1.convection_matrix(mesh, st.U1, S.geo)        # C(u^{n-1})
    C2 = p1.convection_matrix(mesh, st.U2, S.geo)        # C(u^{n-2})
    R = (1.0 / S.dt) * S.M - (0.5 * S.nu) * S.K
    b_tmp = np.stack([S.b0[k] + R @ st.U1[k] - 1.5 * (C1 @ st.U1[k]) + 0.5 * (C2 @ st.U2[k])
                      for k in range(d)])
    A = (1.0 / S.dt) * S.M + (0.5 * S.nu) * S.K
    A = apply_dirichlet_rows(A, mesh.bc_dofs)
    b = tentative_rhs(S, b_tmp, st.p, bc_vals)
    if with_tmp:
        return A.tocsr(), b, b_tmp
    return A.tocsr(), b


def gradient_update_matrices(S: Setup):
    """G^k = M_L^{-1} dP^k (the volume-weighted nodal gradient, see the
    module notes)."""
    Li = sp.diags(1.0 / S.ML)
    return [(Li @ S.dP[k]).tocsr() for k in range(S.mesh.dim)]


def tentative_rhs(S: Setup, b_tmp, p_star, bc_vals):
    """b^k = b_tmp^k - dP^k p* with the Dirichlet values."""
    b = np.stack([b_tmp[k] - S.dP[k] @ p_star for k in range(S.mesh.dim)])
    if S.mesh.bc_dofs.size:
        b[:, S.mesh.bc_dofs] = bc_vals
    return b


def scalar_system(S: Setup, st: State, c1, sc: Scalar, bc_vals):
    """eq:scalar_disc assembled in Alg. 2's order with D in place of nu and
    the scalar's source: returns (A_c after Dirichlet rows, b_c)."""
    ubar = 1.5 * st.U1 - 0.5 * st.U2
    A = p1.convection_matrix(S.mesh, ubar, S.geo)        # A <- C(u_bar)
    A = -0.5 * A
    A = A + (1.0 / S.dt) * S.M
    A = A + (-0.5 * sc.D) * S.K
    b = sc.f * S.ML + A @ c1
    A = -1.0 * A
    A = A + (2.0 / S.dt) * S.M
    A = apply_dirichlet_rows(A, S.mesh.bc_dofs)
    if S.mesh.bc_dofs.size:
        b[S.mesh.bc_dofs] = bc_vals
    return A.tocsr(), b


def consistent_update(S: Setup, UI, phi, g, rtol, maxit):
    """eq:velocity_update by Jacobi-PCG with the Dirichlet dofs eliminated
    symmetrically; returns (U^n [d, N], iterations per component)."""
    mesh = S.mesh
    n = mesh.n_dof
    bc = mesh.bc_dofs
    keep = np.ones(n)
    keep[bc] = 0.0
    Kp = sp.diags(keep)
    Mbc = (Kp @ S.M @ Kp + sp.diags(1.0 - keep)).tocsr()
    Un = np.empty_like(UI)
    its = []
    for k in range(mesh.dim):
        rhs = S.M @ UI[k] - S.dt * (S.dP[k] @ phi)
        if bc.size:
            gk = np.zeros(n)
            gk[bc] = g[k]
            rhs = keep * (rhs - S.M @ gk) + gk
        x0 = UI[k].copy()
        if bc.size:
            x0[bc] = g[k]
        r = krylov.pcg(Mbc, rhs, x0, rtol=rtol, maxit=maxit)
        Un[k] = r.x
        its.append(r.iters)
    if bc.size:
        Un[:, bc] = g
    return Un, its


def pressure_rhs(S: Setup, UI):
    b_phi = -(1.0 / S.dt) * sum(S.dP[k] @ UI[k] for k in range(S.mesh.dim))
    return b_phi - b_phi.mean()


def step(S: Setup, st: State, bc_values, rtol_u=1e-8, rtol_p=1e-8, maxit=10000,
         phi_guess=None, pressure_start="prev", inner_iters=1, update="lumped", scalars=(),
         convection="abcn") -> StepOut:
    """Advance one time step (Alg. 1).  bc_values: callable t -> [d, n_bc]."""
    mesh = S.mesh
    d = mesh.dim
    t_new = st.t + S.dt
    g = bc_values(t_new) if mesh.bc_dofs.size else np.zeros((d, 0))
    A, b, b_tmp = tentative_system(S, st, t_new, g, with_tmp=True, convection=convection)
    UI = st.U1.copy()
    iters_u, res_u = [0] * d, [0.0] * d
    iters_p, res_p, status = 0, 0.0, 0
    p_star = st.p
    phis = []
    for i in range(inner_iters):
        if i > 0:
            b = tentative_rhs(S, b_tmp, p_star, g)
        for k in range(d):
            r = krylov.bicgstab(A, b[k], UI[k], rtol=rtol_u, maxit=maxit)
            UI[k] = r.x
            iters_u[k] += r.iters
            res_u[k] = r.rel_res
            status = max(status, r.status)
        b_phi = pressure_rhs(S, UI)
        if i == 0:
            x0 = plain_pressure_start(st, b_phi, pressure_start) if phi_guess is None else phi_guess
        else:
            x0 = np.zeros_like(b_phi)
        rp = krylov.pcg(S.K, b_phi, x0, rtol=rtol_p, maxit=maxit)
        status = max(status, rp.status)
        iters_p += rp.iters
        res_p = rp.rel_res
        phi = rp.x - rp.x.mean()
        p_star = p_star + phi
        p_star = p_star - p_star.mean()
        phis.append(phi)
    p_new = p_star
    iters_m = []
    if update == "lumped":
        Un = np.stack([UI[k] - S.dt * (S.dP[k] @ phi) / S.ML for k in range(d)])
        if mesh.bc_dofs.size:
            Un[:, mesh.bc_dofs] = g
    elif update == "consistent":
        Un, iters_m = consistent_update(S, UI, phi, g, rtol_u, maxit)
    elif update == "gradient":
        G = gradient_update_matrices(S)
        Un = np.stack([UI[k] - S.dt * (G[k] @ phi) for k in range(d)])
        if mesh.bc_dofs.size:
            Un[:, mesh.bc_dofs] = g
    else:
        raise ValueError(update)
    C1 = st.C1
    Cn, iters_c = None, []
    if scalars:
        Cn = np.empty_like(C1)
        for a, sc in enumerate(scalars):
            gc = sc.bc(t_new) if mesh.bc_dofs.size else np.zeros(0)
            Ac, bc_ = scalar_system(S, st, C1[a], sc, gc)
            r = krylov.bicgstab(Ac, bc_, C1[a], rtol=rtol_u, maxit=maxit)
            Cn[a] = r.x
            iters_c.append(r.iters)
            status = max(status, r.status)
    new = State(Un, st.U1.copy(), p_new, phi, t_new, Cn)
    return StepOut(new, A, b, UI, b_phi, phi, iters_u, iters_p, res_u, res_p, status, phis, iters_m, iters_c)


def plain_pressure_start(st: State, b_phi, pressure_start="prev"):
    if pressure_start == "prev":
        return st.phi_prev
    if pressure_start == "zero":
        return np.zeros_like(b_phi)
    raise ValueError(pressure_start)


def initial_state(problem, C1=None) -> State:
    return State(problem.U1.copy(), problem.U2.copy(), problem.p.copy(),
                 problem.phi_prev.copy(), problem.t0, None if C1 is None else np.array(C1, dtype=float))


def run(problem, steps, rtol_u=None, rtol_p=None, callback=None):
    S = setup(problem.mesh, problem.nu, problem.dt, problem.f)
    st = initial_state(problem)
    out = None
    for n in range(steps):
        out = step(S, st, problem.bc_values,
                   rtol_u=problem.rtol_u if rtol_u is None else rtol_u,
                   rtol_p=problem.rtol_p if rtol_p is None else rtol_p)
        st = out.state
        if callback is not None:
            callback(n, out)
    return S, st, out
