"""Problem data: parameters, initial history and Dirichlet values.

* ``taylor_green``: the 2D Taylor-Green vortex (paper Sec. 6.1).  Either the
  paper's doubly periodic [0,2]^2 box or [0,1]^2 with the exact velocity
  prescribed on the boundary.  The history is started from the exact
  solution: U^{n-1} = u_e(t0), U^{n-2} = u_e(t0 - dt), p* = p_e(t0 - dt/2),
  phi_prev = 0.
* ``channel_flow``: the Sec. 6.2 channel at Re_tau = 180 (nu = 1/180, body
  force (1,0,0), no-slip walls), started from the laminar parabola
  U_c (1 - y^2) plus seeded uniform noise on the non-wall dofs.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

from .meshes import Mesh, channel, permute_mesh, periodic_square, unit_square

# vertex counts (nx, ny, nz) of the channel workloads
CHANNEL_SIZES = {
    "tiny": (9, 9, 7),
    "small": (17, 17, 13),
    "c65": (65, 65, 49),       # 199,680 dofs per field
    "c129": (129, 129, 97),    # 1,585,152 dofs per field
}


def tg_exact_velocity(x: np.ndarray, y: np.ndarray, t: float, nu: float) -> np.ndarray:
    e = np.exp(-2.0 * np.pi ** 2 * nu * t)
    return np.stack([-np.sin(np.pi * y) * np.cos(np.pi * x) * e,
                     np.sin(np.pi * x) * np.cos(np.pi * y) * e])


def tg_exact_pressure(x: np.ndarray, y: np.ndarray, t: float, nu: float) -> np.ndarray:
    return -0.25 * (np.cos(2 * np.pi * x) + np.cos(2 * np.pi * y)) * np.exp(-4.0 * np.pi ** 2 * nu * t)


@dataclasses.dataclass
class Problem:
    mesh: Mesh
    nu: float
    dt: float
    f: np.ndarray                 # [dim] constant body force
    U1: np.ndarray                # [dim, n_dof] U^{n-1}
    U2: np.ndarray                # [dim, n_dof] U^{n-2}
    p: np.ndarray                 # [n_dof] p*
    phi_prev: np.ndarray          # [n_dof]
    t0: float
    bc_values: Callable[[float], np.ndarray]   # t -> [dim, n_bc]
    rtol_u: float
    rtol_p: float
    name: str = ""
    extra: dict = dataclasses.field(default_factory=dict)


def taylor_green(n: int, periodic: bool = False, nu: float = 0.01, dt: float = 1e-3,
                 rtol: float = 1e-10) -> Problem:
    mesh = periodic_square(n, 2.0) if periodic else unit_square(n, 1.0)
    X, Y = mesh.dof_coords[:, 0], mesh.dof_coords[:, 1]
    t0 = 0.0
    U1 = tg_exact_velocity(X, Y, t0, nu)
    U2 = tg_exact_velocity(X, Y, t0 - dt, nu)
    p = tg_exact_pressure(X, Y, t0 - 0.5 * dt, nu)
    bx, by = X[mesh.bc_dofs], Y[mesh.bc_dofs]

    def bc_values(t: float) -> np.ndarray:
        return tg_exact_velocity(bx, by, t, nu)

    return Problem(mesh, nu, dt, np.zeros(2), U1, U2, p, np.zeros(mesh.n_dof), t0,
                   bc_values, rtol, rtol, name=mesh.name)


def channel_flow(size: str | tuple = "c65", seed: int = 0, u_center: float = 1.0,
                 noise: float = 0.05, nu: float = 1.0 / 180.0, dt: float = 0.01,
                 displace_seed: int | None = None, permute_seed: int | None = None,
                 rtol: float = 1e-8) -> Problem:
    nx, ny, nz = CHANNEL_SIZES[size] if isinstance(size, str) else size
    mesh = channel(nx, ny, nz, displace_seed=displace_seed)
    perm = None
    if permute_seed is not None:
        mesh, perm = permute_mesh(mesh, permute_seed)
    y = mesh.dof_coords[:, 1]
    n = mesh.n_dof
    rng = np.random.default_rng(seed)
    U = rng.uniform(-noise, noise, size=(3, n))
    U[0] += u_center * (1.0 - y ** 2)
    U[:, mesh.bc_dofs] = 0.0
    nbc = mesh.bc_dofs.size

    def bc_values(t: float) -> np.ndarray:
        return np.zeros((3, nbc))

    return Problem(mesh, nu, dt, np.array([1.0, 0.0, 0.0]), U, U.copy(), np.zeros(n),
                   np.zeros(n), 0.0, bc_values, rtol, rtol, name=mesh.name,
                   extra={"dof_perm": perm})
