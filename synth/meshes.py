"""Structured simplex meshes shaped like the paper's verification workloads.

* ``unit_square`` / ``periodic_square``: the 2D Taylor-Green meshes of the
  paper's Sec. 6.1 (right triangles, uniform in both directions).
* ``channel``: the Sec. 6.2 channel box, 4*pi x 2 x 4*pi/3, hexahedra split
  into 6 tetrahedra (Kuhn/Freudenthal split along the main diagonal),
  tanh wall-normal stretching, periodic x and z through dof identification
  (footnote of Sec. 6.2), optional seeded interior-node displacement.
* ``permute_mesh``: random relabelling of dofs, vertices and cells.

Every cell is positively oriented (det of [x1-x0, ..., xd-x0] > 0).
Dof numbering of the structured meshes is lexicographic with x fastest.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Mesh:
    dim: int
    coords: np.ndarray        # float64 [n_vert, dim]
    cells: np.ndarray         # int32   [n_cell, dim+1]  vertex indices
    vert2dof: np.ndarray      # int32   [n_vert]         periodic identification
    n_dof: int
    bc_dofs: np.ndarray       # int32   sorted unique velocity-Dirichlet dofs
    dof_coords: np.ndarray    # float64 [n_dof, dim]     coords of one vertex per dof
    name: str = ""
    volume: float = float("nan")   # exact measure of the domain

    @property
    def n_vert(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cell(self) -> int:
        return int(self.cells.shape[0])


def _dof_coords(coords: np.ndarray, vert2dof: np.ndarray, n_dof: int) -> np.ndarray:
    # the lowest-numbered vertex of each dof represents it
    first = np.full(n_dof, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(first, vert2dof.astype(np.int64), np.arange(vert2dof.size, dtype=np.int64))
    return coords[first].copy()


def _square_cells(n: int) -> np.ndarray:
    """Right triangles of an n x n grid, diagonal (i,j)->(i+1,j+1), CCW."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v = lambda a, b: (a + (n + 1) * b)  # noqa: E731  x fastest
    t1 = np.stack([v(i, j), v(i + 1, j), v(i + 1, j + 1)], axis=1)
    t2 = np.stack([v(i, j), v(i + 1, j + 1), v(i, j + 1)], axis=1)
    return np.concatenate([t1, t2], axis=0).astype(np.int32)


def unit_square(n: int, length: float = 1.0) -> Mesh:
    """[0,L]^2 with n x n squares, each split into two right triangles.

    All boundary vertices are velocity-Dirichlet dofs (exact data there)."""
    xs = np.linspace(0.0, length, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")      # row = y index, col = x index
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    cells = _square_cells(n)
    nv = (n + 1) ** 2
    vert2dof = np.arange(nv, dtype=np.int32)
    ix = np.arange(nv) % (n + 1)
    iy = np.arange(nv) // (n + 1)
    bnd = (ix == 0) | (ix == n) | (iy == 0) | (iy == n)
    bc = np.nonzero(bnd)[0].astype(np.int32)
    return Mesh(2, coords, cells, vert2dof, nv, bc, coords.copy(),
                name=f"unit_square_{n}", volume=length * length)


def periodic_square(n: int, length: float = 2.0) -> Mesh:
    """Doubly periodic [0,L]^2 (the paper's Taylor-Green box), no Dirichlet dofs."""
    m = unit_square(n, length)
    nv = m.n_vert
    ix = np.arange(nv) % (n + 1)
    iy = np.arange(nv) // (n + 1)
    dof = (ix % n) + n * (iy % n)
    vert2dof = dof.astype(np.int32)
    n_dof = n * n
    return Mesh(2, m.coords, m.cells, vert2dof, n_dof, np.zeros(0, np.int32),
                _dof_coords(m.coords, vert2dof, n_dof),
                name=f"periodic_square_{n}", volume=length * length)


def _kuhn_cells(nx: int, ny: int, nz: int) -> np.ndarray:
    """6 tets per hex of an (nx-1)x(ny-1)x(nz-1) vertex grid; vertex id = ix + nx*(iy + ny*iz)."""
    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    ci = ci.ravel(order="F")
    cj = cj.ravel(order="F")
    ck = ck.ravel(order="F")
    vid = lambda a, b, c: (ci + a) + nx * ((cj + b) + ny * (ck + c))  # noqa: E731
    unit = np.eye(3, dtype=np.int64)
    out = []
    for perm in itertools.permutations(range(3)):
        o = np.zeros(3, np.int64)
        p1 = unit[perm[0]]
        p2 = p1 + unit[perm[1]]
        p3 = np.ones(3, np.int64)
        verts = [o, p1, p2, p3]
        # parity of the permutation decides the orientation; odd -> swap last two
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        if inv % 2 == 1:
            verts = [verts[0], verts[1], verts[3], verts[2]]
        out.append(np.stack([vid(*v) for v in verts], axis=1))
    # interleave so that the 6 tets of a hex are consecutive
    cells = np.stack(out, axis=1).reshape(-1, 4)
    return cells.astype(np.int32)


def _signed_volumes_x6(coords: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """6x signed tet volume; used only to validate displaced meshes."""
    x0 = coords[cells[:, 0]]
    a = coords[cells[:, 1]] - x0
    b = coords[cells[:, 2]] - x0
    c = coords[cells[:, 3]] - x0
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def channel(nx: int, ny: int, nz: int, beta: float = 2.0,
            lx: float = 4.0 * np.pi, ly: float = 2.0, lz: float = 4.0 * np.pi / 3.0,
            displace_seed: int | None = None, displace_frac: float = 0.2,
            quality_floor: float = 0.1) -> Mesh:
    """Channel box [0,lx] x [-ly/2,ly/2] x [0,lz] with nx*ny*nz vertices.

    y_j = tanh(beta*eta_j)/tanh(beta), eta_j = -1 + 2j/(ny-1).  Vertices on
    x = lx (z = lz) are identified with x = 0 (z = 0), giving
    (nx-1)*ny*(nz-1) dofs.  Dirichlet (no-slip) dofs are the two walls.

    With ``displace_seed``: every vertex off the walls and off the periodic
    faces moves, per axis, by U(-f*h_minus, f*h_plus) with h the spacing to
    the neighbouring grid lines.  Vertices whose incident tets would drop
    below ``quality_floor`` x their undisplaced volume are redrawn (up to 10
    rounds) and finally reset to the grid position.
    """
    xs = np.linspace(0.0, lx, nx)
    eta = -1.0 + 2.0 * np.arange(ny) / (ny - 1)
    ys = (ly / 2.0) * np.tanh(beta * eta) / np.tanh(beta)
    ys[0], ys[-1] = -ly / 2.0, ly / 2.0
    zs = np.linspace(0.0, lz, nz)
    nv = nx * ny * nz
    vidx = np.arange(nv)
    ix = vidx % nx
    iy = (vidx // nx) % ny
    iz = vidx // (nx * ny)
    coords = np.stack([xs[ix], ys[iy], zs[iz]], axis=1)
    cells = _kuhn_cells(nx, ny, nz)

    if displace_seed is not None:
        rng = np.random.default_rng(displace_seed)
        movable = (ix > 0) & (ix < nx - 1) & (iy > 0) & (iy < ny - 1) & (iz > 0) & (iz < nz - 1)
        mv = np.nonzero(movable)[0]
        lo = np.stack([xs[ix[mv]] - xs[ix[mv] - 1], ys[iy[mv]] - ys[iy[mv] - 1],
                       zs[iz[mv]] - zs[iz[mv] - 1]], axis=1)
        hi = np.stack([xs[ix[mv] + 1] - xs[ix[mv]], ys[iy[mv] + 1] - ys[iy[mv]],
                       zs[iz[mv] + 1] - zs[iz[mv]]], axis=1)
        base = coords.copy()
        vol0 = _signed_volumes_x6(base, cells)
        pos_in_mv = np.full(nv, -1, np.int64)
        pos_in_mv[mv] = np.arange(mv.size)

        def draw(sel):  # sel: indices into mv
            u = rng.uniform(0.0, 1.0, size=(sel.size, 3))
            delta = -displace_frac * lo[sel] + u * displace_frac * (lo[sel] + hi[sel])
            coords[mv[sel]] = base[mv[sel]] + delta

        def touching(verts):   # cells with a vertex in verts
            mark = np.zeros(nv, bool)
            mark[verts] = True
            return np.nonzero(mark[cells].any(axis=1))[0]

        draw(np.arange(mv.size))
        vol = _signed_volumes_x6(coords, cells)
        for _ in range(10):
            bad = vol < quality_floor * vol0
            if not bad.any():
                break
            verts = np.unique(cells[bad].ravel())
            sel = pos_in_mv[verts]
            sel = sel[sel >= 0]
            draw(sel)
            t = touching(mv[sel])
            vol[t] = _signed_volumes_x6(coords, cells[t])
        while True:
            bad = vol < quality_floor * vol0
            if not bad.any():
                break
            verts = np.unique(cells[bad].ravel())
            coords[verts] = base[verts]
            t = touching(verts)
            vol[t] = _signed_volumes_x6(coords, cells[t])

    mx, mz = nx - 1, nz - 1
    dof = (ix % mx) + mx * (iy + ny * (iz % mz))
    vert2dof = dof.astype(np.int32)
    n_dof = mx * ny * mz
    ddx = np.arange(n_dof)
    diy = (ddx // mx) % ny
    bc = np.nonzero((diy == 0) | (diy == ny - 1))[0].astype(np.int32)
    tag = "channel_%dx%dx%d" % (nx, ny, nz) + ("_disp%d" % displace_seed if displace_seed is not None else "")
    return Mesh(3, coords, cells, vert2dof, n_dof, bc, _dof_coords(coords, vert2dof, n_dof),
                name=tag, volume=lx * ly * lz)


def permute_mesh(mesh: Mesh, seed: int) -> tuple[Mesh, np.ndarray]:
    """Randomly relabel dofs, vertices and the order of cells.

    Returns the new mesh and ``dof_perm`` with new_dof = dof_perm[old_dof]."""
    rng = np.random.default_rng(seed)
    dof_perm = rng.permutation(mesh.n_dof).astype(np.int32)
    vperm = rng.permutation(mesh.n_vert)
    cperm = rng.permutation(mesh.n_cell)
    coords = np.empty_like(mesh.coords)
    coords[vperm] = mesh.coords
    vert2dof = np.empty_like(mesh.vert2dof)
    vert2dof[vperm] = dof_perm[mesh.vert2dof]
    cells = vperm[mesh.cells].astype(np.int32)[cperm]
    bc = np.sort(dof_perm[mesh.bc_dofs]).astype(np.int32)
    dof_coords = np.empty_like(mesh.dof_coords)
    dof_coords[dof_perm] = mesh.dof_coords
    return (Mesh(mesh.dim, coords, cells, vert2dof, mesh.n_dof, bc, dof_coords,
                 name=mesh.name + "_perm%d" % seed, volume=mesh.volume), dof_perm)


def cell_priorities(n_cell: int, seed: int = 7) -> np.ndarray:
    """Distinct random priorities (a permutation of 0..n_cell-1) for colouring."""
    return np.random.default_rng(seed).permutation(n_cell).astype(np.int32)
