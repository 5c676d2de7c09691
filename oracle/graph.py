"""Sparsity pattern, reverse Cuthill-McKee ordering and cell colouring.

The paper assembles all matrices of the optimised solver on one shared
pattern (Sec. 5, Alg. 2 discussion).  Reordering and colouring are not in
the paper; they serve the GPU data layout, and the definitions below fix one
valid answer so that a device implementation can be compared index by index.

Reverse Cuthill-McKee (RCM) definition used here
  * deg(v) = number of stored entries of row v (diagonal included).
  * Start of each connected component: the unvisited vertex with the least
    (deg, index) is the root r.  Pseudo-peripheral refinement (George-Liu):
    build the BFS level structure of r; among the vertices of its last level
    take x with the least (deg, index); if the level structure of x is deeper
    than that of r, set r = x and repeat, otherwise keep r.
  * Cuthill-McKee order: breadth-first from r; when a vertex is taken from
    the queue its not yet visited neighbours are appended sorted by
    (deg, index).
  * RCM = the Cuthill-McKee sequence reversed over the whole graph.
    ``order[k]`` is the old vertex placed at new position k;
    ``perm[old] = new``.

Cell colouring definition used here
  * Two cells conflict when they share a dof.
  * Cells are visited in decreasing priority (priorities are distinct and
    given); each takes the least colour not used by an already coloured
    conflicting cell (greedy first fit).
  * Colour classes list their cells in increasing cell index.
"""
from __future__ import annotations

from collections import deque

import numpy as np
import scipy.sparse as sp


def csr_pattern(mesh):
    """(row_ptr int32 [N+1], col_idx int32 [nnz]) of the P1 matrix, columns sorted."""
    dofs = mesh.vert2dof[mesh.cells]
    n = mesh.dim + 1
    rows = np.repeat(dofs, n, axis=1).ravel()
    cols = np.tile(dofs, (1, n)).ravel()
    A = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(mesh.n_dof,) * 2).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32)


def _levels(row_ptr, col_idx, root, visited_global):
    n = row_ptr.size - 1
    level = np.full(n, -1, np.int64)
    level[root] = 0
    frontier = [root]
    levels = [[root]]
    while True:
        nxt = []
        for u in frontier:
            for v in col_idx[row_ptr[u]:row_ptr[u + 1]]:
                if level[v] < 0 and not visited_global[v]:
                    level[v] = level[u] + 1
                    nxt.append(int(v))
        if not nxt:
            break
        levels.append(nxt)
        frontier = nxt
    return levels


def pseudo_peripheral(row_ptr, col_idx, deg, start, visited_global):
    r = start
    lv = _levels(row_ptr, col_idx, r, visited_global)
    while True:
        last = lv[-1]
        x = min(last, key=lambda v: (deg[v], v))
        lx = _levels(row_ptr, col_idx, x, visited_global)
        if len(lx) > len(lv):
            r, lv = x, lx
        else:
            return r


def rcm(row_ptr, col_idx):
    """Return (order, perm) of the reverse Cuthill-McKee ordering defined above."""
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx)
    n = row_ptr.size - 1
    deg = np.diff(row_ptr)
    visited = np.zeros(n, bool)
    cm = []
    while len(cm) < n:
        cand = np.nonzero(~visited)[0]
        start = int(cand[np.lexsort((cand, deg[cand]))[0]])
        r = pseudo_peripheral(row_ptr, col_idx, deg, start, visited)
        visited[r] = True
        q = deque([r])
        while q:
            u = q.popleft()
            cm.append(u)
            nb = [int(v) for v in col_idx[row_ptr[u]:row_ptr[u + 1]] if not visited[v]]
            nb.sort(key=lambda v: (deg[v], v))
            for v in nb:
                visited[v] = True
                q.append(v)
    order = np.array(cm[::-1], dtype=np.int32)
    perm = np.empty(n, np.int32)
    perm[order] = np.arange(n, dtype=np.int32)
    return order, perm


def bandwidth(row_ptr, col_idx, perm=None):
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx)
    rows = np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))
    if perm is not None:
        rows = perm[rows]
        cols = perm[col_idx]
    else:
        cols = col_idx
    return int(np.abs(rows.astype(np.int64) - cols).max())


def permute_pattern(row_ptr, col_idx, perm):
    """Pattern of P A P^T with P given by perm[old] = new."""
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    A = sp.coo_matrix((np.ones(rows.size), (perm[rows], perm[col_idx])), shape=(n, n)).tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32)


def greedy_coloring(mesh, priorities):
    """Colour of every cell by greedy first fit in decreasing priority."""
    dofs = mesh.vert2dof[mesh.cells]
    E = dofs.shape[0]
    # cells incident to each dof
    inc = [[] for _ in range(mesh.n_dof)]
    for c in range(E):
        for v in dofs[c]:
            inc[v].append(c)
    color = np.full(E, -1, np.int64)
    for c in np.argsort(-priorities.astype(np.int64), kind="stable"):
        used = set()
        for v in dofs[c]:
            for o in inc[v]:
                if color[o] >= 0:
                    used.add(int(color[o]))
        k = 0
        while k in used:
            k += 1
        color[c] = k
    return color.astype(np.int32)


def color_classes(color):
    """(color_ptr [n_colors+1], cells ordered by (colour, cell index))."""
    order = np.lexsort((np.arange(color.size), color)).astype(np.int32)
    counts = np.bincount(color)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return ptr, order


def coloring_conflicts(mesh, color):
    """Number of (colour, dof) pairs claimed by more than one cell (0 = valid)."""
    dofs = mesh.vert2dof[mesh.cells]
    key = color.astype(np.int64)[:, None] * mesh.n_dof + dofs
    _, counts = np.unique(key.ravel(), return_counts=True)
    return int((counts > 1).sum())
