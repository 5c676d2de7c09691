"""Shared helpers for the GPU tests: upload seeded inputs, build the device
mesh (pattern, colouring) and convert results back for comparison with the
oracle.  Nothing here computes any part of the method."""
import sys

import numpy as np
import torch

import synth


def dev():
    return torch.device("cuda", 0)


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_mesh(mesh, color=True, seed=7):
    import paper_1602_03643_amd as oa
    dm = oa.DeviceMesh.from_arrays(mesh.dim, mesh.coords, mesh.cells, mesh.vert2dof, mesh.n_dof, dev())
    pat = oa.p1_pattern(dm)
    colors = None
    if color:
        pri = T(synth.cell_priorities(mesh.n_cell, seed), torch.int32)
        colors = oa.colorize(dm, pri)
    return dm, pat, colors


def csr_host(pat, val=None):
    import scipy.sparse as sp
    rp = pat.row_ptr.cpu().numpy()
    ci = pat.col_idx.cpu().numpy()
    v = np.ones(ci.size) if val is None else val.cpu().numpy()
    return sp.csr_matrix((v, ci, rp), shape=(rp.size - 1, rp.size - 1))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
