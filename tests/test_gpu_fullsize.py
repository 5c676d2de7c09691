"""Parity at the benchmark's full size: the 129x129x97 channel (1,585,152
dofs, 9,437,184 tets, 23,678,976 CSR entries), in the launch configurations
bench.py times.

The oracle cannot assemble or solve the whole problem within a test, so it
is checked on sampled rows and through properties that hold at any size:

* every preassembled matrix (M, K, dP^k, M_L) on sampled rows (random,
  wall and periodic-seam dofs), against the oracle's assembly of just the
  cells around those rows, which gives those rows exactly;
* after one step, FP64 from phi_prev and the headline mixed configuration
  (FP32 Krylov, phi_0 = 0, learned warm start attached):
  - the tentative matrix, its diagonal and the three right-hand sides on
    the sampled rows (the oracle's Alg. 2 on the same cells from the same
    U^{n-1}, U^{n-2}, p*);
  - b_phi (up to its projection constant) and the velocity update on the
    sampled rows, from the GPU's own U^I and phi;
  - the true residuals of all four solves, recomputed on the host with the
    row-checked GPU matrices at full size;
  - zero-mean p and phi;
* the 23,678,976-entry pattern (15N - 4 walls, sorted rows, symmetric on
  the sampled rows) and a valid colouring;
* the displaced, randomly relabelled mesh reordered by the on-device RCM:
  a bijection whose bandwidth is at most 2 x-y layers and at most 1.5x the
  structured numbering's, a valid colouring of the relabelled mesh, and
  one FP64 step (rtol 1e-12) giving the same fields as the same mesh in
  structured numbering, and matching the oracle on sampled rows (tentative
  equations, pressure right-hand side, velocity update); a mixed step on
  it converges.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import synth
from gpu_util import T, csr_host, dev, rel, say
from oracle import ipcs

pytestmark = pytest.mark.gpu

SIZE = (129, 129, 97)


@pytest.fixture(scope="module")
def oa():
    import paper_1602_03643_amd as m
    return m


def _device(oa, mesh):
    dm = oa.DeviceMesh.from_arrays(mesh.dim, mesh.coords, mesh.cells, mesh.vert2dof, mesh.n_dof, dev())
    pat = oa.p1_pattern(dm)
    oa.colorize(dm, T(synth.cell_priorities(mesh.n_cell), torch.int32))
    return dm, pat


@pytest.fixture(scope="module")
def full(oa):
    pr = synth.channel_flow(SIZE, seed=0)
    say("full size", pr.mesh.name, pr.mesh.n_dof)
    dm, pat = _device(oa, pr.mesh)
    torch.cuda.synchronize()
    return pr, dm, pat


def _sample_rows(mesh, k=240, seed=11):
    nx, ny, nz = SIZE
    mx, mz = nx - 1, nz - 1
    n = mesh.n_dof
    special = [0, 1, mx - 1, mx, mx * (ny - 1), mx * ny - 1, mx * ny, mx * ny + mx - 1,
               mx * ny * (mz - 1), mx * ny * (mz - 1) + mx * (ny // 2), n - mx, n - 1]
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(n, k, replace=False), special])).astype(np.int64)


def _local_setup(pr, rows):
    """Oracle setup over only the cells that touch `rows`: the sampled rows
    of every assembled matrix are then exact."""
    m = pr.mesh
    mask = np.isin(m.vert2dof[m.cells], rows).any(axis=1)
    sub = dataclasses.replace(m, cells=m.cells[mask])
    return ipcs.setup(sub, pr.nu, pr.dt, pr.f)


def _rows_err(G, O, rows):
    """max over rows of ||G_r - O_r|| / ||O_r|| (rows compared densely)."""
    worst = 0.0
    for r in rows:
        g, o = G.getrow(r).toarray().ravel(), O.getrow(r).toarray().ravel()
        no = np.linalg.norm(o)
        worst = max(worst, np.linalg.norm(g - o) / (no if no > 0 else 1.0))
    return worst


def _vec_err(g, o):
    no = np.linalg.norm(o)
    return float(np.linalg.norm(g - o) / (no if no > 0 else 1.0))


def test_fullsize_pattern_and_colouring(oa, full):
    pr, dm, pat = full
    m = pr.mesh
    n = m.n_dof
    assert pat.nnz == 15 * n - 4 * m.bc_dofs.size == 23678976
    rp = pat.row_ptr.cpu().numpy()
    ci = pat.col_idx.cpu().numpy()
    assert np.all(np.diff(rp) >= 11) and np.all(np.diff(rp) <= 15)
    rows = np.repeat(np.arange(n), np.diff(rp))
    d = np.diff(ci.astype(np.int64))
    assert np.all((d > 0) | (rows[1:] != rows[:-1]))          # strictly increasing within rows
    P = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
    for r in _sample_rows(m):
        for c in P.getrow(r).indices:
            assert P[c, r] == 1.0
    _check_colouring(dm)


def _check_colouring(dm):
    ptr = dm.color_ptr
    cells = dm.cells.long()
    v2d = dm.vert2dof.long()
    seen = 0
    for c in range(len(ptr) - 1):
        cl = dm.color_cells[int(ptr[c]): int(ptr[c + 1])].long()
        dofs = v2d[cells[cl]].reshape(-1)
        assert torch.unique(dofs).numel() == dofs.numel(), c
        seen += cl.numel()
    assert seen == dm.n_cell
    allc = torch.sort(dm.color_cells.long()).values
    assert torch.equal(allc, torch.arange(dm.n_cell, device=allc.device))


def test_fullsize_preassembled_matrices_on_sampled_rows(oa, full):
    pr, dm, pat = full
    rows = _sample_rows(pr.mesh)
    say("full-size matrices,", rows.size, "sampled rows")
    S = _local_setup(pr, rows)
    h = oa.IPCS(dm, pat, pr.dt, pr.nu, pr.f, T(pr.mesh.bc_dofs, torch.int32))
    M = csr_host(pat, h.matrix(oa.FORM_MASS)[0])
    Ks, s = h.matrix(oa.FORM_STIFF)
    sv = s.cpu().numpy()
    K = sp.diags(sv) @ csr_host(pat, Ks) @ sp.diags(sv)
    assert _rows_err(M, S.M, rows) < 1e-13
    assert _rows_err(K.tocsr(), S.K, rows) < 1e-12
    for k in range(3):
        Dk = csr_host(pat, h.matrix(oa.FORM_GRAD_X + k)[0])
        assert _rows_err(Dk, S.dP[k], rows) < 1e-13, k
    ML = h.matrix(-1, count=pr.mesh.n_dof)[0].cpu().numpy()
    assert _vec_err(ML[rows], S.ML[rows]) < 1e-14
    h.close()


def _one_step(oa, pr, dm, pat, precision, pstart, warm=None, rtol=1e-8):
    m = pr.mesh
    h = oa.IPCS(dm, pat, pr.dt, pr.nu, pr.f, T(m.bc_dofs, torch.int32), rtol_u=rtol, rtol_p=rtol,
                precision=precision, pressure_start=pstart)
    if warm is not None:
        h.set_warmstart(torch.as_tensor(warm, device=dev()), T(m.dof_coords))
    U1, U2, p, phi = T(pr.U1), T(pr.U2), T(pr.p), T(pr.phi_prev)
    Un, UI = torch.empty_like(U1), torch.empty_like(U1)
    bphi = torch.empty_like(p)
    st = h.step(U1, U2, Un, p, phi, bc_values=T(pr.bc_values(pr.t0 + pr.dt)), UI=UI, b_phi=bphi)
    torch.cuda.synchronize()
    return h, st, Un.cpu().numpy(), UI.cpu().numpy(), p.cpu().numpy(), phi.cpu().numpy(), bphi.cpu().numpy()


@pytest.mark.parametrize("config", ["fp64_prev", "mixed_zero_learned"])
def test_fullsize_step_sampled_rows_and_true_residuals(oa, full, config):
    from paper_1602_03643_amd import warmstart
    pr, dm, pat = full
    m = pr.mesh
    n = m.n_dof
    rows = _sample_rows(m)
    say("full-size step", config)
    if config == "fp64_prev":
        h, st, Un, UI, p, phi, bphi = _one_step(oa, pr, dm, pat, oa.F64, oa.PSTART_PREV)
    else:
        h, st, Un, UI, p, phi, bphi = _one_step(oa, pr, dm, pat, oa.F32, oa.PSTART_ZERO,
                                                warm=warmstart.load()[0])
    rtol = 1e-8
    assert st["status"] == 0
    assert st["res_p"] <= rtol * 1.0001 and max(st["res_u"]) <= rtol * 1.0001
    # oracle rows of Alg. 2 from the same inputs
    S = _local_setup(pr, rows)
    A_o, b_o = ipcs.tentative_system(S, ipcs.initial_state(pr), pr.t0 + pr.dt, pr.bc_values(pr.t0 + pr.dt))
    dA = h.matrix(oa.INSPECT_DIAG_A, count=n)[0].cpu().numpy()
    Ahat = csr_host(pat, h.matrix(oa.INSPECT_A)[0])
    A = (Ahat @ sp.diags(dA)).tocsr()
    assert _rows_err(A, A_o, rows) < 1e-12
    assert _vec_err(dA[rows], A_o.diagonal()[rows]) < 1e-13
    b = np.stack([h.matrix(oa.INSPECT_RHS + k, count=n)[0].cpu().numpy() for k in range(3)])
    assert _vec_err(b[:, rows], b_o[:, rows]) < 1e-12
    # full true residuals with the row-checked matrices
    for k in range(3):
        assert np.linalg.norm(b[k] - A @ UI[k]) <= rtol * 1.0001 * np.linalg.norm(b[k]), k
    Ks, s = h.matrix(oa.FORM_STIFF)
    sv = s.cpu().numpy()
    K = (sp.diags(sv) @ csr_host(pat, Ks) @ sp.diags(sv)).tocsr()
    assert _rows_err(K, S.K, rows) < 1e-12
    assert np.linalg.norm(bphi - K @ phi) <= rtol * 1.0001 * np.linalg.norm(bphi)
    # b_phi rows: -(1/dt) sum_k dP^k U^I, up to the projection constant
    raw = -(1.0 / pr.dt) * sum(S.dP[k][rows] @ UI[k] for k in range(3))
    diff = bphi[rows] - raw
    assert np.abs(diff - diff.mean()).max() <= 1e-12 * np.abs(raw).max()
    assert abs(bphi.mean()) <= 1e-14 * np.abs(bphi).max()
    # velocity update rows; Dirichlet rows take the boundary values (0)
    upd = np.stack([UI[k][rows] - pr.dt * (S.dP[k][rows] @ phi) / S.ML[rows] for k in range(3)])
    bc = np.isin(rows, m.bc_dofs)
    upd[:, bc] = 0.0
    assert _vec_err(Un[:, rows], upd) < 1e-12
    # zero means; p = p* + phi with p* = 0 at the first step
    assert abs(phi.mean()) <= 1e-13 * np.abs(phi).max() and abs(p.mean()) <= 1e-13 * np.abs(p).max()
    assert _vec_err(p, phi) < 1e-13
    h.close()


def test_fullsize_config4_rcm_relabelled_step(oa):
    """Displaced mesh, random relabelling, on-device RCM; the reordered
    problem solves to the same fields as the structured numbering."""
    pr = synth.channel_flow(SIZE, seed=0, displace_seed=1000)
    m0 = pr.mesh
    pm, dof_perm = synth.permute_mesh(m0, 2000)
    n = m0.n_dof
    nx, ny, nz = SIZE
    layer = (nx - 1) * ny
    say("config 4", pm.name, n)
    dmp = oa.DeviceMesh.from_arrays(pm.dim, pm.coords, pm.cells, pm.vert2dof, n, dev())
    patp = oa.p1_pattern(dmp)
    perm, order = oa.rcm(patp)
    assert torch.equal(torch.sort(perm.long()).values, torch.arange(n, device=perm.device))
    assert torch.equal(perm.long()[order.long()], torch.arange(n, device=perm.device))
    rp = patp.row_ptr.long()
    rows = torch.repeat_interleave(torch.arange(n, device=rp.device), rp[1:] - rp[:-1])
    cols = patp.col_idx.long()
    bw_rcm = int((perm.long()[rows] - perm.long()[cols]).abs().max())
    pat0 = oa.p1_pattern(oa.DeviceMesh.from_arrays(m0.dim, m0.coords, m0.cells, m0.vert2dof, n, dev()))
    rp0 = pat0.row_ptr.long()
    rows0 = torch.repeat_interleave(torch.arange(n, device=rp0.device), rp0[1:] - rp0[:-1])
    bw_struct = int((rows0 - pat0.col_idx.long()).abs().max())
    bw_rand = int((rows - cols).abs().max())
    say("bandwidth: random %d, structured %d, rcm %d (x-y layer %d)" % (bw_rand, bw_struct, bw_rcm, layer))
    assert bw_rcm <= 2 * layer and bw_rcm <= 1.5 * bw_struct
    # relabel the mesh's dofs on the device and colour the reordered mesh
    v2d = oa.relabel(dmp.vert2dof, perm)
    bc = oa.relabel(T(pm.bc_dofs, torch.int32), perm)
    dmr = oa.DeviceMesh(3, dmp.coords, dmp.cells, v2d, n)
    patr = oa.p1_pattern(dmr)
    assert patr.nnz == patp.nnz
    oa.colorize(dmr, T(synth.cell_priorities(pm.n_cell), torch.int32))
    _check_colouring(dmr)
    # same fields in both numberings: new = perm[dof_perm[old]]
    to_new = perm.long()[T(dof_perm, torch.int64)]
    dm0, pat0c = _device(oa, m0)

    extra = {}

    def run(dm, pat, bcd, fields, precision, rtol, keep=False):
        h = oa.IPCS(dm, pat, pr.dt, pr.nu, pr.f, bcd, rtol_u=rtol, rtol_p=rtol, precision=precision)
        U1, U2, p, phi = [f.clone() for f in fields]
        Un = torch.empty_like(U1)
        UI, bphi = torch.empty_like(U1), torch.empty_like(p)
        nbc = bcd.numel()
        st = h.step(U1, U2, Un, p, phi, bc_values=torch.zeros(3 * nbc, dtype=torch.float64, device=dev()),
                    UI=UI, b_phi=bphi)
        torch.cuda.synchronize()
        if keep:
            extra.update(UI=UI.cpu().numpy(), bphi=bphi.cpu().numpy(), phi=phi.cpu().numpy(), Un=Un.cpu().numpy())
        h.close()
        return st, Un, p

    f0 = [T(pr.U1), T(pr.U2), T(pr.p), T(pr.phi_prev)]

    def to_rcm(x):
        y = torch.empty_like(x)
        if x.dim() == 1:
            y[to_new] = x
        else:
            y[:, to_new] = x
        return y

    fr = [to_rcm(x) for x in f0]
    st0, Un0, p0 = run(dm0, pat0c, T(m0.bc_dofs, torch.int32), f0, oa.F64, 1e-12)
    str_, Unr, pr_ = run(dmr, patr, bc, fr, oa.F64, 1e-12, keep=True)
    assert st0["status"] == 0 and str_["status"] == 0
    # the oracle on sampled rows of the RCM-numbered displaced mesh: the
    # tentative equations (assembled from the cells around each row) hold
    # for U^I, b_phi is -(1/dt) sum_k dP^k U^I up to the projection constant,
    # and the lumped update follows from U^I and phi
    permh = perm.long().cpu().numpy()
    mr = dataclasses.replace(pm, vert2dof=permh[pm.vert2dof].astype(np.int32),
                             bc_dofs=np.sort(permh[pm.bc_dofs]).astype(np.int32))
    prr = dataclasses.replace(pr, mesh=mr)
    rows = np.unique(np.random.default_rng(17).choice(n, 240, replace=False)).astype(np.int64)
    S = _local_setup(prr, rows)
    frh = [x.cpu().numpy() for x in fr]
    st_in = ipcs.State(frh[0], frh[1], frh[2], frh[3], 0.0)
    A, b = ipcs.tentative_system(S, st_in, pr.dt, np.zeros((3, mr.bc_dofs.size)))
    UI, bphi, phi, Un = extra["UI"], extra["bphi"], extra["phi"], extra["Un"]
    for k in range(3):
        res = A[rows] @ UI[k] - b[k][rows]
        scale = abs(A[rows]) @ np.abs(UI[k]) + np.abs(b[k][rows])
        assert np.abs(res).max() <= 1e-9 * scale.max(), k     # the solve's rtol is 1e-12
    raw = -(1.0 / pr.dt) * sum(S.dP[k][rows] @ UI[k] for k in range(3))
    diff = bphi[rows] - raw
    assert np.abs(diff - diff.mean()).max() <= 1e-12 * np.abs(raw).max()
    upd = np.stack([UI[k][rows] - pr.dt * (S.dP[k][rows] @ phi) / S.ML[rows] for k in range(3)])
    upd[:, np.isin(rows, mr.bc_dofs)] = 0.0
    assert _vec_err(Un[:, rows], upd) < 1e-12
    say("iterations structured %s / %d, rcm %s / %d" % (st0["iters_u"], st0["iters_p"], str_["iters_u"],
                                                         str_["iters_p"]))
    assert rel(Unr[:, to_new].cpu().numpy(), Un0.cpu().numpy()) < 1e-9
    assert rel(pr_[to_new].cpu().numpy(), p0.cpu().numpy()) < 1e-6
    stm, _, _ = run(dmr, patr, bc, fr, oa.F32, 1e-8)
    assert stm["status"] == 0 and stm["res_p"] <= 1.0001e-8 and max(stm["res_u"]) <= 1.0001e-8
