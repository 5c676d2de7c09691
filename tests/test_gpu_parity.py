"""GPU parity: every C-ABI entry point against the FP64 oracle on identical
seeded inputs.  Index work (pattern, colouring, RCM) must match bit for bit;
floating point within the stated tolerances:

* element-matrix assembly and sparse products: relative max error 1e-13
  (only the summation order differs);
* Krylov solves and the IPCS step: both sides run to rtol 1e-13 and must
  agree to 1e-10 in relative L2 (the FP64 tolerance of the method); at the
  production rtol the true residual is checked instead.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import synth
from gpu_util import T, csr_host, dev, device_mesh, rel, say
from oracle import graph, ipcs, krylov, p1, mixed

pytestmark = pytest.mark.gpu


def _meshes():
    return [synth.unit_square(9), synth.periodic_square(8), synth.channel(9, 9, 7),
            synth.channel(9, 9, 7, displace_seed=11), synth.permute_mesh(synth.channel(9, 9, 7), 5)[0],
            synth.channel(17, 17, 13)]


@pytest.fixture(scope="module")
def oa():
    import paper_1602_03643_amd as m
    return m


@pytest.mark.parametrize("mesh", _meshes(), ids=lambda m: m.name)
def test_pattern_and_coloring_bit_exact(oa, mesh):
    say("pattern/colouring", mesh.name)
    dm, pat, color = device_mesh(mesh)
    rp, ci = graph.csr_pattern(mesh)
    assert np.array_equal(pat.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(pat.col_idx.cpu().numpy(), ci)
    if mesh.n_cell <= 5000:
        ref = graph.greedy_coloring(mesh, synth.cell_priorities(mesh.n_cell, 7))
        assert np.array_equal(color.cpu().numpy(), ref)
        cptr, cells = graph.color_classes(ref)
        assert np.array_equal(dm.color_ptr, cptr)
        assert np.array_equal(dm.color_cells.cpu().numpy(), cells)
    assert graph.coloring_conflicts(mesh, color.cpu().numpy()) == 0


@pytest.mark.parametrize("mesh", [synth.permute_mesh(synth.channel(9, 9, 7), 2000)[0],
                                  synth.permute_mesh(synth.channel(17, 17, 13, displace_seed=1000), 2000)[0],
                                  synth.unit_square(12)], ids=lambda m: m.name)
def test_rcm_bit_exact(oa, mesh):
    say("rcm", mesh.name)
    dm, pat, _ = device_mesh(mesh, color=False)
    perm, order = oa.rcm(pat)
    rp, ci = graph.csr_pattern(mesh)
    o_ref, p_ref = graph.rcm(rp, ci)
    assert np.array_equal(perm.cpu().numpy(), p_ref)
    assert np.array_equal(order.cpu().numpy(), o_ref)


@pytest.mark.parametrize("mesh", _meshes(), ids=lambda m: m.name)
def test_assembly_matches_oracle(oa, mesh):
    say("assembly", mesh.name)
    dm, pat, _ = device_mesh(mesh)
    geo = p1.element_geometry(mesh)
    Pp = csr_host(pat)
    forms = [(oa.FORM_MASS, p1.mass_matrix(mesh, geo)), (oa.FORM_STIFF, p1.stiffness_matrix(mesh, geo))]
    for k in range(mesh.dim):
        forms.append((oa.FORM_GRAD_X + k, p1.gradient_matrix(mesh, k, geo)))
    rng = np.random.default_rng(1)
    ub = rng.normal(size=(mesh.dim, mesh.n_dof))
    forms.append((oa.FORM_CONV, p1.convection_matrix(mesh, ub, geo)))
    for form, ref in forms:
        uab = [T(ub[k]) for k in range(mesh.dim)] if form == oa.FORM_CONV else None
        val = oa.assemble_p1(dm, pat, form, uab=uab).cpu().numpy()
        want = p1.on_pattern(ref, Pp)
        err = np.abs(val - want).max() / np.abs(want).max()
        assert err <= 1e-13, (form, err)
    # base + alpha * form
    base = T(rng.normal(size=pat.nnz))
    val = oa.assemble_p1(dm, pat, oa.FORM_STIFF, alpha=-0.25, base=base).cpu().numpy()
    want = base.cpu().numpy() - 0.25 * p1.on_pattern(forms[1][1], Pp)
    assert np.abs(val - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("mesh", [synth.channel(17, 17, 13), synth.unit_square(33)], ids=lambda m: m.name)
def test_spmv_matches_oracle(oa, mesh):
    say("spmv", mesh.name)
    dm, pat, _ = device_mesh(mesh)
    K = p1.stiffness_matrix(mesh)
    Kp = p1.on_pattern(K, csr_host(pat))
    rng = np.random.default_rng(2)
    x = rng.normal(size=mesh.n_dof)
    y0 = rng.normal(size=mesh.n_dof)
    A = pat.with_values(T(Kp))
    y = T(y0)
    oa.spmv(A, T(x), y, alpha=0.5, beta=-2.0)
    want = 0.5 * (K @ x) - 2.0 * y0
    assert np.abs(y.cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()
    # FP32 path accumulates in FP32
    A32 = pat.with_values(T(Kp, torch.float32))
    y32 = torch.zeros(mesh.n_dof, dtype=torch.float32, device=dev())
    oa.spmv(A32, T(x, torch.float32), y32)
    assert rel(y32.cpu().numpy(), K @ x) < 1e-5


def _tent_problem(prob):
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    st = ipcs.initial_state(prob)
    A, b = ipcs.tentative_system(S, st, prob.t0 + prob.dt, prob.bc_values(prob.t0 + prob.dt))
    return S, st, A, b


@pytest.mark.parametrize("prob", [synth.channel_flow("small", seed=3), synth.taylor_green(20)],
                         ids=lambda p: p.name)
def test_pcg_matches_oracle(oa, prob):
    say("pcg", prob.name)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Kp = p1.on_pattern(S.K, csr_host(pat))
    rng = np.random.default_rng(4)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    x0 = rng.normal(size=prob.mesh.n_dof) * 0.1
    ref = krylov.pcg(S.K, bphi, x0, rtol=1e-13)
    x = T(x0)
    out = oa.pcg(pat.with_values(T(Kp)), T(bphi), x, rtol=1e-13)
    assert out["rc"] == 0 and out["rel_res"] <= 1e-13
    xr = ref.x - ref.x.mean()
    xg = x.cpu().numpy()
    xg = xg - xg.mean()
    assert rel(xg, xr) <= 1e-10
    assert abs(out["iters"] - ref.iters) <= max(3, 0.02 * ref.iters), (out["iters"], ref.iters)
    # production tolerance: the oracle's own true residual confirms the GPU answer
    x = T(x0)
    out = oa.pcg(pat.with_values(T(Kp)), T(bphi), x, rtol=1e-8)
    xg = x.cpu().numpy()
    assert np.linalg.norm(bphi - S.K @ xg) <= 1e-8 * np.linalg.norm(bphi) * (1 + 1e-6)


@pytest.mark.parametrize("prob", [synth.channel_flow("small", seed=5), synth.taylor_green(20),
                                  synth.channel_flow("tiny", displace_seed=3)], ids=lambda p: p.name)
def test_bicgstab_matches_oracle(oa, prob):
    say("bicgstab", prob.name)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Ap = p1.on_pattern(A, csr_host(pat))
    d = prob.mesh.dim
    x = T(st.U1)
    out = oa.bicgstab(pat.with_values(T(Ap)), T(b), x, rtol=1e-13)
    for k in range(d):
        ref = krylov.bicgstab(A, b[k], st.U1[k], rtol=1e-13)
        assert out[k]["status"] == 0 and out[k]["rel_res"] <= 1e-13
        assert rel(x[k].cpu().numpy(), ref.x) <= 1e-10
        assert abs(out[k]["iters"] - ref.iters) <= 2, (k, out[k]["iters"], ref.iters)
    # nrhs = 1 agrees with the batched solve
    x1 = T(st.U1[0])
    out1 = oa.bicgstab(pat.with_values(T(Ap)), T(b[0]), x1, rtol=1e-13)
    assert rel(x1.cpu().numpy(), x[0].cpu().numpy()) <= 1e-10 and out1[0]["status"] == 0


def test_krylov_failure_paths(oa):
    say("failure paths")
    prob = synth.channel_flow("tiny", seed=1)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Kp = T(p1.on_pattern(S.K, csr_host(pat)))
    rng = np.random.default_rng(7)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    out = oa.pcg(pat.with_values(Kp), T(bphi), torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev()),
                 rtol=1e-12, maxit=1)
    assert out["rc"] == oa.ENOTCONV and out["iters"] == 1
    bn = bphi.copy()
    bn[3] = np.nan
    out = oa.pcg(pat.with_values(Kp), T(bn), torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev()))
    assert out["rc"] == oa.ENAN
    Ap = T(p1.on_pattern(A, csr_host(pat)))
    out = oa.bicgstab(pat.with_values(Ap), T(b), T(st.U1), rtol=1e-12, maxit=1)
    assert all(o["status"] == oa.ENOTCONV for o in out)
    # zero diagonal: Jacobi is undefined -> EINVAL before any iteration
    with pytest.raises(oa.OasisError):
        oa.pcg(pat.with_values(torch.zeros_like(Kp)), T(bphi), torch.zeros_like(Kp[: prob.mesh.n_dof]))


def _run_gpu_steps(oa, prob, steps, rtol, precision=0, guess=None, assembly=0):
    m = prob.mesh
    dm, pat, _ = device_mesh(m)
    h = oa.IPCS(dm, pat, prob.dt, prob.nu, prob.f, T(m.bc_dofs, torch.int32), rtol_u=rtol, rtol_p=rtol,
                precision=precision, assembly=assembly)
    U = [T(prob.U2), T(prob.U1)]
    p, phi = T(prob.p), T(prob.phi_prev)
    UI = torch.empty_like(U[0])
    bphi = torch.empty_like(p)
    t = prob.t0
    stats = []
    for n in range(steps):
        t += prob.dt
        Un = torch.empty_like(U[0])
        bc = T(prob.bc_values(t)) if m.bc_dofs.size else None
        stats.append(h.step(U[1], U[0], Un, p, phi, bc_values=bc, UI=UI, b_phi=bphi))
        U = [U[1], Un]
    torch.cuda.synchronize()
    return h, U[1], p, phi, UI, bphi, stats


@pytest.mark.parametrize("assembly", [0, 1], ids=["rows", "colours"])
@pytest.mark.parametrize("prob", [synth.taylor_green(16), synth.channel_flow("tiny", seed=2),
                                  synth.channel_flow("small", seed=4, displace_seed=9),
                                  synth.channel_flow("small", seed=5, displace_seed=9, permute_seed=77)],
                         ids=lambda p: p.name)
def test_ipcs_step_matches_oracle(oa, prob, assembly):
    """One step against the oracle; the last mesh has randomly numbered
    dofs, vertices and cells (the row kernels walk their own
    locality-ordered copy of it)."""
    say("ipcs step", prob.name, "assembly", assembly)
    h, Un, p, phi, UI, bphi, stats = _run_gpu_steps(oa, prob, 1, 1e-13, assembly=assembly)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    ref = ipcs.step(S, ipcs.initial_state(prob), prob.bc_values, rtol_u=1e-13, rtol_p=1e-13)
    assert rel(UI.cpu().numpy(), ref.UI) <= 1e-10
    assert rel(bphi.cpu().numpy(), ref.b_phi) <= 1e-10
    assert rel(phi.cpu().numpy(), ref.phi) <= 1e-10
    assert rel(p.cpu().numpy(), ref.state.p) <= 1e-10
    assert rel(Un.cpu().numpy(), ref.state.U1) <= 1e-10
    assert stats[0]["status"] == 0


def test_ipcs_ten_steps_channel(oa):
    prob = synth.channel_flow("tiny", seed=6)
    say("ipcs 10 steps", prob.name)
    h, Un, p, phi, UI, bphi, stats = _run_gpu_steps(oa, prob, 10, 1e-13)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    st = ipcs.initial_state(prob)
    for _ in range(10):
        st = ipcs.step(S, st, prob.bc_values, rtol_u=1e-13, rtol_p=1e-13).state
    assert rel(Un.cpu().numpy(), st.U1) <= 1e-10
    assert rel(p.cpu().numpy(), st.p) <= 1e-10


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_pcg_kernel_timing_leaves_the_solve_unchanged(oa, precision):
    """The timing mode repeats the last product launch after a solve that
    stopped at maxit: it reports maxit timed launches and the returned x is
    bit-for-bit that of an untimed solve."""
    prob = synth.channel_flow("small", seed=3)
    say("pcg timing", prob.name, precision)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Kp = pat.with_values(T(p1.on_pattern(S.K, csr_host(pat))))
    rng = np.random.default_rng(12)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    prec = oa.F64 if precision == "f64" else oa.F32
    outs, xs = [], []
    for timed in (False, True):
        x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev())
        outs.append(oa.pcg(Kp, T(bphi), x, rtol=1e-30, maxit=40, precision=prec, time_kernel=timed,
                           raise_on=False, nullspace_const=True))
        xs.append(x)
    assert outs[0]["rc"] == oa.ENOTCONV and outs[1]["rc"] == oa.ENOTCONV
    assert outs[0]["kernel_count"] == 0
    assert outs[1]["kernel_count"] == 40 and outs[1]["kernel_ms"] > 0
    assert torch.equal(xs[0], xs[1])
    assert outs[0]["iters"] == outs[1]["iters"] == 40


# ---------------------------------------------------------------------------
# mixed precision: FP32 iterations, FP64 refinement.  The answer is any x
# whose FP64 true residual meets rtol; the oracle recomputes that residual
# from the GPU output and compares with its own FP64 solve.

@pytest.mark.parametrize("prob", [synth.channel_flow("small", seed=3), synth.channel_flow((33, 33, 25), seed=1)],
                         ids=lambda p: p.name)
def test_pcg_mixed_meets_fp64_tolerance(oa, prob):
    say("pcg mixed", prob.name)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Kp = p1.on_pattern(S.K, csr_host(pat))
    rng = np.random.default_rng(8)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    ref = krylov.pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-8)
    x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev())
    out = oa.pcg(pat.with_values(T(Kp)), T(bphi), x, rtol=1e-8, precision=oa.F32, nullspace_const=True)
    xg = x.cpu().numpy()
    true = np.linalg.norm(bphi - S.K @ xg) / np.linalg.norm(bphi)
    assert out["rc"] == 0 and true <= 1.0001e-8, (out, true)
    assert out["outer_iters"] >= 1
    assert out["iters"] <= 1.5 * ref.iters + 20, (out["iters"], ref.iters)
    xr = ref.x - ref.x.mean()
    assert rel(xg - xg.mean(), xr) < 1e-5
    # the same reliable-update scheme in the oracle (FP32 recurrences, FP64
    # replacements): iteration counts agree up to FP32 summation order
    rr = mixed.reliable_pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-8, delta=0.1)
    say("mixed PCG iterations: GPU %d, oracle reliable-update %d, FP64 %d" % (out["iters"], rr.iters, ref.iters))
    assert rr.status == krylov.OK
    assert abs(out["iters"] - rr.iters) <= 0.15 * rr.iters + 5, (out["iters"], rr.iters)


def test_pcg_mixed_several_rows_per_lane_group(oa):
    """The FP32 CG iteration walks its rows in a two-stage software pipeline,
    unrolled twice, with the next row's fetch clamped into the lane group's
    range.  At the default grid the test meshes give each lane group at most
    one row per launch; a 64-block grid (the tuning's grid_cap)
    gives the 33x33x25 channel's groups 3 or 4 rows each, so both halves of
    the unrolled loop and the clamped fetch past a range's end run.  The
    solve must meet the FP64 tolerance against the oracle as at the default
    grid, with the same iteration count up to the partial-sum order."""
    prob = synth.channel_flow((33, 33, 25), seed=1)
    say("pcg mixed, 64-block grid", prob.name)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Kp = pat.with_values(T(p1.on_pattern(S.K, csr_host(pat))))
    rng = np.random.default_rng(12)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    ref = krylov.pcg(S.K, bphi, np.zeros_like(bphi), rtol=1e-8)
    outs, xs = [], []
    for grid in (0, 64):
        x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev())
        outs.append(oa.pcg(Kp, T(bphi), x, rtol=1e-8, precision=oa.F32, nullspace_const=True, grid_cap=grid))
        xs.append(x.cpu().numpy())
    xr = ref.x - ref.x.mean()
    for out, xg in zip(outs, xs):
        true = np.linalg.norm(bphi - S.K @ xg) / np.linalg.norm(bphi)
        assert out["rc"] == 0 and true <= 1.0001e-8, (out, true)
        assert rel(xg - xg.mean(), xr) < 1e-5
    assert abs(outs[0]["iters"] - outs[1]["iters"]) <= max(3, outs[0]["iters"] // 50), \
        (outs[0]["iters"], outs[1]["iters"])


def test_pcg_mixed_without_null_vector(oa):
    """FP32 CG iterations on an SPD matrix without a null space (K + M): the
    single-reduction kernel then reads the Jacobi norm weights instead of
    forming them from a null vector, and projects nothing.  At the default
    grid and at a 64-block grid (3-4 rows per lane group) the solve must meet
    the FP64 tolerance in the oracle's residual and match the oracle's FP64
    solution."""
    prob = synth.channel_flow((33, 33, 25), seed=4)
    say("pcg mixed, no null vector", prob.name)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    Am = (S.K + S.M).tocsr()
    dm, pat, _ = device_mesh(prob.mesh)
    Ap = pat.with_values(T(p1.on_pattern(Am, csr_host(pat))))
    rng = np.random.default_rng(16)
    bv = rng.normal(size=prob.mesh.n_dof)
    ref = krylov.pcg(Am, bv, np.zeros_like(bv), rtol=1e-8)
    iters = []
    for grid in (0, 64):
        x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev())
        out = oa.pcg(Ap, T(bv), x, rtol=1e-8, precision=oa.F32, grid_cap=grid)
        xg = x.cpu().numpy()
        true = np.linalg.norm(bv - Am @ xg) / np.linalg.norm(bv)
        assert out["rc"] == 0 and true <= 1.0001e-8, (grid, out, true)
        assert rel(xg, ref.x) < 1e-6
        iters.append(out["iters"])
    assert abs(iters[0] - iters[1]) <= max(3, iters[0] // 50), iters


def test_products_several_rows_per_lane_group(oa):
    """BiCGStab (both precisions) and the FP64 PCG run their ELL products in
    the same straight-line row loops as the FP32 CG iteration.  With the
    producer grid cut to 64 blocks (the tuning's grid_cap) the
    33x33x25 channel gives each lane group 3 or 4 rows, so both halves of
    the unrolled loops and the clamped fetches run; the solves must meet
    their tolerances in the oracle's own residual and agree with the solves
    at the default grid."""
    prob = synth.channel_flow((33, 33, 25), seed=3)
    say("products, 64-block grid", prob.name)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Ap = pat.with_values(T(p1.on_pattern(A, csr_host(pat))))
    Kp = pat.with_values(T(p1.on_pattern(S.K, csr_host(pat))))
    rng = np.random.default_rng(14)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()

    def solves(grid):
        res = []
        for prec in (oa.F64, oa.F32):
            x = T(st.U1)
            out = oa.bicgstab(Ap, T(b), x, rtol=1e-10, precision=prec, grid_cap=grid)
            res.append((out, x.cpu().numpy()))
        x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev())
        out = oa.pcg(Kp, T(bphi), x, rtol=1e-10, nullspace_const=True, grid_cap=grid)
        res.append((out, x.cpu().numpy()))
        return res

    cut = solves(64)
    ref = solves(0)
    for (out, x), (rout, rx) in zip(cut[:2], ref[:2]):
        for k in range(3):
            true = np.linalg.norm(b[k] - A @ x[k]) / np.linalg.norm(b[k])
            assert out[k]["status"] == 0 and true <= 1.0001e-10, (k, out[k], true)
            assert rel(x[k], rx[k]) < 1e-7
    out, x = cut[2]
    true = np.linalg.norm(bphi - S.K @ x) / np.linalg.norm(bphi)
    assert out["rc"] == 0 and true <= 1.0001e-10, (out, true)
    assert abs(out["iters"] - ref[2][0]["iters"]) <= max(3, out["iters"] // 50)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_pcg_poll_schedule_does_not_change_the_solve(oa, precision):
    """The host polls the device-side convergence state between chunks of
    launched iterations (sized from the observed convergence rate by
    default, or every check_every iterations); launches after a raised flag
    return at once, so the iterate, the iteration count and the replacement
    count must be bit-for-bit the same for any schedule."""
    prob = synth.channel_flow((33, 33, 25), seed=2)
    say("pcg poll schedule", prob.name, precision)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Kp = pat.with_values(T(p1.on_pattern(S.K, csr_host(pat))))
    rng = np.random.default_rng(31)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    prec = oa.F64 if precision == "f64" else oa.F32
    outs, xs = [], []
    for every in (0, 1, 7, 64):
        x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=dev())
        outs.append(oa.pcg(Kp, T(bphi), x, rtol=1e-9, precision=prec, nullspace_const=True, check_every=every))
        xs.append(x)
    for o, x in zip(outs[1:], xs[1:]):
        assert o["rc"] == outs[0]["rc"] == 0
        assert o["iters"] == outs[0]["iters"] and o["restarts"] == outs[0]["restarts"], (o, outs[0])
        assert torch.equal(x, xs[0])


def test_bicgstab_mixed_meets_fp64_tolerance(oa):
    prob = synth.channel_flow("small", seed=5)
    say("bicgstab mixed", prob.name)
    S, st, A, b = _tent_problem(prob)
    dm, pat, _ = device_mesh(prob.mesh)
    Ap = p1.on_pattern(A, csr_host(pat))
    x = T(st.U1)
    out = oa.bicgstab(pat.with_values(T(Ap)), T(b), x, rtol=1e-10, precision=oa.F32)
    for k in range(3):
        xg = x[k].cpu().numpy()
        true = np.linalg.norm(b[k] - A @ xg) / np.linalg.norm(b[k])
        assert out[k]["status"] == 0 and true <= 1.0001e-10, (k, out[k], true)


def test_ipcs_mixed_steps_close_to_fp64(oa):
    prob = synth.channel_flow((33, 33, 25), seed=2)
    say("ipcs mixed", prob.name)
    h, Un, p, phi, UI, bphi, stats = _run_gpu_steps(oa, prob, 3, 1e-8, precision=1)
    assert all(s["status"] == 0 for s in stats)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    st = ipcs.initial_state(prob)
    for _ in range(3):
        st = ipcs.step(S, st, prob.bc_values, rtol_u=1e-12, rtol_p=1e-12).state
    assert rel(Un.cpu().numpy(), st.U1) < 1e-6
    assert rel(p.cpu().numpy(), st.p) < 1e-5
    # the last pressure solve met the FP64 tolerance on the oracle's matrix
    ph = phi.cpu().numpy()
    bp = bphi.cpu().numpy()
    assert np.linalg.norm(bp - S.K @ ph) <= 1.0001e-8 * np.linalg.norm(bp)
