"""ELL column storage of the Krylov products.

On the structured channel mesh the rows share few distinct lists of column
offsets (27 at every size: interior rows, the two walls, the periodic
seams and their intersections), so the products read the offsets through a
per-row dictionary id instead of per entry.  Both forms name the same
columns in the same order, so every solve must be bit-for-bit identical
with the dictionary switched off (storage OASIS_STORAGE_ELL), and
the solvers must report which storage they used.  A relabelled mesh whose
rows have as many offset lists as rows keeps the per-entry offsets.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import T, csr_host, device_mesh, say
from oracle import ipcs, p1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_1602_03643_amd as m
    return m


def _storage(oa, on):
    return oa.STORAGE_AUTO if on else oa.STORAGE_ELL


def _problem(mesh_seed=3, permute=None):
    prob = synth.channel_flow("small", seed=mesh_seed)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    st = ipcs.initial_state(prob)
    A, b = ipcs.tentative_system(S, st, prob.t0 + prob.dt, prob.bc_values(prob.t0 + prob.dt))
    return prob, S, A, b


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_pcg_dictionary_is_bit_identical(oa, precision):
    prob, S, _, _ = _problem()
    say("ell dictionary pcg", prob.name, precision)
    dm, pat, _ = device_mesh(prob.mesh)
    K = pat.with_values(T(p1.on_pattern(S.K, csr_host(pat))))
    rng = np.random.default_rng(21)
    bphi = rng.normal(size=prob.mesh.n_dof)
    bphi -= bphi.mean()
    prec = oa.F64 if precision == "f64" else oa.F32
    outs, xs = [], []
    for on in (True, False):
        x = torch.zeros(prob.mesh.n_dof, dtype=torch.float64, device=T(0.0).device)
        outs.append(oa.pcg(K, T(bphi), x, rtol=1e-10, precision=prec, nullspace_const=True,
                           storage=_storage(oa, on)))
        xs.append(x)
    assert 0 < outs[0]["ell_patterns"] <= 64, outs[0]
    assert outs[1]["ell_patterns"] == -1, outs[1]
    assert outs[0]["rc"] == outs[1]["rc"] == 0
    assert outs[0]["iters"] == outs[1]["iters"]
    assert torch.equal(xs[0], xs[1])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_bicgstab_dictionary_is_bit_identical(oa, precision):
    prob, S, A, b = _problem()
    say("ell dictionary bicgstab", prob.name, precision)
    dm, pat, _ = device_mesh(prob.mesh)
    Ap = pat.with_values(T(p1.on_pattern(A, csr_host(pat))))
    prec = oa.F64 if precision == "f64" else oa.F32
    outs, xs = [], []
    for on in (True, False):
        x = T(np.zeros_like(b))
        outs.append(oa.bicgstab(Ap, T(b), x, rtol=1e-10, precision=prec, storage=_storage(oa, on)))
        xs.append(x)
    for k in range(b.shape[0]):
        assert 0 < outs[0][k]["ell_patterns"] <= 64 and outs[1][k]["ell_patterns"] == -1
        assert outs[0][k]["iters"] == outs[1][k]["iters"]
    assert torch.equal(xs[0], xs[1])


def test_ipcs_step_dictionary_is_bit_identical(oa):
    prob = synth.channel_flow("small", seed=5)
    say("ell dictionary ipcs", prob.name)
    dm, pat, _ = device_mesh(prob.mesh)
    m = prob.mesh
    res = []
    for on in (True, False):
        for prec in (oa.F64, oa.F32):
            h = oa.IPCS(dm, pat, prob.dt, prob.nu, prob.f, T(m.bc_dofs, torch.int32), rtol_u=1e-10,
                        rtol_p=1e-10, precision=prec, storage=_storage(oa, on))
            U1, U2, p, phi = T(prob.U1), T(prob.U2), T(prob.p), T(prob.phi_prev)
            bc = T(prob.bc_values(prob.t0 + prob.dt))
            for _ in range(2):
                Un = torch.empty_like(U1)
                st = h.step(U1, U2, Un, p, phi, bc_values=bc)
                assert st["status"] == 0
                U2, U1 = U1, Un
            res.append((U1, p, phi, st["iters_p"], st["iters_u"]))
    for a, b in ((res[0], res[2]), (res[1], res[3])):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
        assert a[3] == b[3] and list(a[4]) == list(b[4])


def test_relabelled_mesh_keeps_per_entry_offsets(oa):
    mesh, _ = synth.permute_mesh(synth.channel(17, 17, 13), 9)
    say("ell per-entry offsets", mesh.name)
    dm, pat, _ = device_mesh(mesh)
    geo = p1.element_geometry(mesh)
    K = pat.with_values(T(p1.on_pattern(p1.stiffness_matrix(mesh, geo), csr_host(pat))))
    rng = np.random.default_rng(2)
    bphi = rng.normal(size=mesh.n_dof)
    bphi -= bphi.mean()
    x = T(np.zeros(mesh.n_dof))
    out = oa.pcg(K, T(bphi), x, rtol=1e-8, nullspace_const=True)
    # a random relabelling leaves nearly every row with its own offset list,
    # more than the n / 8 a dictionary may hold
    assert out["rc"] == 0
    assert out["ell_patterns"] == -1, out
