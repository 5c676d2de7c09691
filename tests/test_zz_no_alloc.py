"""oasis_pcg_noalloc (workspace in the library's file-scope device array)
against oasis_pcg (caller workspace) through the C ABI: the same kernels on
the same inputs, so x, the iteration count and the residual must be bit for
bit those of oasis_pcg with the same column storage.  Two calls in a row,
the second on a smaller system, so that the array's contents from the
first call cannot leak into the second; both precisions; and the size
limit is refused with a clear error."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_util import T, csr_host, dev, device_mesh, say
from oracle import ipcs, p1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_1602_03643_amd as m
    return m


def _system(size, seed):
    prob = synth.channel_flow(size, seed=seed)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    dm, pat, _ = device_mesh(prob.mesh, color=False)
    K = pat.with_values(T(p1.on_pattern(S.K, csr_host(pat))))
    rng = np.random.default_rng(seed)
    b = rng.normal(size=prob.mesh.n_dof)
    b -= b.mean()
    return K, T(b)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_pcg_matches_workspace_pcg(oa, precision):
    prec = oa.F64 if precision == "f64" else oa.F32
    for size, seed in (("small", 3), ("tiny", 5)):           # the second system is smaller
        say("pcg_noalloc", size, precision)
        K, b = _system(size, seed)
        x_ws = torch.zeros_like(b)
        x_na = torch.full_like(b, 0.0)
        ref = oa.pcg(K, b, x_ws, rtol=1e-10, precision=prec, nullspace_const=True, storage=oa.STORAGE_ELL)
        out = oa.pcg_noalloc(K, b, x_na, rtol=1e-10, precision=prec, nullspace_const=True)
        assert out["rc"] == ref["rc"] == 0
        assert out["iters"] == ref["iters"] and out["restarts"] == ref["restarts"]
        assert out["rel_res"] == ref["rel_res"]
        assert torch.equal(x_na, x_ws)


def test_noalloc_pcg_refuses_oversized_systems(oa):
    from paper_1602_03643_amd import _lib as L
    K, b = _system("c65", 1)
    o = L.KrylovOpts(1e-8, 100, L.F64, 0.1, 0, 0, 0)
    nb = C.c_size_t()
    assert L.load().oasis_krylov_workspace_size(K.n, K.nnz, 1, C.byref(o), C.byref(nb)) == 0
    assert nb.value > L.PCG_NOALLOC_BYTES
    x = torch.zeros_like(b)
    out = oa.pcg_noalloc(K, b, x, raise_on=False)
    assert out["rc"] == oa.EUNSUPPORTED
    assert torch.count_nonzero(x) == 0
    # timing mode needs events: refused
    with pytest.raises(oa.OasisError):
        o2 = L.KrylovOpts(1e-8, 100, L.F64, 0.1, 0, 0, L.KRYLOV_TIME)
        st = L.KrylovStats()
        K2, b2 = _system("tiny", 2)
        rc = L.load().oasis_pcg_noalloc(None, C.byref(K2.c()), C.c_void_p(b2.data_ptr()),
                                        C.c_void_p(torch.zeros_like(b2).data_ptr()), C.byref(o2), C.byref(st))
        L.check(rc, "oasis_pcg_noalloc")
