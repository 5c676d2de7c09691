"""GPU parity of the warm-start network against the FP64 oracle.

The GPU keeps activations in BF16 and runs the dense layers on MFMA with
FP32 accumulation, so forward outputs and parameter gradients are compared
with a relative L2 tolerance of 3e-2 per tensor (BF16 has an 8-bit
significand; errors compound over 4 layers).  Adam is FP32 elementwise and
matches to 1e-5.  Training on solver-generated pairs must lower the loss.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import T, csr_host, dev, device_mesh, rel, say
from oracle import ipcs, mpnn, p1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_1602_03643_amd as m
    return m


def _flat(P):
    return np.concatenate([np.asarray(P[k], dtype=np.float64).reshape(-1) for k, _ in mpnn.PARAM_SHAPES])


def _unflat(v):
    P, o = {}, 0
    for k, shp in mpnn.PARAM_SHAPES:
        size = int(np.prod(shp))
        P[k] = v[o:o + size].reshape(shp).astype(np.float64)
        o += size
    return P


def _setup(size=(17, 17, 13), seed=2):
    pr = synth.channel_flow(size, seed=seed)
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values, rtol_u=1e-12, rtol_p=1e-12)
    rng = np.random.default_rng(seed)
    phi_prev = out.phi + 0.2 * np.abs(out.phi).max() * rng.normal(size=out.phi.size)
    return pr, S, out, phi_prev


def _gpu_graph(oa, pr, S):
    dm, pat, _ = device_mesh(pr.mesh)
    K = csr_host(pat, T(p1.on_pattern(S.K, csr_host(pat))))
    d = K.diagonal()
    s = np.sqrt(d)
    Ks = (K.multiply(1.0 / s[:, None]).multiply(1.0 / s[None, :])).tocsr()
    Ksp = p1.on_pattern(Ks, csr_host(pat))
    return pat.with_values(T(Ksp)), T(s)


def _params(seed):
    P = mpnn.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    P["wd"] = rng.normal(size=mpnn.HID) * 0.3
    P["cd"] = np.array([0.05])
    P["c"] = rng.normal(size=P["c"].shape) * 0.1
    P["ce"] = rng.normal(size=P["ce"].shape) * 0.1
    return P


def test_mpnn_forward_matches_oracle(oa):
    pr, S, out, phi_prev = _setup()
    say("mpnn forward", pr.name)
    Ks, s = _gpu_graph(oa, pr, S)
    P = _params(1)
    net = oa.MPNN(Ks, s, T(pr.mesh.dof_coords))
    n = pr.mesh.n_dof
    guess = torch.empty(n, dtype=torch.float64, device=dev())
    delta = torch.empty(n, dtype=torch.float32, device=dev())
    net.forward(T(_flat(P), torch.float32), T(out.b_phi), T(phi_prev), guess, delta)
    torch.cuda.synchronize()
    X, sigma = mpnn.features(S.K, out.b_phi, phi_prev, pr.mesh.dof_coords)
    d_ref, _ = mpnn.forward(P, X, mpnn.edge_weights(S.K))
    assert rel(delta.cpu().numpy(), d_ref) < 3e-2
    g_ref = phi_prev + sigma * d_ref
    assert rel(guess.cpu().numpy() - phi_prev, g_ref - phi_prev) < 3e-2
    # zero decoder: the guess is exactly phi_prev
    Z = _params(1)
    Z["wd"][:] = 0.0
    Z["cd"][:] = 0.0
    net.forward(T(_flat(Z), torch.float32), T(out.b_phi), T(phi_prev), guess, delta)
    assert torch.equal(guess, T(phi_prev))


@pytest.mark.parametrize("kind", ["mse", "knorm"])
def test_mpnn_backward_matches_oracle(oa, kind):
    pr, S, out, phi_prev = _setup()
    say("mpnn backward", kind, pr.name)
    Ks, s = _gpu_graph(oa, pr, S)
    P = _params(2)
    net = oa.MPNN(Ks, s, T(pr.mesh.dof_coords))
    n = pr.mesh.n_dof
    pt = T(_flat(P), torch.float32)
    net.forward(pt, T(out.b_phi), T(phi_prev))
    grad = torch.zeros(oa.MPNN.NPARAM, dtype=torch.float32, device=dev())
    code = oa.MPNN_LOSS_KNORM if kind == "knorm" else oa.MPNN_LOSS_MSE
    loss = net.backward(pt, T(out.phi), T(phi_prev), grad, code)
    X, sigma = mpnn.features(S.K, out.b_phi, phi_prev, pr.mesh.dof_coords)
    W = mpnn.edge_weights(S.K)
    d_ref, cache = mpnn.forward(P, X, W)
    target = (out.phi - phi_prev) / sigma
    G = mpnn.backward(P, cache, d_ref, target, W, kind, S.K)
    ref = mpnn.loss(d_ref, target, kind, S.K)
    say("loss", loss, "oracle", ref)
    assert abs(loss / ref - 1.0) < 3e-2
    g = _unflat(grad.cpu().numpy())
    for k, _ in mpnn.PARAM_SHAPES:
        if kind == "knorm" and k == "cd":
            # K 1 = 0: a constant added to delta leaves the K-norm loss
            # unchanged, so the output bias has zero gradient (rounding
            # only on both sides)
            scale = np.linalg.norm(G["wd"])
            assert abs(G["cd"][0]) < 1e-12 * scale and abs(g["cd"][0]) < 1e-5 * scale, (g["cd"], G["cd"])
            continue
        assert rel(g[k], G[k]) < 5e-2, (k, rel(g[k], G[k]))


def test_mpnn_knorm_loss_of_the_zero_decoder_is_one(oa):
    """With a zero decoder the guess is phi_prev (delta = 0), so the K-norm
    loss is exactly t^T K t / t^T K t = 1 and, for phi = phi_prev, the
    degenerate sample gives loss 0 and a zero gradient."""
    pr, S, out, phi_prev = _setup(seed=3)
    Ks, s = _gpu_graph(oa, pr, S)
    Z = _params(4)
    Z["wd"][:] = 0.0
    Z["cd"][:] = 0.0
    net = oa.MPNN(Ks, s, T(pr.mesh.dof_coords))
    pt = T(_flat(Z), torch.float32)
    net.forward(pt, T(out.b_phi), T(phi_prev))
    grad = torch.zeros(oa.MPNN.NPARAM, dtype=torch.float32, device=dev())
    loss = net.backward(pt, T(out.phi), T(phi_prev), grad, oa.MPNN_LOSS_KNORM)
    assert abs(loss - 1.0) < 1e-12
    net.forward(pt, T(out.b_phi), T(out.phi))
    loss = net.backward(pt, T(out.phi), T(out.phi), grad, oa.MPNN_LOSS_KNORM)
    assert loss == 0.0 and not torch.any(grad)
    with pytest.raises(oa.OasisError):
        net.backward(pt, T(out.phi), T(phi_prev), grad, 2)


def test_mpnn_adam_matches_oracle(oa):
    P = _params(3)
    rng = np.random.default_rng(4)
    Gs = [_unflat(rng.normal(size=oa.MPNN.NPARAM)) for _ in range(3)]
    pt = T(_flat(P), torch.float32)
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    opt = mpnn.Adam({k: P[k].copy() for k in P}, lr=1e-3)
    Q = {k: P[k].copy() for k in P}
    for t, G in enumerate(Gs, start=1):
        oa.MPNN.adam(pt, T(_flat(G), torch.float32), m, v, t, lr=1e-3)
        Q = opt.step(Q, G)
    torch.cuda.synchronize()
    assert np.abs(pt.cpu().numpy() - _flat(Q)).max() < 1e-5


def test_mpnn_training_on_gpu_reduces_loss(oa):
    pr, S, out, phi_prev = _setup(seed=5)
    say("mpnn training", pr.name)
    Ks, s = _gpu_graph(oa, pr, S)
    net = oa.MPNN(Ks, s, T(pr.mesh.dof_coords))
    pt = T(_flat(mpnn.init_params(7)), torch.float32)
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    grad = torch.zeros_like(pt)
    b, f, fp = T(out.b_phi), T(out.phi), T(phi_prev)
    losses = []
    for t in range(1, 81):
        net.forward(pt, b, fp)
        losses.append(net.backward(pt, f, fp, grad))
        oa.MPNN.adam(pt, grad, m, v, t, lr=3e-3)
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
