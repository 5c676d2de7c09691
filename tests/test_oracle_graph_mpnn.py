"""Pins for the oracle's reordering, colouring and warm-start network.

RCM is pinned by properties that characterise a Cuthill-McKee sequence (a
bijection; breadth-first levels appear in non-decreasing order; every
vertex after a component root has an earlier neighbour; siblings appear in
(degree, index) order) and by the known answer on a scrambled path graph.
Greedy colouring is pinned by validity and by the first-fit property.
The network's backward pass is pinned by central finite differences.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import graph, ipcs, mpnn


def test_rcm_on_scrambled_path():
    n = 12
    rng = np.random.default_rng(0)
    lab = rng.permutation(n)
    rows, cols = [], []
    for i in range(n - 1):
        a, b = lab[i], lab[i + 1]
        rows += [a, b, a, b]
        cols += [b, a, a, b]
    A = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    A.sort_indices()
    order, perm = graph.rcm(A.indptr, A.indices)
    assert sorted(order.tolist()) == list(range(n))
    assert graph.bandwidth(A.indptr, A.indices, perm) == 1
    # the path end with the smaller label is the pseudo-peripheral root, placed last
    ends = sorted([lab[0], lab[-1]])
    assert order[-1] == ends[0]


@pytest.mark.parametrize("prob", [synth.channel_flow("tiny", permute_seed=2000),
                                  synth.channel_flow("small", permute_seed=2000, displace_seed=1000)],
                         ids=lambda p: p.name)
def test_rcm_is_a_cuthill_mckee_sequence(prob):
    rp, ci = graph.csr_pattern(prob.mesh)
    order, perm = graph.rcm(rp, ci)
    n = rp.size - 1
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(perm[order], np.arange(n))
    cm = order[::-1]
    pos = np.empty(n, np.int64)
    pos[cm] = np.arange(n)
    deg = np.diff(rp)
    root = cm[0]
    # BFS distance from the root is non-decreasing along the sequence
    dist = np.full(n, -1)
    dist[root] = 0
    frontier = [root]
    while frontier:
        nxt = []
        for u in frontier:
            for v in ci[rp[u]:rp[u + 1]]:
                if dist[v] < 0:
                    dist[v] = dist[u] + 1
                    nxt.append(v)
        frontier = nxt
    assert np.all(np.diff(dist[cm]) >= 0)
    # parent = earliest neighbour; children of one parent sorted by (deg, index)
    parent = np.array([min((pos[v] for v in ci[rp[u]:rp[u + 1]] if v != u), default=-1) for u in cm])
    parent[0] = -1                                    # the root has no parent
    for k in range(1, n):
        assert parent[k] < k
        if parent[k] == parent[k - 1]:
            a, b = cm[k - 1], cm[k]
            assert (deg[a], a) < (deg[b], b)
        else:
            assert parent[k] > parent[k - 1]
    # bandwidth no worse than 1.5x the lexicographic structured numbering
    nx, ny, nz = prob.mesh.name.split("_")[1].split("x")[:3]
    nat = synth.channel(int(nx), int(ny), int(nz.split("_")[0]))
    rpn, cin = graph.csr_pattern(nat)
    assert graph.bandwidth(rp, ci, perm) <= 1.5 * graph.bandwidth(rpn, cin)


def test_greedy_coloring_is_valid_first_fit():
    m = synth.channel(9, 9, 7)
    pri = synth.cell_priorities(m.n_cell, 7)
    color = graph.greedy_coloring(m, pri)
    assert color.min() == 0
    assert graph.coloring_conflicts(m, color) == 0
    dofs = m.vert2dof[m.cells]
    inc = [[] for _ in range(m.n_dof)]
    for c in range(m.n_cell):
        for v in dofs[c]:
            inc[v].append(c)
    for c in range(m.n_cell):
        higher = {int(color[o]) for v in dofs[c] for o in inc[v] if o != c and pri[o] > pri[c]}
        assert all(k in higher for k in range(color[c]))      # first fit
    ptr, cells = graph.color_classes(color)
    assert ptr[-1] == m.n_cell and np.array_equal(np.sort(cells), np.arange(m.n_cell))
    for k in range(ptr.size - 1):
        seg = cells[ptr[k]:ptr[k + 1]]
        assert np.all(color[seg] == k) and np.all(np.diff(seg) > 0)


def _mpnn_problem():
    pr = synth.channel_flow("tiny", seed=2)
    S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
    out = ipcs.step(S, ipcs.initial_state(pr), pr.bc_values)
    rng = np.random.default_rng(4)
    phi_prev = out.phi + 0.1 * rng.normal(size=out.phi.size) * np.abs(out.phi).max()
    return S, out, phi_prev


@pytest.mark.parametrize("kind", ["mse", "knorm"])
def test_mpnn_backward_matches_finite_differences(kind):
    S, out, phi_prev = _mpnn_problem()
    X, sigma = mpnn.features(S.K, out.b_phi, phi_prev, S.mesh.dof_coords)
    W = mpnn.edge_weights(S.K)
    P = mpnn.init_params(1)
    rng = np.random.default_rng(6)
    P["wd"] = rng.normal(size=mpnn.HID) * 0.3
    P["c"] = rng.normal(size=P["c"].shape) * 0.1
    target = (out.phi - phi_prev) / sigma
    delta, cache = mpnn.forward(P, X, W)
    G = mpnn.backward(P, cache, delta, target, W, kind, S.K)
    h = 1e-6
    for name in ["We", "ce", "Ws", "Wn", "c", "wd", "cd"]:
        flat = P[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mpnn.loss(mpnn.forward(P, X, W)[0], target, kind, S.K)
            flat[i] = old - h
            lm = mpnn.loss(mpnn.forward(P, X, W)[0], target, kind, S.K)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = G[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (name, i, fd, an)


def test_mpnn_zero_decoder_is_fallback_and_guard():
    S, out, phi_prev = _mpnn_problem()
    P = mpnn.init_params(0)                # wd = 0, cd = 0
    g = mpnn.predict_guess(P, S.K, out.b_phi, phi_prev, S.mesh.dof_coords)
    np.testing.assert_array_equal(g, phi_prev)
    bad = phi_prev + 1e6
    bad[0] = np.nan
    x0, used = mpnn.guarded_start(S.K, out.b_phi, phi_prev, bad)
    assert not used and x0 is phi_prev                  # falls back to the plain start
    zero = np.zeros_like(phi_prev)
    x0, used = mpnn.guarded_start(S.K, out.b_phi, zero, bad)
    assert not used and x0 is zero
    # the converged correction itself has the lowest energy: it is taken
    x0, used = mpnn.guarded_start(S.K, out.b_phi, phi_prev, out.phi)
    assert used and x0 is out.phi


def test_guard_energy_orders_starts_by_their_k_norm_error():
    """J(x) - J(x*) = 1/2 ||x - x*||_K^2: of two starts the guard keeps the
    one closer to the solution in the K-norm (the solution from a dense
    pseudo-inverse, the error norm from K), whatever their residual norms
    say, and is blind to shifts along the null vector 1."""
    S, out, phi_prev = _mpnn_problem()
    K = S.K.toarray()
    b = out.b_phi
    xs = np.linalg.pinv(K) @ b
    rng = np.random.default_rng(11)
    smooth = np.sin(np.pi * S.mesh.dof_coords[:, 1])          # low-frequency error
    rough = rng.standard_normal(b.size)                       # high-frequency error
    knorm = lambda e: e @ (K @ e)  # noqa: E731
    res = lambda x: np.linalg.norm(b - K @ x)  # noqa: E731
    a = xs + 0.3 * smooth / np.sqrt(knorm(smooth))
    c = xs + 0.2 * rough / np.sqrt(knorm(rough))
    assert knorm(c - xs) < knorm(a - xs)
    assert res(c) > res(a)               # the residual norm ranks them the other way
    x0, used = mpnn.guarded_start(S.K, b, a, c)
    assert used and x0 is c
    x0, used = mpnn.guarded_start(S.K, b, c, a)
    assert not used and x0 is c
    x0, used = mpnn.guarded_start(S.K, b, c + 5.0, a)   # a constant shift changes nothing
    assert not used


def test_knorm_loss_is_the_relative_energy_gap():
    """With x* the exact solution (dense pseudo-inverse) and J the CG
    energy, the K-norm loss of a network output delta equals
    (J(phi_prev + sigma delta) - J(x*)) / (J(phi_prev) - J(x*)): 1 for
    delta = 0 (the guess is phi_prev), 0 for the exact correction and for
    it shifted by a constant, and below 1 exactly when the guard would take
    the guess over phi_prev."""
    S, out, phi_prev = _mpnn_problem()
    K = S.K.toarray()
    b = out.b_phi
    xs = np.linalg.pinv(K) @ b
    X, sigma = mpnn.features(S.K, b, phi_prev, S.mesh.dof_coords)
    t = (xs - phi_prev) / sigma
    assert mpnn.loss(np.zeros_like(t), t, "knorm", S.K) == 1.0
    assert abs(mpnn.loss(t, t, "knorm", S.K)) < 1e-20
    assert abs(mpnn.loss(t + 3.7, t, "knorm", S.K)) < 1e-10
    rng = np.random.default_rng(12)
    gap = lambda x: mpnn.energy(S.K, b, x) - mpnn.energy(S.K, b, xs)  # noqa: E731
    for scale in [0.05, 0.5, 2.0]:
        d = t + scale * rng.standard_normal(t.size)
        lk = mpnn.loss(d, t, "knorm", S.K)
        ratio = gap(phi_prev + sigma * d) / gap(phi_prev)
        assert abs(lk - ratio) <= 1e-8 * max(1.0, ratio), (scale, lk, ratio)
        _, used = mpnn.guarded_start(S.K, b, phi_prev, phi_prev + sigma * d)
        assert used == (lk < 1.0)
    # the MSE loss does not rank guesses this way: a rough error of small
    # MSE can cost more energy than a smooth one of larger MSE
    smooth = np.sin(np.pi * S.mesh.dof_coords[:, 1])
    rough = rng.standard_normal(t.size)
    a = t + 0.3 * smooth / np.sqrt(np.mean(smooth ** 2))
    c = t + 0.2 * rough / np.sqrt(np.mean(rough ** 2))
    assert mpnn.loss(c, t) < mpnn.loss(a, t)
    assert mpnn.loss(c, t, "knorm", S.K) > mpnn.loss(a, t, "knorm", S.K)


def test_mpnn_training_reduces_loss():
    S, out, phi_prev = _mpnn_problem()
    X, sigma = mpnn.features(S.K, out.b_phi, phi_prev, S.mesh.dof_coords)
    W = mpnn.edge_weights(S.K)
    target = (out.phi - phi_prev) / sigma
    P = mpnn.init_params(3)
    opt = mpnn.Adam(P, lr=3e-3)
    l0 = mpnn.loss(mpnn.forward(P, X, W)[0], target)
    for _ in range(60):
        d, c = mpnn.forward(P, X, W)
        opt.step(P, mpnn.backward(P, c, d, target, W))
    l1 = mpnn.loss(mpnn.forward(P, X, W)[0], target)
    assert l1 < 0.5 * l0


def test_adam_matches_torch_optim_adam():
    """The oracle's Adam (Kingma & Ba, Algorithm 1: bias-corrected moments,
    eps added to sqrt of the second moment) against torch.optim.Adam, an
    implementation written independently of the oracle, over several steps
    with gradients that change sign and scale."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    P = {"a": rng.normal(size=(4, 3)), "b": rng.normal(size=5)}
    lr, b1, b2, eps = 3e-2, 0.8, 0.95, 1e-3     # non-default values expose swapped roles
    opt = mpnn.Adam({k: v.copy() for k, v in P.items()}, lr=lr, b1=b1, b2=b2, eps=eps)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    topt = torch.optim.Adam(list(tp.values()), lr=lr, betas=(b1, b2), eps=eps)
    for step in range(5):
        G = {k: rng.normal(size=v.shape) * 10.0 ** (step - 2) for k, v in P.items()}
        P = opt.step(P, G)
        topt.zero_grad()
        for k, t in tp.items():
            t.grad = torch.tensor(G[k], dtype=torch.float64)
        topt.step()
        for k in P:
            np.testing.assert_allclose(P[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)
