"""The learned warm start inside the IPCS step.

* The guard: a caller guess is taken only when its CG energy is below that
  of the plain start (phi_prev, or phi_0 = 0); the converged correction of
  the oracle is taken and leaves almost nothing to iterate, a useless one
  is refused and the step is then identical to the plain step.
* The phi_0 = 0 start matches the oracle's zero start.
* The trained networks (packaged weights, one trained on the K-norm of the
  error, one on the mean squared error of the scaled correction): on a
  held-out seeded channel run each must lower the loss it was trained on
  well below that of phi_prev, every warm-started step must reach the same
  tolerance as the plain one, and where the guard refuses the guess the
  iteration count must equal the plain one.  The K-norm network's guess
  must pass the energy guard on most steps and, with the multigrid
  preconditioner, not need more iterations than phi_prev.  The measured
  change in PCG iterations and pressure-solve time is printed.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import T, dev, device_mesh, rel, say
from oracle import ipcs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_1602_03643_amd as m
    return m


def _handle(oa, prob, dm, pat, precision=0, rtol=1e-10, pstart=0):
    m = prob.mesh
    return oa.IPCS(dm, pat, prob.dt, prob.nu, prob.f, T(m.bc_dofs, torch.int32), rtol_u=rtol, rtol_p=rtol,
                   precision=precision, pressure_start=pstart)


def _state(prob):
    return dict(U1=T(prob.U1), U2=T(prob.U2), p=T(prob.p), phi=T(prob.phi_prev),
                bc=T(prob.bc_values(prob.t0 + prob.dt)))


def _step(h, st, guess=None):
    Un = torch.empty_like(st["U1"])
    r = h.step(st["U1"], st["U2"], Un, st["p"], st["phi"], bc_values=st["bc"], phi_guess=guess)
    st["U2"], st["U1"] = st["U1"], Un
    return r


@pytest.mark.parametrize("pstart", [0, 1], ids=["prev", "zero"])
def test_guard_takes_good_guess_and_refuses_bad_one(oa, pstart):
    prob = synth.channel_flow("tiny", seed=11)
    say("warm start guard", prob.name, "pressure start", pstart)
    dm, pat, _ = device_mesh(prob.mesh)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    ref = ipcs.step(S, ipcs.initial_state(prob), prob.bc_values, rtol_u=1e-12, rtol_p=1e-12)
    h = _handle(oa, prob, dm, pat, pstart=pstart)
    a, b, c = _state(prob), _state(prob), _state(prob)
    plain = _step(h, a)
    good = _step(h, b, guess=T(ref.phi))
    bad = _step(h, c, guess=T(ref.phi * 50.0 + 1.0))
    assert plain["guess_used"] == 0
    assert good["guess_used"] == 1 and good["iters_p"] < 0.2 * plain["iters_p"], (good, plain)
    assert bad["guess_used"] == 0 and bad["iters_p"] == plain["iters_p"]
    assert torch.equal(c["phi"], a["phi"]) and torch.equal(c["U1"], a["U1"])
    for st in (a, b):
        assert rel(st["phi"].cpu().numpy(), ref.phi) < 1e-8
        assert rel(st["U1"].cpu().numpy(), ref.state.U1) < 1e-8


def test_zero_pressure_start_matches_oracle(oa):
    prob = synth.channel_flow("tiny", seed=13)
    say("zero pressure start", prob.name)
    dm, pat, _ = device_mesh(prob.mesh)
    S = ipcs.setup(prob.mesh, prob.nu, prob.dt, prob.f)
    st = ipcs.initial_state(prob)
    h = _handle(oa, prob, dm, pat, rtol=1e-13, pstart=1)
    g = _state(prob)
    for _ in range(3):          # phi_prev is nonzero from the second step on
        ref = ipcs.step(S, st, prob.bc_values, rtol_u=1e-13, rtol_p=1e-13, pressure_start="zero")
        r = _step(h, g)
        assert r["status"] == 0
        assert rel(g["phi"].cpu().numpy(), ref.phi) <= 1e-10
        assert rel(g["p"].cpu().numpy(), ref.state.p) <= 1e-10
        assert rel(g["U1"].cpu().numpy(), ref.state.U1) <= 1e-10
        st = ref.state


def test_random_network_never_breaks_the_step(oa):
    from paper_1602_03643_amd import warmstart
    prob = synth.channel_flow("tiny", seed=12)
    say("warm start random net", prob.name)
    dm, pat, _ = device_mesh(prob.mesh)
    P = warmstart.init_params(5)
    P[-33:] = np.random.default_rng(5).normal(size=33).astype(np.float32)   # nonzero decoder
    plain, warm = _handle(oa, prob, dm, pat), _handle(oa, prob, dm, pat)
    warm.set_warmstart(torch.as_tensor(P, device=dev()), T(prob.mesh.dof_coords))
    a, b = _state(prob), _state(prob)
    for _ in range(3):
        ra, rb = _step(plain, a), _step(warm, b)
        assert ra["status"] == 0 and rb["status"] == 0
        assert rb["res_p"] <= 1e-10 * 1.0001
        if not rb["guess_used"]:
            assert rb["iters_p"] == ra["iters_p"]
        assert rel(b["phi"].cpu().numpy(), a["phi"].cpu().numpy()) < 1e-6
    warm.set_warmstart(None, None)
    rb = _step(warm, b)
    assert rb["guess_used"] == 0


@pytest.mark.parametrize("which", ["knorm", "mse"])
def test_trained_network_gain_on_held_out_run(oa, which):
    from paper_1602_03643_amd import warmstart
    P, meta = warmstart.load(warmstart.DEFAULT_WEIGHTS if which == "knorm" else warmstart.MSE_WEIGHTS)
    kind = warmstart.loss_kind(meta)
    assert kind == (oa.MPNN_LOSS_KNORM if which == "knorm" else oa.MPNN_LOSS_MSE)
    size, steps, seed = "c65", 8, 97           # seed far outside the training seeds
    say("trained warm start", which, size, "seed", seed, "weights trained on", meta["sizes"])
    case = warmstart.Case(size, dev())
    Pt = torch.as_tensor(P, device=dev())
    st = case.initial(seed)
    data = warmstart.collect(case.h, st, steps)
    samples = [(case.net,) + d for d in data]
    l_prev = warmstart.eval_loss(samples, torch.as_tensor(warmstart.init_params(0), device=dev()), kind)
    l_net = warmstart.eval_loss(samples, Pt, kind)
    say("held-out %s loss: guess = phi_prev %.3f, trained network %.3f" % (which, l_prev, l_net))
    assert l_net < (0.3 if which == "knorm" else 0.6) * l_prev
    for amg in [False, True]:
        c = warmstart.compare(case, Pt, seed=seed, steps=steps, amg=amg)
        say("%s: PCG iterations plain %.1f, warm %.1f (guess used in %.0f%% of steps); pressure ms %.2f vs %.2f"
            % ("multigrid" if amg else "Jacobi", c["iters_plain"], c["iters_warm"], 100 * c["guess_used"],
               c["ms_pressure_plain"], c["ms_pressure_warm"]))
        assert c["rel_diff_phi"] < 1e-5
        if c["guess_used"] == 0.0:
            assert c["iters_warm"] == c["iters_plain"]
        if which == "knorm":
            assert c["guess_used"] >= 0.5
            if amg:
                assert c["iters_warm"] <= c["iters_plain"]
