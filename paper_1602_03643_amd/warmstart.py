"""Training and evaluation of the learned pressure-correction warm start.

Data are (b_phi, phi_prev, phi) triples produced by the IPCS solver itself
(oasis_ipcs_step with the projected right-hand side requested) on seeded
channel-flow runs; the network is trained on the GPU with
oasis_mpnn_forward / oasis_mpnn_backward / oasis_mpnn_adam.  Nothing here
computes the method: it only drives the C ABI.

    python -m paper_1602_03643_amd.warmstart --sizes c65:40,c129:8 --steps 50 --amg

trains on the listed mesh sizes (size:seeds, `--steps` steps per seed) on
the K-norm loss (or `--loss mse`), validates on held-out seeds, measures the
PCG iterations the attached guess saves against phi_prev on held-out runs
(with Jacobi and, with `--amg`, multigrid preconditioning), and writes
weights/mpnn_channel.npz next to this file (the packaged weights;
weights/mpnn_channel_mse.npz holds a network trained on the mean squared
error).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _lib as L
from .api import IPCS, MPNN, DeviceCSR, DeviceMesh, colorize, p1_pattern

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "mpnn_channel.npz")
MSE_WEIGHTS = os.path.join(HERE, "weights", "mpnn_channel_mse.npz")


def loss_kind(meta):
    """The training loss recorded in a weights file's metadata."""
    return L.MPNN_LOSS_KNORM if meta.get("loss", "mse") == "knorm" else L.MPNN_LOSS_MSE
# flat parameter layout of oasis_mpnn_* (offsets in include/oasis.h)
SHAPES = [("We", (32, 6)), ("ce", (32,)), ("Ws", (3, 32, 32)), ("Wn", (3, 32, 32)), ("c", (3, 32)),
          ("wd", (32,)), ("cd", (1,))]


def init_params(seed=0):
    """He-style encoder, damped message-passing weights, zero biases and a
    zero decoder (so the untrained guess equals phi_prev)."""
    rng = np.random.default_rng(seed)
    parts = {
        "We": rng.normal(0.0, np.sqrt(2.0 / 6), (32, 6)),
        "ce": np.zeros(32),
        "Ws": rng.normal(0.0, 0.5 / np.sqrt(32), (3, 32, 32)),
        "Wn": rng.normal(0.0, 0.5 / np.sqrt(32), (3, 32, 32)),
        "c": np.zeros((3, 32)),
        "wd": np.zeros(32),
        "cd": np.zeros(1),
    }
    flat = np.concatenate([parts[k].reshape(-1) for k, _ in SHAPES]).astype(np.float32)
    assert flat.size == L.MPNN_NPARAM
    return flat


def save(path, params, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=np.asarray(params, np.float32), meta=np.array(json.dumps(meta)))


def load(path=DEFAULT_WEIGHTS):
    """(params float32 [NPARAM], meta dict) from a weights file."""
    with np.load(path, allow_pickle=False) as z:
        p = z["params"].astype(np.float32)
        meta = json.loads(str(z["meta"]))
    if p.size != L.MPNN_NPARAM:
        raise ValueError("%s holds %d parameters, expected %d" % (path, p.size, L.MPNN_NPARAM))
    return p, meta


class Case:
    """One mesh on the device: pattern, colouring, a mixed-precision IPCS
    handle and an MPNN workspace on its scaled pressure matrix."""

    def __init__(self, size, dev, precision=L.F32, seed=0):
        import synth
        self.size = size
        pr = synth.channel_flow(size, seed=seed)
        m = pr.mesh
        self.mesh = m
        self.dt, self.nu, self.f = pr.dt, pr.nu, pr.f
        self.dev = dev
        self.dm = DeviceMesh.from_arrays(m.dim, m.coords, m.cells, m.vert2dof, m.n_dof, dev)
        self.pat = p1_pattern(self.dm)
        colorize(self.dm, torch.as_tensor(synth.cell_priorities(m.n_cell), device=dev))
        self.bc_dofs = torch.as_tensor(m.bc_dofs, device=dev)
        self.h = self.handle(precision)
        Ks, s = self.h.matrix(L.FORM_STIFF)
        self.coords = torch.as_tensor(m.dof_coords, dtype=torch.float64, device=dev).contiguous()
        self.net = MPNN(self.pat.with_values(Ks), s, self.coords)

    def handle(self, precision=L.F32):
        return IPCS(self.dm, self.pat, self.dt, self.nu, self.f, self.bc_dofs, precision=precision)

    def initial(self, seed):
        import synth
        q = synth.channel_flow(self.size, seed=seed)
        T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=self.dev)  # noqa: E731
        return dict(U1=T(q.U1), U2=T(q.U2), p=T(q.p), phi=T(q.phi_prev), bc=T(q.bc_values(0.0)))


def collect(h: IPCS, st, steps):
    """Advance state dict st by `steps` IPCS steps in place; return the
    (b_phi, phi_prev, phi) device triples of every step."""
    out = []
    U2, U1 = st["U2"], st["U1"]
    for _ in range(steps):
        phi_prev = st["phi"].clone()
        bphi = torch.empty_like(phi_prev)
        Un = torch.empty_like(U1)
        r = h.step(U1, U2, Un, st["p"], st["phi"], bc_values=st["bc"], b_phi=bphi)
        if r["status"] != 0:
            raise RuntimeError("solver did not converge while collecting data: %s" % r)
        U2, U1 = U1, Un
        out.append((bphi, phi_prev, st["phi"].clone()))
    st["U2"], st["U1"] = U2, U1
    return out


def train(samples, epochs=3, lr=1e-3, seed=0, params=None, log=None, loss_kind=L.MPNN_LOSS_MSE):
    """samples: [(net, b_phi, phi_prev, phi)]; one Adam step per sample,
    shuffled each epoch, on the loss loss_kind.  Returns (params, mean loss
    per epoch)."""
    dev = samples[0][1].device
    P = torch.as_tensor(init_params(seed) if params is None else params, device=dev).contiguous()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.zeros_like(P)
    rng = np.random.default_rng(seed)
    t = 0
    hist = []
    for ep in range(epochs):
        tot = 0.0
        t0 = time.perf_counter()
        for i in rng.permutation(len(samples)):
            net, b, fp, f = samples[i]
            net.forward(P, b, fp)
            tot += net.backward(P, f, fp, g, loss_kind)
            t += 1
            MPNN.adam(P, g, m, v, t, lr=lr)
        hist.append(tot / len(samples))
        if log:
            log("epoch %d: mean loss %.4g (%.1f s)" % (ep, hist[-1], time.perf_counter() - t0))
    return P, hist


def eval_loss(samples, P, loss_kind=L.MPNN_LOSS_MSE):
    g = torch.zeros_like(P)
    tot = 0.0
    for net, b, fp, f in samples:
        net.forward(P, b, fp)
        tot += net.backward(P, f, fp, g, loss_kind)
    return tot / len(samples)


def compare(case: Case, P, seed, steps, precision=L.F32, amg=False):
    """Run the same seeded trajectory with a plain handle and one with the
    warm start attached, in lockstep; per-step PCG iterations, whether the
    guess was taken, pressure-solve milliseconds and the final difference of
    the two phi fields (both solves stop at the same tolerance).  amg: both
    handles precondition the pressure solve with the multigrid cycle."""
    plain = case.handle(precision)
    warm = case.handle(precision)
    keep = [plain.pressure_amg(precision=precision), warm.pressure_amg(precision=precision)] if amg else []
    warm.set_warmstart(P, case.coords)
    sa, sb = case.initial(seed), case.initial(seed)
    rows = []
    for _ in range(steps):
        ra = _advance(plain, sa)
        rb = _advance(warm, sb)
        rows.append((ra["iters_p"], rb["iters_p"], rb["guess_used"], ra["ms_pressure"], rb["ms_pressure"]))
    a = np.array(rows, dtype=np.float64)
    dphi = float(torch.linalg.vector_norm(sa["phi"] - sb["phi"]) / torch.linalg.vector_norm(sa["phi"]))
    plain.close()
    warm.close()
    del keep
    return dict(size=case.size, seed=seed, steps=steps, amg=amg, iters_plain=float(a[:, 0].mean()),
                iters_warm=float(a[:, 1].mean()), guess_used=float(a[:, 2].mean()),
                ms_pressure_plain=float(a[:, 3].mean()), ms_pressure_warm=float(a[:, 4].mean()),
                rel_diff_phi=dphi)


def _advance(h, st):
    Un = torch.empty_like(st["U1"])
    r = h.step(st["U1"], st["U2"], Un, st["p"], st["phi"], bc_values=st["bc"])
    if r["status"] != 0:
        raise RuntimeError("step did not converge: %s" % r)
    st["U2"], st["U1"] = st["U1"], Un
    return r


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", default="c65:40,c129:8", help="size:training seeds, comma separated")
    ap.add_argument("--val-seeds", type=int, default=2, help="held-out seeds per size")
    ap.add_argument("--steps", type=int, default=50, help="steps per seeded run")
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--compare-steps", type=int, default=20)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--loss", choices=["mse", "knorm"], default="knorm",
                    help="training loss: mean squared error of the scaled correction, or the K-norm of the error")
    ap.add_argument("--amg", action="store_true", help="compare with the multigrid-preconditioned pressure solve too")
    ap.add_argument("--eval", metavar="WEIGHTS", default=None,
                    help="skip training: compare plain and warm-started runs with these weights")
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    kind = L.MPNN_LOSS_KNORM if args.loss == "knorm" else L.MPNN_LOSS_MSE
    sizes = [(s.split(":")[0], int(s.split(":")[1])) for s in args.sizes.split(",") if s]
    if args.eval:
        P = torch.as_tensor(load(args.eval)[0], device=dev)
        cmp = []
        for size, nseed in sizes:
            case = Case(size, dev)
            for amg in ([False, True] if args.amg else [False]):
                c = compare(case, P, seed=nseed + args.val_seeds + 1, steps=args.compare_steps, amg=amg)
                log("compare %s" % c)
                cmp.append(c)
        print(json.dumps(dict(weights=args.eval, compare=cmp)), flush=True)
        return
    t0 = time.perf_counter()
    train_s, val_s, cases = [], [], {}
    for size, nseed in sizes:
        case = Case(size, dev)
        cases[size] = case
        log("%s: %d dofs, nnz %d" % (size, case.mesh.n_dof, case.pat.nnz))
        for sd in range(1, nseed + args.val_seeds + 1):
            ss = collect(case.h, case.initial(sd), args.steps)
            (train_s if sd <= nseed else val_s).extend((case.net,) + s for s in ss)
            log("%s seed %d: %d pairs (%.1f s)" % (size, sd, len(ss), time.perf_counter() - t0))
    t1 = time.perf_counter()
    P, hist = train(train_s, epochs=args.epochs, lr=args.lr, log=log, loss_kind=kind)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    v0 = eval_loss(val_s, torch.as_tensor(init_params(0), device=dev), kind)
    v1 = eval_loss(val_s, P, kind)
    log("validation %s loss %.4g (guess = phi_prev: %.4g)" % (args.loss, v1, v0))
    # the other loss of the same network, for comparison between the two
    other = L.MPNN_LOSS_MSE if kind == L.MPNN_LOSS_KNORM else L.MPNN_LOSS_KNORM
    v1o = eval_loss(val_s, P, other)
    v0o = eval_loss(val_s, torch.as_tensor(init_params(0), device=dev), other)
    log("validation %s loss %.4g (guess = phi_prev: %.4g)" % ("mse" if kind else "knorm", v1o, v0o))
    del train_s, val_s
    cmp = []
    for size, nseed in sizes:
        for amg in ([False, True] if args.amg else [False]):
            c = compare(cases[size], P, seed=nseed + args.val_seeds + 1, steps=args.compare_steps, amg=amg)
            log("compare %s" % c)
            cmp.append(c)
    meta = dict(sizes=args.sizes, steps_per_seed=args.steps, val_seeds=args.val_seeds, epochs=args.epochs,
                lr=args.lr, loss=args.loss, train_loss=hist, val_loss=v1, val_loss_prev_phi=v0,
                val_other_loss=v1o, val_other_loss_prev_phi=v0o, data_s=t1 - t0,
                train_s=t2 - t1, compare=cmp)
    save(args.out, P.cpu().numpy(), meta)
    log("saved %s" % args.out)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
