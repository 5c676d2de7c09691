#!/usr/bin/env python
"""Benchmark: IPCS time steps per second on the 1.6M-node channel mesh.

Workload: the paper's channel box (Sec. 6.2: 4*pi x 2 x 4*pi/3, Re_tau =
180, body force (1,0,0), no-slip walls, periodic x/z) at 129 x 129 x 97
vertices, 6 tetrahedra per hexahedron, tanh wall stretching (beta = 2):
1,585,152 dofs per field, 9,437,184 cells, 23,678,976 CSR entries.
Synthetic initial field: laminar parabola + seeded U(-0.05, 0.05) noise,
dt = 0.01, Krylov relative tolerance 1e-8 (true residual, FP64).

Variants (same inputs, separate handles; every pressure solve starts from
phi_prev unless the name ends in _zero, where it starts from 0):
  fp64         plain FP64 BiCGStab + Jacobi-PCG
  mixed        FP32 inner Krylov with FP64 dot products and FP64 refinement
  learned      mixed + the trained message-passing warm start (its guess is
               used only when the guard prefers it to phi_prev)
  *_amg        the pressure solve is FP64 CG preconditioned by one
               smoothed-aggregation V(1,1) cycle per iteration (FP64 cycle
               for fp64_amg, FP32 for mixed_amg / learned_amg, whose
               level-0 smoothing reads the matrix values stored as FP16)
All reach the same FP64 true-residual tolerance.  The headline `value` is
the fastest variant whose pressure solve starts from phi_prev (the plain
start that is the fallback of the learned guess and its reference); `speedups` compare
it with plain FP64 Jacobi-PCG from phi_prev and like for like.

Also printed in the one JSON line:
  mixed_error   per-field relative L2 (u, v, w, p) of the FP32-inner run
                against the FP64 run after --error-steps steps from the same
                initial state (both on the GPU; the FP64 path is parity-
                tested against the oracle)
  config4       the displaced mesh with randomly permuted numbering,
                reordered by the on-device RCM, timed with the headline
                solver configuration
  extensions    the headline configuration with Alg. 1's inner iterations
                (2), the consistent-mass update, the gradient-matrix update,
                the explicit Adams-Bashforth convection, or one passive
                scalar
  roofline      the dominant kernel timed live over repeated launches
                against its algorithmic bytes, with the HBM traffic of the
                committed rocprofv3 counter summary when its sources match
  cpu_baseline  the FP64 oracle as it stands: one whole step (step 2, after
                an untimed step 1) on the same 129 x 129 x 97 mesh, in a
                single-threaded child process that runs on one host core
                while the GPU variants are timed
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IPCS steps/s + SpMV HBM GB/s, 1.6M-node P1 mesh; learned+FP32 vs plain FP64"
HBM_PEAK_GBS = 8000.0
# FP32 multigrid cycles read level 0's matrix values stored as FP16 (the CG
# around the cycle multiplies in FP64 and stops on its FP64 residual);
# --amg-fp32-level0 turns it off
AMG_HALF_LEVEL0 = True
# sources of the CG kernels; a PMC summary whose recorded hash differs from
# these files was taken on another kernel and is not used
CG_KERNEL_SOURCES = ["paper_1602_03643_amd/csrc/krylov.hip", "paper_1602_03643_amd/csrc/krylov.hpp",
                     "paper_1602_03643_amd/csrc/spmv.hpp", "paper_1602_03643_amd/csrc/internal.hpp"]
PMC_SUMMARIES = {"k_cg_p1_ell<double>": "profiles/k_cg_p1_ell_double_channel129_pmc.txt",
                 "k_cg_sr<float>": "profiles/k_cg_sr_float_channel129_pmc.txt"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cg_kernel_bytes(n, nnz, vbytes, single_reduction=False):
    """Algorithmic bytes of one launch of a CG kernel on the pressure matrix.

    Direction + product part of the two-kernel iteration (k_cg_p1*, also the
    product of the multigrid-preconditioned CG): the SpMV unit (values and
    int32 columns per entry, row pointers) with its vector streams: the
    gathered (r, p_old) pair read, the new (r, p) pair and q written, five
    vectors in all: vbytes*nnz + 4*nnz + 4(n+1) + 5*vbytes*n.

    Single-reduction FP32 iteration (k_cg_sr, a whole CG iteration): the FP32
    PCG-iteration unit 8*nnz + 56*n (values and columns per entry; r, w, s,
    p read and written, x read and written, the weights and the null vector
    read, 4 bytes each) plus the row pointers."""
    if not single_reduction:
        return vbytes * nnz + 4 * nnz + 4 * (n + 1) + 5 * vbytes * n
    return 8 * nnz + 56 * n + 4 * (n + 1)


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_summary(kernel):
    """The committed rocprofv3 PMC summary of `kernel` as a dict, or None
    when there is none or the kernel's sources changed since it was taken."""
    rel = PMC_SUMMARIES.get(kernel)
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    kv = {}
    with open(os.path.join(ROOT, rel)) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("sources_sha256") != sources_sha256(CG_KERNEL_SOURCES):
        return None
    return kv


def device_problem(oa, torch, synth, pr, dev, rcm=False):
    """Pattern and colouring of a problem's mesh on the device; with rcm, the
    dofs are first reordered by the on-device reverse Cuthill-McKee ordering
    (the mesh arrives with a random numbering).  Returns the device mesh,
    the pattern, the Dirichlet dofs, the permutation (or None) and the
    set-up times."""
    m = pr.mesh
    t0 = time.perf_counter()
    dm = oa.DeviceMesh.from_arrays(m.dim, m.coords, m.cells, m.vert2dof, m.n_dof, dev)
    bcd = torch.as_tensor(m.bc_dofs, dtype=torch.int32, device=dev)
    perm = None
    times = {}
    if rcm:
        pat0 = oa.p1_pattern(dm)
        t1 = time.perf_counter()
        perm, _ = oa.rcm(pat0)
        torch.cuda.synchronize()
        times["rcm_s"] = time.perf_counter() - t1
        dm = oa.DeviceMesh(m.dim, dm.coords, dm.cells, oa.relabel(dm.vert2dof, perm), m.n_dof)
        bcd = oa.relabel(bcd, perm)
    pat = oa.p1_pattern(dm)
    oa.colorize(dm, torch.as_tensor(synth.cell_priorities(m.n_cell), device=dev))
    torch.cuda.synchronize()
    times["graph_s"] = time.perf_counter() - t0
    return dm, pat, bcd, perm, times


def run_variant(oa, torch, pr, dm, pat, bcd, precision, steps, warmup, tag, warm=None, pstart=0, amg=None,
                perm=None, dof_coords=None, inner_iters=1, velocity_update=0, scalars=0, convection=0, amg_theta=0.0,
                inner_rtol=0.0, pressure_delta=0.0, amg_half=None):
    """Time `steps` steps after `warmup` untimed ones; returns the handle, the
    results and the final (U, p, phi).  scalars: that many passive scalars
    with Prandtl number 0.71 (D = nu / 0.71), Dirichlet values y on the
    walls and the start y plus seeded U(-0.05, 0.05) noise."""
    import numpy as np
    dev = dm.coords.device
    m = pr.mesh
    t0 = time.perf_counter()
    h = oa.IPCS(dm, pat, pr.dt, pr.nu, pr.f, bcd, rtol_u=pr.rtol_u, rtol_p=pr.rtol_p, precision=precision,
                inner_rtol=inner_rtol, pressure_delta=pressure_delta, pressure_start=pstart, inner_iters=inner_iters, velocity_update=velocity_update,
                diffusivity=[pr.nu / 0.71] * scalars, convection=convection)

    def T(a):
        """Host field [..., n] onto the device, in the reordered numbering."""
        t = torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        if perm is None:
            return t
        out = torch.empty_like(t)
        out[..., perm.long()] = t
        return out

    if warm is not None:
        h.set_warmstart(torch.as_tensor(warm, device=dev), T(m.dof_coords.T).T.contiguous()
                        if dof_coords is None else dof_coords)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    t_amg, levels = 0.0, 0
    if amg is not None:
        t0 = time.perf_counter()
        hamg = h.pressure_amg(precision=amg, theta=amg_theta,
                              half_level0=AMG_HALF_LEVEL0 if amg_half is None else amg_half)
        torch.cuda.synchronize()
        t_amg = time.perf_counter() - t0
        levels = hamg.n_levels()
        log("[%s] multigrid set-up %.2f s: %d levels" % (tag, t_amg, levels))
    U = [T(pr.U2), T(pr.U1)]
    p, phi = T(pr.p), T(pr.phi_prev)
    bc = torch.zeros(3 * bcd.numel(), dtype=torch.float64, device=dev)      # no-slip walls
    bufs = [torch.empty_like(U[0]) for _ in range(3)]
    stats = []
    Cs = None
    if scalars:
        y = m.dof_coords[:, 1]
        rng = np.random.default_rng(17)
        c1 = np.stack([y + rng.uniform(-0.05, 0.05, y.size) for _ in range(scalars)])
        c1[:, m.bc_dofs] = y[m.bc_dofs]
        Cs = [T(c1), torch.empty_like(T(c1))]
        cbc = torch.as_tensor(np.stack([y[m.bc_dofs]] * scalars), dtype=torch.float64, device=dev)

    def one(i):
        Un = bufs[i % 3] if bufs[i % 3].data_ptr() not in (U[0].data_ptr(), U[1].data_ptr()) else bufs[(i + 1) % 3]
        if Cs is not None:
            st = h.step(U[1], U[0], Un, p, phi, bc_values=bc, C1=Cs[0], Cn=Cs[1], C_bc=cbc)
            Cs.reverse()
        else:
            st = h.step(U[1], U[0], Un, p, phi, bc_values=bc)
        U[0], U[1] = U[1], Un
        return st

    for i in range(warmup):
        st = one(i)
        log("[%s] warmup step %d: iters_u %s iters_p %d outer %d/%d guess %d %.1f ms" %
            (tag, i, st["iters_u"], st["iters_p"], st["outer_u"], st["outer_p"], st["guess_used"],
             st["ms_total"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        stats.append(one(warmup + i))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for k, st in enumerate(stats):
        if st["status"] != 0:
            raise RuntimeError("%s step %d did not converge: %s" % (tag, k, st))
    res = {"create_s": t_create}
    if amg is not None:
        res.update(amg_setup_s=t_amg, amg_levels=levels)
    if steps:
        mean = lambda key: float(np.mean([s[key] for s in stats]))  # noqa: E731
        res.update(steps_per_s=steps / wall, ms_per_step=1e3 * wall / steps,
                   iters_p=mean("iters_p"),
                   iters_u=[float(np.mean([s["iters_u"][k] for s in stats])) for k in range(3)],
                   outer_p=mean("outer_p"), outer_u=mean("outer_u"),
                   ms_assemble=mean("ms_assemble"), ms_velocity=mean("ms_velocity"),
                   ms_pressure=mean("ms_pressure"), ms_update=mean("ms_update"),
                   guess_used=mean("guess_used"),
                   max_res_p=float(max(s["res_p"] for s in stats)),
                   max_res_u=float(max(max(s["res_u"]) for s in stats)))
        if velocity_update:
            res["iters_m"] = [float(np.mean([s["iters_m"][k] for s in stats])) for k in range(3)]
        if scalars:
            res.update(iters_c=[float(np.mean([s["iters_c"][a] for s in stats])) for a in range(scalars)],
                       ms_scalars=mean("ms_scalars"))
        log("[%s] %.2f steps/s (%.2f ms/step), iters_p %.1f, iters_u %s" %
            (tag, res["steps_per_s"], res["ms_per_step"], res["iters_p"], res["iters_u"]))
    return h, res, (U[1], p, phi)


def time_cg_kernel(oa, torch, h, pat, precision, iters=200):
    """Average duration of a CG kernel on the pressure matrix of the
    benchmark mesh: k_cg_sr (a whole iteration) for FP32 values, k_cg_p1_ell
    (the direction + product part, also the product kernel of the multigrid-
    preconditioned CG) for FP64 ones.  A standalone PCG on the singular
    matrix runs `iters` iterations, then its last launch of that kernel is
    repeated `iters` times back to back between two HIP events on the launch
    stream.  The grid is the one each kernel has in the timed steps: the FP64
    product at the multigrid handle's cap (768 blocks), the FP32 iteration
    at the Krylov default (512)."""
    Ks, _ = h.matrix(oa.FORM_STIFF)
    A = pat.with_values(Ks)
    n = pat.n
    g = torch.Generator(device="cpu").manual_seed(3)
    b = torch.randn(n, generator=g, dtype=torch.float64).to(Ks.device)
    b -= b.mean()
    x = torch.zeros_like(b)
    out = oa.pcg(A, b, x, rtol=1e-30, maxit=iters, precision=precision, time_kernel=True,
                 raise_on=False, nullspace_const=True, grid_cap=768 if precision == oa.F64 else 0)
    return out["kernel_ms"] / max(1, out["kernel_count"]), out["kernel_count"]


def field_errors(a, b):
    """Per-field relative L2 of final fields a = (U, p, phi) against b."""
    import numpy as np
    Ua, pa = a[0].cpu().numpy(), a[1].cpu().numpy()
    Ub, pb = b[0].cpu().numpy(), b[1].cpu().numpy()
    r = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))  # noqa: E731
    return {"u": r(Ua[0], Ub[0]), "v": r(Ua[1], Ub[1]), "w": r(Ua[2], Ub[2]), "p": r(pa, pb)}


CPU_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, %(root)r)
import synth
from oracle import ipcs
pr = synth.channel_flow(%(size)r, seed=0)
t0 = time.perf_counter()
S = ipcs.setup(pr.mesh, pr.nu, pr.dt, pr.f)
t_setup = time.perf_counter() - t0
st = ipcs.initial_state(pr)
t0 = time.perf_counter()
o1 = ipcs.step(S, st, pr.bc_values, rtol_u=pr.rtol_u, rtol_p=pr.rtol_p)
t1 = time.perf_counter() - t0
print("step 1: %%.1f s" %% t1, file=sys.stderr, flush=True)
t0 = time.perf_counter()
o2 = ipcs.step(S, o1.state, pr.bc_values, rtol_u=pr.rtol_u, rtol_p=pr.rtol_p)
t2 = time.perf_counter() - t0
print(json.dumps(dict(setup_s=t_setup, step1_s=t1, step2_s=t2, iters_p=[int(o1.iters_p), int(o2.iters_p)],
                      iters_u=[list(map(int, o1.iters_u)), list(map(int, o2.iters_u))])))
"""


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline_start(size, threads):
    """Start the oracle as it stands on the benchmark mesh in a child process
    whose BLAS/OpenMP pools are held to `threads` threads (scipy's CSR
    product is single-threaded whatever the setting): set-up untimed, step 1
    untimed, step 2 timed.  It uses no GPU and one host core, so it runs
    while the GPU variants are timed."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = str(threads)
    code = CPU_SNIPPET % {"root": ROOT, "size": size}
    return subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, text=True, env=env)


def cpu_baseline_wait(proc):
    out, _ = proc.communicate(timeout=1200)
    if proc.returncode != 0:
        raise RuntimeError("oracle baseline failed (%d)" % proc.returncode)
    return json.loads(out.strip().split("\n")[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", default="c129")
    ap.add_argument("--variants", default="fp64,mixed,learned,fp64_amg,mixed_amg,learned_amg")
    ap.add_argument("--weights", default=None, help="warm-start weights (.npz); default: the packaged ones")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a known-size kernel for PMC calibration)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-all-cores", action="store_true", help="also time the oracle with every host thread")
    ap.add_argument("--error-steps", type=int, default=50, help="0 skips the per-field mixed-precision error")
    ap.add_argument("--no-config4", action="store_true")
    ap.add_argument("--ext-steps", type=int, default=10,
                    help="timed steps of the headline configuration with each option beyond the channel runs' "
                         "(inner iterations, consistent update, a passive scalar); 0 skips them")
    ap.add_argument("--kernel-iters", type=int, default=200)
    ap.add_argument("--amg-fp32-level0", action="store_true",
                    help="FP32 cycles read level 0's values as FP32 (default: stored as FP16)")
    ap.add_argument("--pressure-delta", type=float, default=0.0,
                    help="FP32 pressure CG: residual replacement factor (0: the library's default)")
    args = ap.parse_args()
    global AMG_HALF_LEVEL0
    AMG_HALF_LEVEL0 = not args.amg_fp32_level0
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path here is single-GPU (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1602_03643_amd as oa
    import synth

    dev = torch.device("cuda", 0)
    cpu_proc = None
    if not args.no_cpu:
        log("starting the CPU oracle on %s (set-up and step 1 untimed, step 2 timed) ..." % args.size)
        cpu_proc = cpu_baseline_start(args.size, 1)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (src.numel() * 4, dst.numel() * 4))
        del src, dst
    t0 = time.perf_counter()
    pr = synth.channel_flow(args.size, seed=0)
    m = pr.mesh
    log("mesh %s: %d dofs, %d cells (%.1f s)" % (m.name, m.n_dof, m.n_cell, time.perf_counter() - t0))
    dm, pat, bcd, _, gtimes = device_problem(oa, torch, synth, pr, dev)
    log("pattern nnz %d, %d colours (%.2f s)" % (pat.nnz, dm.n_colors, gtimes["graph_s"]))

    def parse(v):
        parts = v.split("_")
        base = parts[0]
        if base not in ("fp64", "mixed", "learned") or any(q not in ("amg", "zero") for q in parts[1:]):
            raise SystemExit("unknown variant %s" % v)
        prec = oa.F64 if base == "fp64" else oa.F32
        pstart = oa.PSTART_ZERO if "zero" in parts else oa.PSTART_PREV
        amg = prec if "amg" in parts else None
        return base, prec, pstart, amg

    warm = None
    results, handles = {}, {}
    for v in args.variants.split(","):
        base, prec, pstart, amg = parse(v)
        w = None
        if base == "learned":
            from paper_1602_03643_amd import warmstart
            if warm is None:
                warm, wmeta = warmstart.load(args.weights or warmstart.DEFAULT_WEIGHTS)
                log("warm start: %s, trained on %s" % (args.weights or warmstart.DEFAULT_WEIGHTS,
                                                       wmeta.get("sizes")))
            w = warm
        h, res, _ = run_variant(oa, torch, pr, dm, pat, bcd, prec, args.steps, args.warmup, v, w, pstart, amg,
                                pressure_delta=args.pressure_delta)
        results[v] = res
        handles[v] = h
    # headline: the fastest variant whose pressure solve starts from phi_prev
    prev = [k for k in results if "zero" not in k.split("_")]
    head = max(prev or list(results), key=lambda k: results[k]["steps_per_s"])
    hres = results[head]
    hbase, hprec, hstart, hamg = parse(head)

    def ratio(a, b):
        return round(results[a]["steps_per_s"] / results[b]["steps_per_s"], 3) if b in results else None

    same_fp64 = "fp64" + ("_amg" if hamg is not None else "") + ("_zero" if hstart == oa.PSTART_ZERO else "")
    speedups = {"vs_fp64_jacobi_phi_prev": ratio(head, "fp64"),
                "vs_fp64_same_preconditioner_and_start": ratio(head, same_fp64),
                "same_preconditioner_reference": same_fp64}
    learned_gain = {}
    for k in results:
        if k.startswith("learned"):
            ref = "mixed" + k[len("learned"):]
            if ref in results:
                learned_gain[k] = {"ms_per_step": round(results[k]["ms_per_step"], 3), "vs": ref,
                                   "ref_ms_per_step": round(results[ref]["ms_per_step"], 3),
                                   "guess_used": results[k]["guess_used"]}

    # per-field error of the FP32-inner runs against the FP64 runs
    # (and, for scale, the spread between two FP64 runs with different
    # pressure solvers at the same tolerance)
    mixed_error = None
    if args.error_steps > 0:
        mixed_error = {"steps": args.error_steps}
        finals = {}
        for tag in ("fp64_amg", "mixed_amg", "fp64", "mixed"):
            if tag in results:
                _, prec, pstart, amg = parse(tag)
                hh, _, finals[tag] = run_variant(oa, torch, pr, dm, pat, bcd, prec, 0, args.error_steps,
                                                 tag + "/error", None, pstart, amg)
                hh.close()
        for v, ref in (("mixed_amg", "fp64_amg"), ("mixed", "fp64"), ("fp64_amg", "fp64")):
            if v in finals and ref in finals:
                key = v if v.startswith("mixed") else "%s_vs_%s" % (v, ref)
                mixed_error[key] = dict(field_errors(finals[v], finals[ref]), against=ref)
                log("[%s] per-field relative L2 vs %s after %d steps: %s" % (v, ref, args.error_steps,
                                                                             mixed_error[key]))

    # config 4: displaced mesh, random numbering, on-device RCM
    config4 = None
    if not args.no_config4:
        t0 = time.perf_counter()
        pr4 = synth.channel_flow(args.size, seed=0, displace_seed=1000, permute_seed=2000)
        log("config 4 mesh %s (%.1f s)" % (pr4.mesh.name, time.perf_counter() - t0))
        dm4, pat4, bcd4, perm4, t4 = device_problem(oa, torch, synth, pr4, dev, rcm=True)
        h4, res4, _ = run_variant(oa, torch, pr4, dm4, pat4, bcd4, hprec, args.steps, args.warmup,
                                  "config4/" + head, warm if hbase == "learned" else None, hstart, hamg,
                                  perm=perm4)
        config4 = dict(res4, variant=head, rcm_s=t4["rcm_s"], graph_s=t4["graph_s"],
                       workload="129x129x97 channel displaced by up to 0.2 of the local spacing (seed 1000), "
                                "dofs randomly permuted (seed 2000), reordered by the on-device RCM")
        h4.close()

    # options beyond the channel runs' configuration, on the headline solvers
    extensions = None
    if args.ext_steps > 0:
        extensions = {}
        for name, kw in (("inner_iters_2", dict(inner_iters=2)),
                         ("consistent_update", dict(velocity_update=oa.UPDATE_CONSISTENT)),
                         ("gradient_update", dict(velocity_update=oa.UPDATE_GRADIENT)),
                         ("abe_convection", dict(convection=oa.CONV_ABE)),
                         ("one_scalar", dict(scalars=1))):
            hh, res, _ = run_variant(oa, torch, pr, dm, pat, bcd, hprec, args.ext_steps, 3, head + "+" + name,
                                     None, hstart, hamg, **kw)
            extensions[name] = dict(res, base=head)
            hh.close()

    # dominant kernel of the headline path and its live timing
    sr = hprec == oa.F32 and hamg is None    # the FP32 Jacobi-CG iteration is one single-reduction kernel
    vbytes = 4 if sr else 8
    kname = "k_cg_sr<float>" if sr else "k_cg_p1_ell<double>"
    avg_ms, cnt = time_cg_kernel(oa, torch, handles[head], pat, oa.F32 if sr else oa.F64, args.kernel_iters)
    kb = cg_kernel_bytes(pat.n, pat.nnz, vbytes, sr)
    achieved = kb / (avg_ms * 1e-3) / 1e9
    pmc = pmc_summary(kname) if args.size == "c129" else None
    traffic = float(pmc["traffic_bytes_per_launch"]) if pmc else None
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=kname,
                bytes_per_launch=kb, avg_launch_ms=avg_ms, launches_timed=cnt)
    if traffic:
        roof["traffic_gbs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    if not sr:
        a32, _ = time_cg_kernel(oa, torch, handles[head], pat, oa.F32, args.kernel_iters)
        kb32 = cg_kernel_bytes(pat.n, pat.nnz, 4, True)
        roof["jacobi_fp32_kernel"] = dict(kernel="k_cg_sr<float>", avg_launch_ms=a32, bytes_per_launch=kb32,
                                          achieved=round(kb32 / (a32 * 1e-3) / 1e9, 1))

    cpu = None
    if cpu_proc is not None:
        log("waiting for the CPU oracle ...")
        d1 = cpu_baseline_wait(cpu_proc)
        cpu = dict(value=1.0 / d1["step2_s"], unit="steps/s", cores=1, kind="oracle",
                   sample=("one whole FP64 oracle step (step 2, after an untimed step 1) of the %s channel "
                           "(%d dofs/field; %d Jacobi-PCG, %s BiCGStab iterations) in a single-threaded "
                           "process: %.1f s; host %s, %d threads" %
                           (m.name.split("_")[1], m.n_dof, d1["iters_p"][1], d1["iters_u"][1], d1["step2_s"],
                            cpu_model(), os.cpu_count() or 0)),
                   step2_s=d1["step2_s"], step1_s=d1["step1_s"], setup_s=d1["setup_s"],
                   cpu_model=cpu_model(), host_threads=os.cpu_count())
        if args.cpu_all_cores:
            nt = os.cpu_count() or 1
            d2 = cpu_baseline_wait(cpu_baseline_start(args.size, nt))
            cpu["all_cores"] = dict(value=1.0 / d2["step2_s"], cores=nt, step2_s=d2["step2_s"])
    line = {
        "metric": METRIC,
        "value": round(hres["steps_per_s"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hres["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if hprec == oa.F64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "channel %s: %d dofs/field, %d tets, nnz %d, Re_tau 180, dt 0.01, rtol 1e-8"
                   % (m.name.split("_")[1], m.n_dof, m.n_cell, pat.nnz),
                   "variant": head, "pressure_start": "phi_prev" if hstart == oa.PSTART_PREV else "zero",
                   "pressure_preconditioner": "smoothed-aggregation AMG" if hamg is not None else "Jacobi",
                   "parallelism": "single GPU"},
        "variants": results,
        "speedup_vs_fp64": speedups["vs_fp64_jacobi_phi_prev"],
        "speedups": speedups,
        "guess_used": hres["guess_used"],
        "learned_gain": learned_gain,
        "mixed_error": mixed_error,
        "config4": config4,
        "extensions": extensions,
        "roofline": roof,
        "cpu_baseline": cpu,
        "setup_s": {"graph": gtimes["graph_s"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
