#!/usr/bin/env python3
"""Benchmark of the electrostatic PIC step on one MI355X.

Workload (default): Landau damping (k = 0.5, alpha = 0.05, L = 4 pi) on a
512^3 grid with 8 particles per cell (2^30 particles, FP64 positions and
velocities), Jacobi-PCG to relative residual 1e-10, dt = 0.05 -- the paper's
case A shape (Sec. 4.1, Table setup_sizes) on one GPU.  A step is one pass of
the whole hot path: gather + push -> stable cell sort -> CIC deposit -> PCG
solve (warm start) -> field.  Inputs are synthetic and seeded, drawn on the
device; initialisation and the t = 0 solve are not timed (Sec. 4.1 times the
run minus initialisation).

Prints ONE JSON line.  `roofline` is for the dominant kernel (the FP64
PCG's single-reduction sweep; with --two-sweep, or for the other solver
forms, the PCG update sweep), timed with HIP events on the stream it runs on
during the timed steps; `cpu_baseline` times the CPU oracle on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s/PIC step + PCG HBM GB/s, 512^3x8ppc; learned vs plain time at rtol 1e-10"
PEAK_HBM_GBS = 8000.0
# algorithmic bytes per grid point of one launch of each PCG sweep (FP64):
# direction sweep reads r, p_old and writes p_new; update sweep reads p, x, r
# and writes x, r.  (FP32 inner sweeps of the mixed form: half.)
SWEEP_BYTES = {"pcg_fp64": (24, 40), "pcg_mixed": (12, 20), "fcg_learned": (24, 40),
               "pcg_ssor": (24, 40), "fft": (24, 40),
               "pif": (24, 40)}
# The Jacobi-PCG single-reduction sweep (the default on the periodic box)
# reads r and p_old and writes r and p at every iteration, and reads and
# writes x every other iteration (the two steps of a pair applied together):
# 32 and 48 bytes per grid point in FP64, 40 on average over the sampled
# pairs; the mixed form's FP32 inner sweeps likewise (their correction d
# every other iteration): 16 and 24, 20 on average.
SINGLE_SWEEP_BYTES = 40
SINGLE_SWEEP_BYTES_FP32 = 20
# SSOR preconditioner, fused triangular solves of its last outer step:
# forward reads the right side and writes y, backward reads y, the running z
# and r (for r . z) and writes z
SSOR_FWD_BYTES = 16
SSOR_BWD_BYTES = 32
# s-step form (three iterations per outer step): Gram sweep reads p and r,
# update sweep reads p, r, x and writes them
SSTEP_S = 3
SSTEP_GRAM_BYTES = 16
SSTEP_UPD_BYTES = 48
# HBM bytes per launch of the dominant kernel at 512^3, from rocprofv3
# FETCH_SIZE (x2) + WRITE_SIZE of this kernel version
# (profiles/pcg_sweeps_landau512_hbm_counters.md); None for other workloads.
SWEEP_TRAFFIC = {(512, "pcg_fp64", "pcg_sstep_update"): 6.945e9}
TRAFFIC_SOURCE = ("rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of this kernel "
                  "(profiles/pcg_sweeps_landau512_hbm_counters.md)")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(N, ppc, p, sim, iters_per_step, budget_s):
    """Time the CPU oracle on a bounded sample of the same step and scale it
    to seconds per step: PCG iterations at the full grid (from the GPU's
    right-hand side) x iterations per step, plus the particle phases timed at
    two sample sizes and extrapolated linearly to all particles, plus the
    field at the full grid."""
    import numpy as np
    import torch

    import oracle

    oracle.build()
    L = p.length
    threads = oracle.num_threads()
    npart = ppc * N ** 3
    if npart <= (1 << 22):
        # small workloads: whole oracle steps from the GPU's current state
        st = oracle.State(N, L, p.charge, p.qm, p.dt, *[a.cpu().numpy() for a in sim.particles])
        st.phi = sim.phi.cpu().numpy().copy()
        st.ex, st.ey, st.ez = (t.cpu().numpy() for t in (sim.ex, sim.ey, sim.ez))
        nsteps, t0 = 0, time.perf_counter()
        while nsteps < 1 or (time.perf_counter() - t0 < budget_s and nsteps < 20):
            st.step(p.rtol, p.max_iter)
            nsteps += 1
        s_step = (time.perf_counter() - t0) / nsteps
        return {"value": s_step, "unit": "s/step", "cores": threads, "kind": "oracle",
                "sample": "%d whole oracle steps (push, sort, deposit, PCG, field) from the "
                          "GPU run's state" % nsteps}
    b = sim.rho.cpu().numpy()
    phi = sim.phi.cpu().numpy()
    ex, ey, ez = (t.cpu().numpy() for t in (sim.ex, sim.ey, sim.ez))
    # PCG: k iterations from the previous potential
    tm = {}
    for m in (1, 5):
        t0 = time.perf_counter()
        oracle.pcg(N, L, b, phi, p.rtol, m)
        tm[m] = time.perf_counter() - t0
    t_iter = max((tm[5] - tm[1]) / 4.0, tm[1] / 2.0)
    # field at the full grid
    t0 = time.perf_counter()
    oracle.efield(N, L, phi)
    t_field = time.perf_counter() - t0
    # particle phases (push, keys, sort, deposit) at two sample sizes
    cur = sim.particles
    samples = []
    for n in (1 << 20, 1 << 21):
        parts = [a[:n].cpu().numpy() for a in cur]
        t0 = time.perf_counter()
        out = oracle.gather_push(N, L, p.dt, p.qm, *parts, ex, ey, ez)
        perm, cs = oracle.sort_by_key(out[6], N ** 3)
        xs = [out[k][perm] for k in range(3)]
        oracle.deposit(N, L, p.charge, p.rho_bg, *xs)
        samples.append((n, time.perf_counter() - t0))
    (n1, s1), (n2, s2) = samples
    per_particle = max((s2 - s1) / (n2 - n1), 0.0)
    fixed = max(s1 - per_particle * n1, 0.0)
    t_particles = fixed + per_particle * npart
    s_step = iters_per_step * t_iter + t_particles + t_field
    sample = ("oracle PCG: 1 and 5 iterations at %d^3 (%.3f s/iteration) x %.0f iterations/step; "
              "gather+push+sort+deposit on 2^20 and 2^21 particles extrapolated linearly to %d "
              "(%.1f s); field at %d^3 (%.2f s)" % (N, t_iter, iters_per_step, npart, t_particles,
                                                   N, t_field))
    return {"value": s_step, "unit": "s/step", "cores": threads, "kind": "oracle",
            "sample": sample}


def load_weights(ctx, path):
    import numpy as np
    import torch

    if path is None:
        path = os.path.join(ROOT, "paper_2605_05469_amd", "weights", "unet_landau128.npy")
    w = np.load(path, allow_pickle=False).astype(np.float32)
    ctx.set_unet(torch.from_numpy(w).cuda())


def accuracy_vs_fp64(args, sim, p):
    """Re-run warm-up + timed steps from the same seeded state with the FP64
    solver; report the differences of phi, E and positions."""
    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    q = P.landau_params(args.grid, args.ppc, rtol=args.rtol, solver="pcg_fp64", check_every=32)
    ctx = P.Context(q)
    parts = synth.landau_particles_torch(args.grid, args.ppc, seed=args.seed, device="cuda")
    ref = P.Simulation(ctx, *parts)
    del parts
    ref.init()
    for _ in range(args.warmup + args.steps):
        ref.step(timed=False)
    h = p.length / args.grid

    def rel(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    dx = max(float(torch.max(torch.abs(torch.remainder(a - b + 0.5 * p.length, p.length)
                                      - 0.5 * p.length))) for a, b in
             zip(sim.particles[:3], ref.particles[:3]))
    res = {"phi_rel_l2": rel(sim.phi, ref.phi),
           "E_rel_l2": max(rel(a, b) for a, b in ((sim.ex, ref.ex), (sim.ey, ref.ey),
                                                   (sim.ez, ref.ez))),
           "max_position_diff_over_h": dx / h,
           "steps": args.warmup + args.steps}
    del ref, ctx
    return res


def bench_poisson(args):
    """Standalone solves of the deposit of Landau particles (1 ppc by default
    at 1024^3): cold start, each solver form, timed."""
    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    N, ppc = args.grid, args.ppc
    p = P.landau_params(N, ppc, rtol=args.rtol, solver="pcg_fp64", check_every=32,
                        inner_rtol=args.inner_rtol)
    if args.no_warm_start:
        p.flags = P.FLAG_NO_WARM_START
    ctx = P.Context(p)
    parts = synth.landau_particles_torch(N, ppc, seed=args.seed, device="cuda")
    rho = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
    ctx.deposit(parts[0], parts[1], parts[2], None, rho)
    del parts
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the library allocates the network outside torch
    forms = {}
    all_forms = ("pcg_fp64", "pcg_fp64_single", "pcg_fp64_two_sweep", "pcg_mixed",
                 "pcg_mixed_reliable",
                 "pcg_ssor", "pcg_ssor_unfused",
                 "fcg_learned",
                 "learned_warm_start_only", "learned_warm_start_mixed", "fft", "fft_spectral")
    for form in (args.forms.split(",") if args.forms else all_forms):
        if form not in all_forms:
            raise SystemExit("unknown form %r (choose from %s)" % (form, ", ".join(all_forms)))
        solver = ("fcg_learned" if form.startswith("learned") else
                  "pcg_mixed" if form.startswith("pcg_mixed") else
                  "pcg_ssor" if form.startswith("pcg_ssor") else
                  "fft" if form.startswith("fft") else
                  "pcg_fp64" if form.startswith("pcg_fp64") else form)
        if solver == "fcg_learned":
            try:
                load_weights(ctx, args.weights)
            except (OSError, ValueError) as e:
                forms[form] = {"skipped": repr(e)}
                continue
        ctx.set_flags((P.FLAG_NO_WARM_START if args.no_warm_start else 0)
                      | (P.FLAG_WARM_START_ONLY if form.startswith("learned_") else 0)
                      | (P.FLAG_MIXED_RELIABLE if form in ("pcg_mixed_reliable",
                                                           "learned_warm_start_mixed") else 0)
                      | (P.FLAG_LEARNED_MIXED if form == "learned_warm_start_mixed" else 0)
                      | (P.FLAG_FFT_SPECTRAL if form == "fft_spectral" else 0)
                      | (P.FLAG_SSOR_UNFUSED if form == "pcg_ssor_unfused" else 0)
                      | (P.FLAG_PCG_TWO_SWEEP if form == "pcg_fp64_two_sweep" else 0)
                      | (P.FLAG_PCG_SINGLE_SWEEP if form == "pcg_fp64_single" else 0))
        ctx.set_solver(solver)
        phi = torch.zeros_like(rho)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.poisson(rho, phi)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        forms[form] = {"s_per_solve": dt, "iterations": info["iterations"],
                         "outer_iterations": info["outer_iterations"],
                         "flex_iterations": info["flex_iterations"],
                         "fell_back": info["fell_back"], "warm_start_used": info["warm_start_used"],
                         "rel_res": info["rel_res"], "converged": bool(info["converged"])}
        log("%s: %.3f s, %d iterations, rel_res %.2e" % (form, dt, info["iterations"],
                                                         info["rel_res"]))
    name = args.solver
    if name == "pcg_mixed" and args.mixed_reliable:
        name = "pcg_mixed_reliable"
    if name == "fft" and args.fft_spectral:
        name = "fft_spectral"
    if name == "fcg_learned" and args.warm_start_only:
        name = "learned_warm_start_mixed" if args.learned_mixed else "learned_warm_start_only"
    sel = forms.get(name, {})
    n3 = N ** 3
    out = {"metric": METRIC, "value": sel.get("s_per_solve"), "unit": "s/solve", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": 1e3 * sel.get("s_per_solve", float("nan")),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "poisson_solve_%d^3_rhs_%dppc_landau" % (N, ppc), "grid": N,
                      "ppc": ppc, "rtol": args.rtol, "solver": args.solver},
           "forms": forms}
    print(json.dumps(out), flush=True)


# flops of one network application per fine-grid point: 2 * 27 * ci * co per
# output point of each 3^3 convolution, levels 1, 2, 3 at 1, 1/8, 1/64 points
NET_LAYERS = (("e1a", 1, 16, 1), ("e1b", 16, 16, 1), ("e2a", 16, 32, 2), ("e2b", 32, 32, 2),
              ("b3a", 32, 64, 3), ("b3b", 64, 32, 3), ("d2a", 32, 32, 2), ("d2b", 32, 16, 2),
              ("d1a", 16, 16, 1), ("out", 16, 1, 1))
PEAK_BF16_TFLOPS = 2500.0


def net_flops(n):
    return sum(2 * 27 * ci * co * (n >> (lvl - 1)) ** 3 for _, ci, co, lvl in NET_LAYERS)


def bench_network(args):
    """The learned preconditioner's network alone: z = s NN(h^2 r / s) - mean
    on an n^3 grid (inference), and one training step (forward, loss,
    backward, Adam) at the training grid; HIP events on the library's stream."""
    import numpy as np
    import torch

    import paper_2605_05469_amd as P

    n = args.grid
    net = P.Net(n)
    path = args.weights or os.path.join(ROOT, "paper_2605_05469_amd", "weights",
                                        "unet_landau128.npy")
    params = torch.from_numpy(np.load(path, allow_pickle=False).astype(np.float32)).cuda()
    net.set_params(params)
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    r = torch.randn(n ** 3, device="cuda", dtype=torch.float64, generator=g)
    z = torch.empty_like(r)
    h = 4 * math.pi / n

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = timed(lambda: net.precondition(r, h, z), args.steps)
    fl = net_flops(n)
    del net
    torch.cuda.empty_cache()
    nt = 128
    tnet = P.Net(nt, training=True)
    tnet.set_params(params)
    x = torch.randn(nt ** 3, device="cuda", generator=g)
    t = torch.randn(nt ** 3, device="cuda", generator=g)
    ms_train = timed(lambda: tnet.train_step(x, t, lam=1.0, lr=1e-5, want_loss=False), args.steps)
    tf = fl / (ms * 1e-3) / 1e12
    out = {"metric": "network preconditioner application time (ms), BF16 MFMA",
           "value": ms, "unit": "ms/application", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "unet_precondition_%d^3" % n, "grid": n,
                      "channels": [16, 32, 64], "levels": 3},
           "tflop_per_application": fl / 1e12,
           "train_step_ms_128": ms_train,
           "train_tflops_128": 3 * net_flops(nt) / (ms_train * 1e-3) / 1e12,
           "roofline": {"bound": "mfma", "kernel": "whole network", "achieved": tf,
                        "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / PEAK_BF16_TFLOPS, "traffic": None}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--ppc", type=int, default=8)
    ap.add_argument("--solver", default="pcg_fp64", choices=sorted(SWEEP_BYTES))
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=20262)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--weights", default=None,
                    help="FP32 network parameters (.npy, canonical order) for fcg_learned")
    ap.add_argument("--inner-rtol", type=float, default=1e-3)
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--forms", default=None,
                    help="poisson workload: comma-separated solver forms to time (default: all)")
    ap.add_argument("--fft-spectral", action="store_true",
                    help="fft solver: pseudo-spectral symbol and E = -i k phi")
    ap.add_argument("--learned-mixed", action="store_true",
                    help="learned form: hand over to the mixed form (not FP64 PCG)")
    ap.add_argument("--mixed-reliable", action="store_true",
                    help="mixed form: keep the inner direction across refinements")
    ap.add_argument("--two-sweep", action="store_true",
                    help="FP64 Jacobi-PCG as a direction and an update sweep per iteration "
                         "(instead of the single-reduction sweep)")
    ap.add_argument("--single-sweep", action="store_true",
                    help="FP64 Jacobi-PCG as one single-reduction sweep per iteration "
                         "(instead of the s-step form's Gram and update sweeps)")
    ap.add_argument("--warm-start-only", action="store_true",
                    help="learned form: network warm start, then Jacobi-PCG")
    ap.add_argument("--no-1024", action="store_true",
                    help="default run: skip the 1024^3 standalone solves")
    ap.add_argument("--no-learned", action="store_true",
                    help="default run: skip the learned + mixed form and the 32^3 line")
    ap.add_argument("--accuracy-vs-fp64", action="store_true",
                    help="rerun the same steps with the FP64 solver and report the differences")
    ap.add_argument("--workload", default="pic", choices=["pic", "poisson", "network"],
                    help="pic: full PIC steps; poisson: standalone solves of a deposited rho; "
                         "network: the learned preconditioner alone")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    torch.cuda.set_device(0)
    # the achievable-bandwidth reference first, on fresh device memory
    triad = bench_triad() if args.workload == "pic" and not args.no_learned else None
    if args.workload == "poisson":
        return bench_poisson(args)
    if args.workload == "network":
        return bench_network(args)
    N, ppc = args.grid, args.ppc
    flags = 0
    if args.no_warm_start:
        flags |= P.FLAG_NO_WARM_START
    if args.warm_start_only:
        flags |= P.FLAG_WARM_START_ONLY
    if args.mixed_reliable:
        flags |= P.FLAG_MIXED_RELIABLE
    if args.learned_mixed:
        flags |= P.FLAG_LEARNED_MIXED
    if args.fft_spectral:
        flags |= P.FLAG_FFT_SPECTRAL
    if args.two_sweep:
        flags |= P.FLAG_PCG_TWO_SWEEP
    if args.single_sweep:
        flags |= P.FLAG_PCG_SINGLE_SWEEP
    fp32_inner = args.solver == "pcg_mixed" or args.learned_mixed
    run = run_pic(args, args.solver, flags, args.inner_rtol, fp32_inner, "main")
    sim, ctx, p, infos = run.pop("_sim"), run.pop("_ctx"), run.pop("_p"), run.pop("_infos")
    out = {
        "metric": METRIC,
        "value": run["s_per_step"],
        "unit": "s/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * run["s_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32_inner else "f64",
        "data": "synthetic",
        "config": {"workload": "landau_damping_%d^3_%dppc_%s" % (N, ppc, args.solver),
                   "grid": N, "ppc": ppc, "particles": ppc * N ** 3, "solver": args.solver,
                   "rtol": args.rtol, "dt": p.dt, "k": 0.5, "alpha": 0.05,
                   "pcg_form": run["pcg_form"], "parallelism": "single_gpu"},
    }
    out.update({k: v for k, v in run.items() if k not in ("s_per_step", "pcg_form")})
    if args.accuracy_vs_fp64 and args.solver != "pcg_fp64":
        out["accuracy_vs_fp64"] = accuracy_vs_fp64(args, sim, p)
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(N, ppc, p, sim, run["pcg_iterations_per_step"],
                                               args.cpu_budget)
        except Exception as e:  # the GPU line must still be printed
            out["cpu_baseline"] = {"error": repr(e)}
    default_run = (args.solver == "pcg_fp64" and not flags and not args.no_learned)
    if default_run:
        # the metric's second half: the mixed-precision + learned form on the
        # same seeded state, same steps; then its difference from this run
        ref = save_state(sim)
        del sim
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        mixed_desc = ("the mixed form: FP32 inner Jacobi-PCG (single-reduction sweeps, dot "
                      "products in FP64), reliable updates, inner tolerance 0.1, FP64 "
                      "refinement to the same rtol")
        forms = (("mixed", "pcg_mixed", P.FLAG_MIXED_RELIABLE, mixed_desc),
                 ("learned_mixed", "fcg_learned",
                  P.FLAG_WARM_START_ONLY | P.FLAG_LEARNED_MIXED | P.FLAG_MIXED_RELIABLE,
                  "the trained network's warm start, then " + mixed_desc))
        for key, solver, fl, desc in forms:
            r2 = run_pic(args, solver, fl, 0.1, True, key)
            s2, c2, p2 = r2.pop("_sim"), r2.pop("_ctx"), r2.pop("_p")
            infos2 = r2.pop("_infos")
            r2["accuracy_vs_fp64"] = compare_state(s2, ref, p2)
            if solver == "fcg_learned":
                r2["warm_start_used_steps"] = sum(1 for i in infos2 if i["warm_start_used"])
            r2["config"] = {"solver": solver, "form": desc, "rtol": args.rtol}
            if solver == "fcg_learned":
                r2["config"]["weights"] = "unet_landau128.npy"
            out[key] = r2
            del s2
            c2.close()
            del c2
            torch.cuda.empty_cache()
        out["learned_vs_plain"] = {
            "plain_s_per_step": out["value"],
            "mixed_s_per_step": out["mixed"]["s_per_step"],
            "learned_mixed_s_per_step": out["learned_mixed"]["s_per_step"],
            "speedup_learned_mixed": out["value"] / out["learned_mixed"]["s_per_step"],
            "speedup_mixed": out["value"] / out["mixed"]["s_per_step"],
            "learned_over_mixed": out["mixed"]["s_per_step"] / out["learned_mixed"]["s_per_step"]}
        del ref
        out["config0"] = bench_config0(args)
        if not args.no_1024:
            try:
                out["config4"] = bench_config4(args)
            except Exception as e:  # the main line must still be printed
                out["config4"] = {"error": repr(e)}
        out["hbm_triad"] = triad
    print(json.dumps(out), flush=True)


def bench_triad():
    """The library's STREAM triad (a = b + s c, 24 bytes per element) on
    three 2 GiB arrays: the achievable HBM bandwidth beside the 8 TB/s peak."""
    import torch

    import paper_2605_05469_amd as P

    n = 1 << 28
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    ms = P.stream_triad(b, c, a, 3.0, 20)
    ok = bool(torch.equal(a[-1024:], b[-1024:] + 3.0 * c[-1024:]))
    del a, b, c
    torch.cuda.empty_cache()
    return {"kernel": "pic_stream_triad (16-byte loads and non-temporal stores)",
            "elements": n, "bytes_per_launch": 24 * n, "avg_ms": ms,
            "gbs": 24 * n / (ms * 1e-3) / 1e9, "frac_of_peak": 24 * n / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "checked": ok}


def save_state(sim):
    """Host copies of phi, E and positions (for the accuracy comparison)."""
    return {"phi": sim.phi.cpu(), "E": [t.cpu() for t in (sim.ex, sim.ey, sim.ez)],
            "x": [t.cpu() for t in sim.particles[:3]]}


def compare_state(sim, ref, p):
    """Relative L2 differences of phi and E and the largest periodic position
    difference (in cells) against the saved FP64 state."""
    import torch

    def rel(a, b):
        b = b.to(a.device)
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    h = p.length / p.n
    dx, far = 0.0, 0
    for a, b in zip(sim.particles[:3], ref["x"]):
        d = torch.remainder(a - b.to(a.device) + 0.5 * p.length, p.length) - 0.5 * p.length
        d = torch.abs(d)
        far += int(torch.count_nonzero(d > 1e-6 * h))
        dx = max(dx, float(torch.max(d)))
        del d
    return {"reference": "the FP64 Jacobi-PCG run of this benchmark (same seeded state, same "
                         "steps; its solver matches the CPU oracle in the parity tests)",
            "phi_rel_l2": rel(sim.phi, ref["phi"]),
            "E_rel_l2": max(rel(a, b) for a, b in zip((sim.ex, sim.ey, sim.ez), ref["E"])),
            "max_position_diff_over_h": dx / h,
            "position_slots_differing_by_more_than_1e-6_h": far}


def run_pic(args, solver, flags, inner_rtol, fp32_inner, label):
    """Init (untimed), warm-up steps, then `args.steps` timed PIC steps with
    the dominant PCG kernel sampled by HIP events on its stream."""
    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    N, ppc = args.grid, args.ppc
    p = P.landau_params(N, ppc, rtol=args.rtol, solver=solver, check_every=32,
                        inner_rtol=inner_rtol, flags=flags)
    ctx = P.Context(p)
    if solver == "fcg_learned":
        load_weights(ctx, args.weights)
    t0 = time.perf_counter()
    parts = synth.landau_particles_torch(N, ppc, seed=args.seed, device="cuda")
    sim = P.Simulation(ctx, *parts)
    del parts
    info0 = sim.init()
    torch.cuda.synchronize()
    log("%s init: %.1f s, t=0 solve %d iterations" % (label, time.perf_counter() - t0,
                                                       info0["iterations"]))
    for k in range(args.warmup):
        w = sim.step()
        log("%s warmup %d: %d iterations, %.1f ms solve" % (label, k, w["iterations"],
                                                             w["ms_solve"]))
    ctx.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(sim.step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s_step = elapsed / args.steps
    iters = sum(i["iterations"] for i in infos) / len(infos)
    n3 = N ** 3
    npart = ppc * n3
    bdir, bupd = SWEEP_BYTES["pcg_mixed" if fp32_inner else solver]
    ms_dir, cnt_dir = P.Context.kernel_time(ctx, 0)
    ms_upd, cnt_upd = P.Context.kernel_time(ctx, 1)
    ms_f, cnt_f = P.Context.kernel_time(ctx, 2)  # SSOR-PCG only
    ms_b, cnt_b = P.Context.kernel_time(ctx, 3)
    ctx.set_kernel_timing(False)
    # Jacobi-PCG (FP64, the mixed form's FP32 inner solves, the learned form's
    # hand-over) runs as one kernel per iteration on the periodic box unless
    # two sweeps are asked for; its launches are sampled in timing slot 0
    sstep = (solver == "pcg_fp64" and N % 32 == 0
             and not (flags & (P.FLAG_PCG_TWO_SWEEP | P.FLAG_PCG_SINGLE_SWEEP)))
    single = (not sstep and solver in ("pcg_fp64", "pcg_mixed", "fcg_learned")
              and not (flags & P.FLAG_PCG_TWO_SWEEP) and N % 32 == 0)
    if sstep:
        # s-step form: per outer step (three iterations) a Gram sweep reading
        # p and r (16 B/point) and an update sweep reading p, r, x and writing
        # them (48 B/point); timing slots 0 and 1
        bg, bu = SSTEP_GRAM_BYTES, SSTEP_UPD_BYTES
        gbs_gram = bg * n3 / (ms_dir * 1e-3) / 1e9 if ms_dir > 0 else 0.0
        gbs_upd = bu * n3 / (ms_upd * 1e-3) / 1e9 if ms_upd > 0 else 0.0
        kernels = {"pcg_sstep_gram": {"avg_ms": ms_dir, "launches_timed": cnt_dir,
                                      "bytes_per_point": bg, "gbs": gbs_gram},
                   "pcg_sstep_update": {"avg_ms": ms_upd, "launches_timed": cnt_upd,
                                        "bytes_per_point": bu, "gbs": gbs_upd}}
        gbs_iter = (bg + bu) * n3 / ((ms_dir + ms_upd) * 1e-3) / 1e9 if ms_upd > 0 else 0.0
        dom, gbs_dom = "pcg_sstep_update", gbs_upd
    elif single:
        b1 = SINGLE_SWEEP_BYTES_FP32 if fp32_inner else SINGLE_SWEEP_BYTES
        dom = "pcg_single_sweep_fp32" if fp32_inner else "pcg_single_sweep"
        gbs_one = b1 * n3 / (ms_dir * 1e-3) / 1e9 if ms_dir > 0 else 0.0
        kernels = {dom: {"avg_ms": ms_dir, "launches_timed": cnt_dir, "bytes_per_point": b1,
                         "gbs": gbs_one}}
        gbs_dom, gbs_iter = gbs_one, gbs_one
    else:
        gbs_upd = bupd * n3 / (ms_upd * 1e-3) / 1e9 if ms_upd > 0 else 0.0
        gbs_dir = bdir * n3 / (ms_dir * 1e-3) / 1e9 if ms_dir > 0 else 0.0
        gbs_iter = (bdir + bupd) * n3 / ((ms_dir + ms_upd) * 1e-3) / 1e9 if ms_upd > 0 else 0.0
        kernels = {"pcg_direction_sweep": {"avg_ms": ms_dir, "launches_timed": cnt_dir,
                                           "bytes_per_point": bdir, "gbs": gbs_dir},
                   "pcg_update_sweep": {"avg_ms": ms_upd, "launches_timed": cnt_upd,
                                        "bytes_per_point": bupd, "gbs": gbs_upd}}
        dom, gbs_dom = "pcg_update_sweep", gbs_upd
        if solver == "pcg_ssor" and not (flags & P.FLAG_SSOR_UNFUSED):
            # the preconditioner's fused triangular solves of its last outer
            # step (timing slots 2, 3): forward reads r - A z and writes y
            # (16 B/point), backward reads y, z and r and writes z (32)
            gbs_f = SSOR_FWD_BYTES * n3 / (ms_f * 1e-3) / 1e9 if ms_f > 0 else 0.0
            gbs_b = SSOR_BWD_BYTES * n3 / (ms_b * 1e-3) / 1e9 if ms_b > 0 else 0.0
            kernels["ssor_forward_solve"] = {"avg_ms": ms_f, "launches_timed": cnt_f,
                                             "bytes_per_point": SSOR_FWD_BYTES, "gbs": gbs_f}
            kernels["ssor_backward_solve"] = {"avg_ms": ms_b, "launches_timed": cnt_b,
                                              "bytes_per_point": SSOR_BWD_BYTES, "gbs": gbs_b}
            # per SSOR-PCG iteration two backward solves (the last one with
            # its added terms) take the most time
            dom, gbs_dom = "ssor_backward_solve", gbs_b
    phases = {k: sum(i[k] for i in infos) / len(infos)
              for k in ("ms_push", "ms_sort", "ms_deposit", "ms_solve", "ms_field")}
    for i, inf in enumerate(infos):
        log("%s step %d: %d iterations, rel_res %.2e, solve %.0f ms" % (
            label, i, inf["iterations"], inf["rel_res"], inf["ms_solve"]))
    traffic = SWEEP_TRAFFIC.get((N, "pcg_mixed" if fp32_inner else solver, dom))
    return {
        "s_per_step": s_step,
        "pcg_form": ("sstep_%d" % SSTEP_S if sstep else
                     "single_reduction_sweep" if single else "two_sweeps"),
        "particles_per_s": npart / s_step,
        "pcg_iterations_per_step": iters,
        "pcg_outer_iterations_per_step": sum(i["outer_iterations"] for i in infos) / len(infos),
        "pcg_gbs_per_iteration": gbs_iter,
        "all_converged": all(i["converged"] for i in infos),
        "max_rel_res": max(i["rel_res"] for i in infos),
        "phases_ms": phases,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": gbs_dom,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs_dom / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "traffic_source": TRAFFIC_SOURCE if traffic else None},
        "_sim": sim, "_ctx": ctx, "_p": p, "_infos": infos,
    }


def bench_config4(args):
    """The 1024^3 standalone solves: the CIC deposit of 2^30 Landau particles
    (1 ppc, seed 20265) solved from zero to the same rtol three ways -- plain
    FP64 Jacobi-PCG (s-step form), the mixed form (reliable updates, inner
    tolerance 0.1) and the trained network's warm start followed by the mixed
    form -- with the s-step sweeps' kernel times of the FP64 solve."""
    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    N, ppc = 1024, 1
    p = P.landau_params(N, ppc, rtol=args.rtol, solver="pcg_fp64", check_every=32,
                        inner_rtol=0.1)
    ctx = P.Context(p)
    parts = synth.landau_particles_torch(N, ppc, seed=20265, device="cuda")
    rho = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
    ctx.deposit(parts[0], parts[1], parts[2], None, rho)
    del parts
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out = {"workload": "poisson_solve_1024^3_rhs_1ppc_landau", "rtol": args.rtol}
    n3 = N ** 3
    for name, solver, flags in (
            ("pcg_fp64", "pcg_fp64", 0),
            ("mixed", "pcg_mixed", P.FLAG_MIXED_RELIABLE),
            ("learned_mixed", "fcg_learned",
             P.FLAG_WARM_START_ONLY | P.FLAG_LEARNED_MIXED | P.FLAG_MIXED_RELIABLE)):
        if solver == "fcg_learned":
            load_weights(ctx, args.weights)
        ctx.set_flags(flags)
        ctx.set_solver(solver)
        phi = torch.zeros_like(rho)
        ctx.set_kernel_timing(name == "pcg_fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.poisson(rho, phi)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = {"s_per_solve": dt, "iterations": info["iterations"],
             "outer_iterations": info["outer_iterations"], "rel_res": info["rel_res"],
             "converged": bool(info["converged"])}
        if solver == "fcg_learned":
            r["warm_start_used"] = bool(info["warm_start_used"])
        if name == "pcg_fp64":
            ms_g, c_g = ctx.kernel_time(0)
            ms_u, c_u = ctx.kernel_time(1)
            r["kernels"] = {
                "pcg_sstep_gram": {"avg_ms": ms_g, "launches_timed": c_g,
                                   "gbs": SSTEP_GRAM_BYTES * n3 / (ms_g * 1e-3) / 1e9
                                   if ms_g > 0 else 0.0},
                "pcg_sstep_update": {"avg_ms": ms_u, "launches_timed": c_u,
                                     "gbs": SSTEP_UPD_BYTES * n3 / (ms_u * 1e-3) / 1e9
                                     if ms_u > 0 else 0.0}}
        ctx.set_kernel_timing(False)
        out[name] = r
        log("1024^3 %s: %.2f s, %d iterations, rel_res %.2e" % (name, dt, info["iterations"],
                                                              info["rel_res"]))
        del phi
    ctx.close()
    del ctx, rho
    torch.cuda.empty_cache()
    return out


def bench_config0(args):
    """The small configuration (32^3, 8 ppc, plain FP64 Jacobi-PCG, dt 0.05,
    20 steps after 2 warm-up steps): seconds per step and iterations."""
    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    N, ppc, steps = 32, 8, 20
    p = P.landau_params(N, ppc, rtol=args.rtol, check_every=32)
    ctx = P.Context(p)
    sim = P.Simulation(ctx, *synth.landau_particles_torch(N, ppc, seed=20260, device="cuda"))
    sim.init()
    for _ in range(2):
        sim.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [sim.step() for _ in range(steps)]
    torch.cuda.synchronize()
    s = (time.perf_counter() - t0) / steps
    ctx.close()
    return {"workload": "landau_damping_32^3_8ppc_pcg_fp64", "steps": steps, "warmup": 2,
            "s_per_step": s, "particles_per_s": ppc * N ** 3 / s,
            "pcg_iterations_per_step": sum(i["iterations"] for i in infos) / steps,
            "all_converged": all(i["converged"] for i in infos)}


if __name__ == "__main__":
    main()
