"""Benchmark: DP-steps/s of the MCD hot path on one MI355X.

A step is one projection step of the 512x512 periodic Taylor-Green vortex
(262,144 DPs): DP update and role pass, remap, MLS weights for every DP,
u* and the PPE right-hand side, Bi-CGSTAB to a true relative residual of
1e-8 (FP64), projection.  Inputs are resident in HBM before the timed
region starts.  Prints one JSON line.

Other forms: --workload cylinder|sphere|flapping|manufactured (flapping: the
512x512 hovering elliptic wing, a rotating discrete-SDF body; manufactured: the 32x32
manufactured-solution Poisson problem, a step being the MLS build plus one
PPE solve from zero, a latency figure), --precision mixed (FP32-stored
matrix with FP64 residual replacement) or refine (FP32 Bi-CGSTAB inside
FP64 refinement), --guess zero|learned (--weights: a file written by
paper_2404_17542_amd.learned).  The tolerance is checked on the FP64
operator in every form.

--gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DP-steps/s (MLS build + PPE to rel-res 1e-8), plain FP64 vs learned+mixed"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes(n_unknown, dim, matrix_bytes, vector_bytes):
    """Algorithmic bytes of one S-stage launch (s = r - alpha v; t = A s):
    A (3^dim planes) + r, v, rhat read once + s, t written once."""
    slots = 3 ** dim
    return n_unknown * (slots * matrix_bytes + 5 * vector_bytes)


PRECISIONS = {"fp64": ("PREC_FP64", 8, 8, "f64", "FP64"),
              "mixed": ("PREC_FP32_MATRIX", 4, 8, "f32 matrix + f64",
                        "FP32-stored matrix, FP64 vectors, FP64 residual replacement"),
              "refine": ("PREC_FP32_REFINE", 4, 4, "f32 + f64 refinement",
                         "FP32 Bi-CGSTAB inside FP64 refinement")}


def workload_name(case, n_active, precision):
    grid = "x".join(str(v) for v in case.n)
    if case.name.startswith("C1"):
        what = "periodic Taylor-Green vortex"
    elif case.name.startswith("C2"):
        what = "oscillating cylinder (D=1, A=0.2D, moving DPs and roles)"
    elif case.name.startswith("C6"):
        what = ("flapping elliptic wing (chord 1, aspect 4, discrete SDF at posture theta(t), "
                "translating and rotating, moving DPs and roles)")
    else:
        what = "moving sphere (D=0.25, A=0.2D, moving DPs and roles)"
    stencil = "3x3" if case.dim == 2 else "3x3x3"
    return (f"{what} {grid}, {n_active} active DPs (one per cell, +-0.2 l0 jitter), Re=100, "
            f"quadratic MLS {stencil}, PPE Bi-CGSTAB to 1e-8 ({precision})")


def measured_traffic(workload_key, dim=2):
    """HBM bytes per S-stage launch from the committed counter summary of this
    workload, or None when there is none or the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_k_t{dim}_{workload_key}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    with open(os.path.join(ROOT, d["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != d["source_sha256"]:
            return None
    return d["bytes_per_launch"]


def cpu_baseline(case, steps):
    from threadpoolctl import threadpool_limits

    from oracle.sim import OracleSim
    with threadpool_limits(limits=1):
        sim = OracleSim(case)
        n_active = int((sim.role != 0).sum())
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step()
        dt = time.perf_counter() - t0
    return {"value": n_active * steps / dt, "unit": "DP-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} projection steps of the same {case.n[0]}x{case.n[1]} workload "
                      f"(after its initial arrangement and weights), numpy/scipy FP64, 1 thread, "
                      f"{dt:.1f} s; host {platform.processor() or platform.machine()}, "
                      f"{os.cpu_count()} logical CPUs"}


def bench_manufactured(args):
    """32x32 unit square, p = sin 2pi x sin 2pi y with Dirichlet walls and the
    Gaussian weight: each step rebuilds the weights and solves the PPE from
    zero to 1e-8 (FP64).  Latency of the smallest configuration."""
    import numpy as np
    import torch

    from paper_2404_17542_amd import configs, inputs, mcd
    from paper_2404_17542_amd.sim import GpuSim

    torch.cuda.set_device(0)
    mcd.load()
    case = configs.c0_manufactured(n=args.n or 32)
    sim = GpuSim(case, update_info=False)
    ctx = sim.ctx
    pos_h = sim.pos.cpu().numpy()
    role_h = sim.role.cpu().numpy()
    rhs = torch.tensor(inputs.manufactured_rhs(pos_h), dtype=torch.float64, device="cuda")
    g = np.where(role_h == mcd.ROLE_INNER, 0.0, inputs.manufactured_pressure(pos_h))
    p0 = torch.tensor(g, dtype=torch.float64, device="cuda")
    p = p0.clone()

    def step():
        ctx.build_stencils(0, sim.pos, sim.role, sim.normal, case.bc_pressure)
        p.copy_(p0)
        return ctx.solve_ppe(0, rhs, p, tol=1e-8, guess=mcd.GUESS_ZERO)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(i["converged"] for i in infos)
    n_active = int((role_h != mcd.ROLE_VOID).sum())
    err = np.abs(p.cpu().numpy() - inputs.manufactured_pressure(pos_h))[role_h == mcd.ROLE_INNER].max()
    out = {"metric": METRIC, "value": n_active * args.steps / elapsed, "unit": "DP-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"manufactured Poisson p = sin(2 pi x) sin(2 pi y), unit square "
                                  f"{case.n[0]}x{case.n[1]}, {n_active} DPs (+-0.2 l0 jitter, walls on the "
                                  f"boundary), Gaussian-weight quadratic MLS 3x3, Dirichlet walls, one PPE "
                                  f"solve from zero to 1e-8 (FP64) per step",
                      "dps": n_active, "precision": "fp64", "initial_guess": "zero",
                      "ppe_iters_per_step": sum(i["iterations"] for i in infos) / len(infos),
                      "max_true_rel_res": max(i["true_rel_residual"] for i in infos),
                      "max_abs_error_vs_exact": float(err)},
           "roofline": None}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import mcd_oracle as O
        m = O.Mesh.from_case(case)
        nrm = sim.normal.cpu().numpy()
        with threadpool_limits(limits=1):
            reps = 0
            t0 = time.perf_counter()
            while reps < 5 or time.perf_counter() - t0 < 2.0:
                st = O.mls_build(m, pos_h, role_h, nrm, case.bc_pressure, case.re_over_l0 * case.l0, case.l0,
                                 case.weight)
                O.solve_ppe(m, st, role_h, case.bc_pressure, inputs.manufactured_rhs(pos_h), g, None, 1e-8)
                reps += 1
            dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_active * reps / dt, "unit": "DP-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{reps} steps (MLS build + PPE solve) of the same problem, numpy/scipy "
                                         f"FP64, 1 thread, {dt:.1f} s"}
    print(json.dumps(out), flush=True)


def error_vs_plain_fp64(sim, mcd):
    """One extra (untimed) step: its PPE is solved by the form under test and,
    from the same previous pressure, by the plain method (FP64, warm start, no
    preconditioner); returns ||P_form - P_plain|| / ||P_plain|| over unknown
    DPs.  The step then continues with the form's solution."""
    import torch
    pset, bodies_new, upd = sim.prepare()
    p_k = sim.P.clone()
    info = sim.solve(pset, sim.initial_guess(pset, sim.guess))
    p_form = sim.P.clone()
    sim.P.copy_(p_k)
    sim.ctx.solve_ppe(pset, sim.rhs, sim.P, sim.fP, tol=sim.case.tol, precision=mcd.PREC_FP64,
                      guess=mcd.GUESS_CALLER, precond=mcd.PRECOND_NONE, check_every=sim.check_every)
    unk = sim.role == mcd.ROLE_INNER
    for bid, typ in sim.case.bc_pressure.items():
        if typ == mcd.BC_NEUMANN:
            unk |= sim.role == bid
    ref = sim.P[unk]
    rel = float(torch.linalg.vector_norm(p_form[unk] - ref) / torch.linalg.vector_norm(ref))
    sim.P.copy_(p_form)
    sim.finish(pset, bodies_new, info, upd)
    return rel


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["tgv", "cylinder", "sphere", "flapping", "manufactured"], default="tgv",
                    help="tgv: 512^2 periodic Taylor-Green (default line); cylinder: 1024^2 oscillating "
                         "cylinder; sphere: 128^3 moving sphere; flapping: 512^2 hovering elliptic wing")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default="fp64")
    ap.add_argument("--guess", choices=["warm", "zero", "learned"], default="warm",
                    help="PPE initial guess: previous pressure (default), zero, or the learned correction")
    ap.add_argument("--weights", default=None, help="network weights for --guess learned")
    ap.add_argument("--precond", choices=["none", "jacobi"], default="none",
                    help="none: the plain method (default); jacobi: diagonal right preconditioning")
    ap.add_argument("--no-step-graph", action="store_true",
                    help="issue the calls around the PPE solve one by one instead of as recorded HIP graphs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default stage-kernel shape instead of timing the candidates after warm-up")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=3,
                    help="steps after the timed region whose stage kernels are timed one by one")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is not built.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "manufactured":
        return bench_manufactured(args)

    import torch

    from paper_2404_17542_amd import configs, mcd
    from paper_2404_17542_amd.sim import GpuSim

    torch.cuda.set_device(0)
    mcd.load()
    if args.workload == "tgv":
        case = configs.c1_taylor_green(n=args.n or 512, steps=args.steps)
    elif args.workload == "cylinder":
        case = configs.c2_oscillating_cylinder(n=args.n or 1024, steps=args.steps)
    elif args.workload == "flapping":
        case = configs.c6_flapping_ellipse(n=args.n or 512, steps=args.steps)
    else:
        case = configs.c4_moving_sphere(n=args.n or 128, steps=args.steps)
    prec_name, mat_b, vec_b, dtype, prec_text = PRECISIONS[args.precision]
    prec = getattr(mcd, prec_name)
    log(f"setting up {case.name}")
    sim = GpuSim(case, precision=prec, update_info=False,
                 precond=mcd.PRECOND_JACOBI if args.precond == "jacobi" else mcd.PRECOND_NONE,
                 graph=not args.no_step_graph)
    if args.guess == "learned":
        if not args.weights:
            raise SystemExit("--guess learned needs --weights (written by paper_2404_17542_amd.learned)")
        from paper_2404_17542_amd import learned
        sim.model = learned.load_model(sim.ctx, args.weights)
    sim.guess = args.guess
    for _ in range(args.warmup):
        sim.step()
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} steps)")
    tune = None
    if not args.no_autotune:
        tune = sim.ctx.autotune(sim.tuning_set())
        log(f"autotuned stage-kernel shape: {tune['shape']} from "
            + ", ".join(f"{c['grid']}x{c['depth']}: {c['us_per_iter']:.2f} us" for c in tune["candidates"]))
    n_active = sim.n_active()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sim.step()
        if (k + 1) % 25 == 0:
            log(f"step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = sim.log[-args.steps:]
    iters = [r["iters"] for r in timed]
    worst = max(r["rel_res"] for r in timed)
    assert all(r["converged"] for r in timed), "a PPE solve did not converge"
    value = n_active * args.steps / elapsed
    roofline = None
    if not args.no_kernel_timing and args.timing_steps > 0:
        # same operator, vectors and launch shape; every stage launch carries
        # start/stop events stamped by its own dispatch
        sim.ctx.profile(True)
        sim.ctx.profile_read(reset=True)
        for _ in range(args.timing_steps):
            sim.step()
        torch.cuda.synchronize()
        prof = sim.ctx.profile_read(reset=True)
        sim.ctx.profile(False)
        n_unknown = int(sim.ctx_unknown_count()) if hasattr(sim, "ctx_unknown_count") else n_active
        bytes_per = stage_bytes(n_unknown, case.dim, mat_b, vec_b)
        avg_s = prof["s_ms"] / max(prof["s_n"], 1) * 1e-3
        achieved = bytes_per / avg_s / 1e9 if avg_s > 0 else None
        flow = {"C1": "taylor_green", "C2": "cylinder", "C4": "sphere", "C6": "flapping"}[case.name[:2]]
        traffic = measured_traffic(f"{flow}_{case.n[0]}_{args.precision}", case.dim)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                    "traffic_unit": "bytes per launch (FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
                    "kernel": f"k_t{case.dim}_S (Bi-CGSTAB S-stage: s = r - alpha v, t = A s, 4 dots)",
                    "avg_us": avg_s * 1e6, "launches": prof["s_n"], "bytes_per_launch": bytes_per,
                    "timed_launches_from": f"{args.timing_steps} steps after the timed region",
                    "p_stage_avg_us": prof["p_ms"] / max(prof["p_n"], 1) * 1e3}
    out = {"metric": METRIC, "value": value, "unit": "DP-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic",
           "config": {"workload": workload_name(case, n_active, prec_text),
                      "dps": n_active, "precision": args.precision, "initial_guess": args.guess,
                      "preconditioner": args.precond,
                      "stage_shape": sim.ctx.get_shape(), "autotuned": tune is not None,
                      "step_graphs": sim.graph,
                      "ppe_iters_per_step": sum(iters) / len(iters), "max_true_rel_res": worst},
           "roofline": roofline}
    if args.precision != "fp64" or args.guess != "warm" or args.precond != "none":
        # the error of this form against the plain FP64 method, on one more step
        out["config"]["error_vs_plain_fp64"] = error_vs_plain_fp64(sim, mcd)
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        log(f"timing the CPU oracle on {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
