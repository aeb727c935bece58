"""Benchmark: DP-steps/s of the MCD hot path on one MI355X.

Default line: the 128^3 moving sphere (2.1 M cells, D = 0.25 of the box,
oscillating with A = 0.2 D, Re = 100) in the metric's two forms, one after
the other in one invocation:
  plain        FP64 weights, FP64 Bi-CGSTAB from the previous pressure;
  learned+mixed  the learned initial guess (3D U-Net, BF16 MFMA), FP64
               Bi-CGSTAB right-preconditioned by one FP32 multigrid V-cycle
               (the stencil products of the preconditioner in FP32; FP64 for
               the weights, the outer products, residuals and inner
               products).
A step is: DP rearrangement and role reassignment, remap, MLS weights of the
velocity and pressure sets, u* and the PPE right-hand side, Bi-CGSTAB to a
true relative residual of 1e-8 on the FP64 operator, projection.  Inputs are
resident in HBM before the timed region starts.  `value` is the plain FP64
form's DP-steps/s; the learned+mixed form sits beside it with its own
figures and its error against the plain form.  Prints one JSON line.

Other workloads: --workload cylinder|tgv|flapping|manufactured (1024^2
oscillating cylinder with both forms; 512^2 Taylor-Green vortex and 512^2
flapping wing in plain FP64; 32^2 manufactured Poisson, a latency figure).
A single form: --precision, --guess, --precond, --weights.  Measurement
aids: --mode sweep (stage-kernel bandwidth on large periodic meshes, with a
measured device copy for comparison), --mode copy (known-size copies for
calibrating hardware byte counters).

--gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DP-steps/s (MLS build + PPE to rel-res 1e-8), plain FP64 vs learned+mixed"
HBM_PEAK_GBS = 8000.0
WEIGHTS = {"sphere": "paper_2404_17542_amd/weights/unet_c4_128.npz",
           "cylinder": "paper_2404_17542_amd/weights/unet_c3_1024.npz"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes(n_unknown, dim, matrix_bytes, vector_bytes, stage="S", centre_formed=False):
    """Algorithmic bytes of one stage launch over n_unknown rows: the 3^dim
    matrix planes plus, S-stage (s = r - alpha v; t = A s), r, v, rhat read
    and s, t written (5 vector streams); P-stage (r, x, p updates; v = A p),
    s, t, p, v, x, rhat read and r, p', x, v' written (10 streams).
    centre_formed (the stages on the set's own FP64 operator): the 3^dim - 1
    off-centre planes, the kernel forming the centre from them, and in 3D the
    row's 1-byte unknown flag (rows of cells that are not unknown are not
    read)."""
    slots = 3 ** dim
    streams = 5 if stage == "S" else 10
    if centre_formed:
        per_row = (slots - 1) * matrix_bytes + (1 if dim == 3 else 0)
    else:
        per_row = slots * matrix_bytes
    return n_unknown * (per_row + streams * vector_bytes)


PRECISIONS = {"fp64": ("PREC_FP64", 8, 8, "f64", "FP64"),
              "mixed": ("PREC_FP32_MATRIX", 4, 8, "f32 matrix + f64",
                        "FP32-stored matrix, FP64 vectors, FP64 residual replacement"),
              "refine": ("PREC_FP32_REFINE", 4, 4, "f32 + f64 refinement",
                         "FP32 Bi-CGSTAB inside FP64 refinement")}


def make_case(workload, n, steps):
    from paper_2404_17542_amd import configs
    if workload == "tgv":
        return configs.c1_taylor_green(n=n or 512, steps=steps)
    if workload == "cylinder":
        return configs.c2_oscillating_cylinder(n=n or 1024, steps=steps)
    if workload == "flapping":
        return configs.c6_flapping_ellipse(n=n or 512, steps=steps)
    return configs.c4_moving_sphere(n=n or 128, steps=steps)


def workload_name(case, n_active):
    grid = "x".join(str(v) for v in case.n)
    if case.name.startswith("C1"):
        what = "periodic Taylor-Green vortex"
    elif case.name.startswith("C2"):
        what = "oscillating cylinder (D=1, A=0.2D, moving DPs and roles)"
    elif case.name.startswith("C6"):
        what = ("flapping elliptic wing (chord 1, aspect 4, discrete SDF at posture theta(t), "
                "translating and rotating, moving DPs and roles)")
    else:
        what = "moving sphere (D=0.25 of the box, A=0.2D, Re=100, moving DPs and roles)"
    stencil = "3x3" if case.dim == 2 else "3x3x3"
    return (f"{what} {grid}, {n_active} active DPs (one per cell, +-0.2 l0 jitter), "
            f"quadratic MLS {stencil}, PPE Bi-CGSTAB to 1e-8")


def measured_traffic(workload_key, dim, stage):
    """HBM bytes per launch of the stage kernel from the committed counter
    summary of this workload, or None when there is none or the kernel source
    has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_k_t{dim}_{workload_key}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    with open(os.path.join(ROOT, d["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != d["source_sha256"]:
            return None
    if stage == "S":
        return d["bytes_per_launch"]
    return d.get("p_stage", {}).get("bytes_per_launch")


# ---------------------------------------------------------------------------
# one form of the time step
# ---------------------------------------------------------------------------

def run_form(case, args, precision, guess, precond, weights, label):
    """Warm-up, autotune, `args.steps` timed steps, then kernel timing and
    the error against the plain FP64 solve on one more step.  Returns a dict
    of figures (the simulation object is released)."""
    import torch

    from paper_2404_17542_amd import mcd
    from paper_2404_17542_amd.sim import GpuSim

    prec_name, mat_b, vec_b, dtype, prec_text = PRECISIONS[precision]
    if precond == "mg":
        dtype = ("f32 matrix products + f32 multigrid, f64 vectors and residual" if precision == "mixed"
                 else "f64 Krylov + f32 multigrid")
    log(f"{label}: setting up {case.name} ({prec_text}, guess {guess}, preconditioner {precond})")
    sim = GpuSim(case, precision=getattr(mcd, prec_name), update_info=False,
                 precond={"none": mcd.PRECOND_NONE, "jacobi": mcd.PRECOND_JACOBI, "mg": mcd.PRECOND_MG}[precond],
                 graph=not args.no_step_graph)
    if guess == "learned":
        from paper_2404_17542_amd import learned
        sim.model = learned.load_model(sim.ctx, os.path.join(ROOT, weights))
    sim.guess = guess
    for _ in range(args.warmup):
        sim.step()
    torch.cuda.synchronize()
    tune = None
    if not args.no_autotune and precond != "mg":      # the multigrid path does not use the stage kernels
        tune = sim.ctx.autotune(sim.tuning_set())
        log(f"{label}: autotuned stage-kernel shape {tune['shape']} from "
            + ", ".join(f"{c['grid']}x{c['depth']}: {c['us_per_iter']:.2f} us" for c in tune["candidates"]))
    n_active = sim.n_active()
    # Python's cyclic garbage collector stays off over the timed steps (a
    # collection can pause the host for tens of milliseconds between two
    # launches); every step's device work runs as without it
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            sim.step()
            if (k + 1) % 10 == 0:
                log(f"{label}: step {k + 1}/{args.steps}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    finally:
        gc.enable()
    timed = sim.log[-args.steps:]
    assert all(r["converged"] for r in timed), "a PPE solve did not converge"
    iters = [r["iters"] for r in timed]
    out = {"value": n_active * args.steps / elapsed, "ms_per_step": elapsed / args.steps * 1e3,
           "dps": n_active, "precision": precision, "dtype": dtype, "initial_guess": guess,
           "preconditioner": precond, "ppe_iters_per_step": sum(iters) / len(iters),
           "max_true_rel_res": max(r["rel_res"] for r in timed), "stage_shape": sim.ctx.get_shape(),
           "autotuned": tune is not None, "step_graphs": sim.graph}
    if guess == "learned":
        out["weights"] = weights
    if not args.no_kernel_timing and args.timing_steps > 0:
        # the same operator, vectors and launch shape; every stage launch carries
        # start/stop events stamped by its own dispatch on the solve stream
        sim.ctx.profile(True)
        sim.ctx.profile_read_split(reset=True)
        for _ in range(args.timing_steps):
            sim.step()
        torch.cuda.synchronize()
        prof = sim.ctx.profile_read_split(reset=True)
        sim.ctx.profile(False)
        n_unk = sim.ctx_unknown_count()
        stages = {}
        for stage in ("P", "S"):
            ms = n = nbytes = 0.0
            for mat, mb in (("fp64", 8), ("fp32", 4)):
                k = stage.lower()
                ms += prof[mat][f"{k}_ms"]
                n += prof[mat][f"{k}_n"]
                # the Jacobi-scaled copy stores its centre; the set's operator does not need it
                cf = mb == 8 and precond != "jacobi"
                nbytes += prof[mat][f"{k}_n"] * stage_bytes(n_unk, case.dim, mb, vec_b, stage, cf)
            if n:
                avg_s = ms / n * 1e-3
                stages[stage] = {"kernel": f"k_t{case.dim}_{stage}", "launches": int(n), "total_ms": ms,
                                 "avg_us": avg_s * 1e6, "bytes_per_launch": nbytes / n,
                                 "achieved_GBs": nbytes / n / avg_s / 1e9,
                                 "fp32_matrix_launches": int(prof["fp32"][f"{stage.lower()}_n"])}
        out["stages"] = stages
        out["unknowns"] = n_unk
        out["timed_launches_from"] = f"{args.timing_steps} steps after the timed region"
    if precision != "fp64" or guess != "warm" or precond != "none":
        out["error_vs_plain_fp64"] = error_vs_plain_fp64(sim, mcd)
    out["graph_fallbacks"] = sim.graph_fallbacks
    sim.ctx.close()
    del sim
    gc.collect()
    torch.cuda.empty_cache()
    return out


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


# ---------------------------------------------------------------------------
# CPU oracle baseline on a bounded sample of the workload
# ---------------------------------------------------------------------------

def cpu_baseline_full_steps(case, steps):
    """The oracle on `steps` whole projection steps (after its initial
    arrangement and weights), one thread; for workloads whose oracle step
    takes seconds."""
    from threadpoolctl import threadpool_limits

    from oracle.sim import OracleSim
    with threadpool_limits(limits=1):
        sim = OracleSim(case)
        n_active = int((sim.role != 0).sum())
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step()
        dt = time.perf_counter() - t0
    grid = "x".join(str(v) for v in case.n)
    return {"value": n_active * steps / dt, "unit": "DP-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} whole projection steps of the same {grid} workload (after its initial "
                      f"arrangement and weights), numpy/scipy FP64, 1 thread, {dt:.1f} s; host "
                      f"{platform.processor() or platform.machine()}, {os.cpu_count()} logical CPUs"}


def _sampled_step(case, iters_per_step, n_sample, n_iters, threads):
    """The oracle's cost of one step of the full-size workload from bounded
    samples, with the BLAS thread pools limited to `threads`:
      DP update   the oracle's update_dps on the whole mesh (from the seeded
                  positions and the t = 0 masks, one step's sweeps);
      weights     mls_build of the velocity and the pressure set on n_sample
                  random DPs, scaled to every active DP;
      field ops   the weight applications of one step (remap, MOC + viscous
                  term, divergence: three components each; pressure gradient)
                  on the same DPs, scaled likewise;
      PPE         n_iters of the oracle's Bi-CGSTAB on an operator with the
                  workload's size and 3^dim sparsity, per iteration times the
                  plain form's measured iterations per step.
    Returns (active DPs, seconds per step, phase seconds, sample text)."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import mcd_oracle as O
    from oracle.sim import oracle_bodies
    from paper_2404_17542_amd import inputs

    t_start = time.perf_counter()
    with threadpool_limits(limits=threads):
        m = O.Mesh.from_case(case)
        consts = O.RelaxConsts.make(case.l0, case.kappa, case.eps_relax, case.band_over_l0, case.fit_alpha,
                                    case.fit_re_over_l0)
        pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
        b0, b1 = oracle_bodies(case, 0.0), oracle_bodies(case, case.dt)
        role0 = O.roles(m, b0)
        t0 = time.perf_counter()
        up = O.update_dps(m, consts, b1, pos, role0, case.n_relax)
        t_update = time.perf_counter() - t0
        n_active = int((up.role != O.VOID).sum())
        rng = np.random.Generator(np.random.PCG64(12345))
        act = np.nonzero(up.role != O.VOID)[0]
        idx = np.sort(rng.choice(act, min(n_sample, len(act)), replace=False))
        re, rs = case.re_over_l0 * case.l0, case.rs_over_l0 * case.l0
        t0 = time.perf_counter()
        st_u = O.mls_build(m, up.pos, up.role, up.normal, case.bc_velocity, re, rs, case.weight, idx=idx)
        st_p = O.mls_build(m, up.pos, up.role, up.normal, case.bc_pressure, re, rs, case.weight, idx=idx)
        t_build = time.perf_counter() - t0
        u = rng.standard_normal((case.dim, m.Nc))
        p = rng.standard_normal(m.Nc)
        t0 = time.perf_counter()
        shift = up.pos[:, idx] - pos[:, idx]
        for a in range(case.dim):                                      # remap
            Phi = O.poly_coeffs(m, st_u, u[a])
            O.taylor_shift(u[a, idx], Phi, shift, rs)
        for a in range(case.dim):                                      # MOC + viscous
            Phi = O.poly_coeffs(m, st_u, u[a])
            O.taylor_shift(u[a, idx], Phi, -u[:, idx] * case.dt, rs) + O.lap_from_phi(Phi, rs, case.dim)
        acc = 0.0
        for a in range(case.dim):                                      # divergence
            acc = acc + O.poly_coeffs(m, st_u, u[a])[a] / rs
        O.grad_from_phi(O.poly_coeffs(m, st_p, p), rs, case.dim)      # projection
        t_ops = time.perf_counter() - t0
        # an operator of the workload's size and sparsity (3^dim slots per row)
        cols, rows = [], []
        ijk = m.ijk(np.arange(m.Nc))
        for off in m.offsets:
            j, _ = m.neighbour(ijk, off)
            ok = j >= 0
            rows.append(np.nonzero(ok)[0])
            cols.append(j[ok])
        r_ = np.concatenate(rows)
        c_ = np.concatenate(cols)
        vals = np.where(r_ == c_, -float(len(m.offsets)), 1.0) + 0.01 * rng.standard_normal(len(r_))
        A = sp.csr_matrix((vals, (r_, c_)), shape=(m.Nc, m.Nc))
        b = rng.standard_normal(m.Nc)
        t0 = time.perf_counter()
        _, info = O.bicgstab(A, b, np.zeros(m.Nc), 1e-30, max_iter=n_iters)
        t_iter = (time.perf_counter() - t0) / max(info.iterations, 1)
    scale = n_active / len(idx)
    t_step = t_update + (t_build + t_ops) * scale + t_iter * iters_per_step
    grid = "x".join(str(v) for v in case.n)
    sample = (f"one step of the same {grid} workload assembled from bounded samples of the oracle "
              f"(numpy/scipy FP64, BLAS limited to {threads} thread(s)): DP update on the whole mesh "
              f"{t_update:.1f} s; MLS weights of both sets on {len(idx)} random DPs {t_build:.1f} s and their "
              f"field operations {t_ops:.1f} s, both scaled by {scale:.1f} to every active DP; "
              f"{info.iterations} Bi-CGSTAB iterations on an operator of the workload's size and sparsity, "
              f"{t_iter:.3f} s each, times the plain form's {iters_per_step:.0f} iterations per step; "
              f"estimated step {t_step:.0f} s, measured in {time.perf_counter() - t_start:.0f} s")
    phases = {"update": t_update, "weights": t_build * scale, "field_ops": t_ops * scale,
              "ppe": t_iter * iters_per_step}
    return n_active, t_step, phases, sample


def host_cores():
    """Logical CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_baseline_sampled(case, iters_per_step, n_sample=1 << 18, n_iters=48):
    """The oracle's cost of one step of the full-size workload, measured on
    bounded samples (`_sampled_step`), once with one thread (the reported
    `value`) and once with every host core available to the BLAS pools (the
    oracle's elementwise numpy work and scipy's sparse products run on one
    thread either way)."""
    host = f"host {platform.processor() or platform.machine()}, {host_cores()} logical CPUs available"
    n_active, t1, ph1, s1 = _sampled_step(case, iters_per_step, n_sample, n_iters, 1)
    nc = host_cores()
    _, tn, phn, _ = _sampled_step(case, iters_per_step, n_sample, n_iters, nc)
    return {"value": n_active / t1, "unit": "DP-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{s1}; {host}", "phases_s": ph1,
            "all_cores": {"value": n_active / tn, "cores": nc, "phases_s": phn,
                          "sample": "the same sample with the BLAS thread pools at every available core"}}


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

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


def roofline_of(form, case, key):
    """Roofline object of the dominant stage kernel (the larger total time)
    of a form's timed launches."""
    st = form.get("stages") or {}
    if not st:
        return None
    name = max(st, key=lambda k: st[k]["total_ms"])
    d = st[name]
    other = {k: {"avg_us": v["avg_us"], "achieved_GBs": v["achieved_GBs"],
                 "frac": v["achieved_GBs"] / HBM_PEAK_GBS, "bytes_per_launch": v["bytes_per_launch"]}
             for k, v in st.items() if k != name}
    return {"bound": "hbm", "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["achieved_GBs"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(key, case.dim, name) if form["precision"] == "fp64" else None,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
            "kernel": f"{d['kernel']}<double, double> (Bi-CGSTAB {name}-stage)", "avg_us": d["avg_us"],
            "launches": d["launches"], "bytes_per_launch": d["bytes_per_launch"],
            "unknowns": form.get("unknowns"), "timed_launches_from": form.get("timed_launches_from"),
            "other_stage": other}


def bench_step(args):
    import torch

    from paper_2404_17542_amd import mcd

    torch.cuda.set_device(0)
    mcd.load()
    case = make_case(args.workload, args.n, args.steps)
    single = (args.precision is not None or args.guess is not None or args.precond is not None
              or args.weights is not None or args.workload not in WEIGHTS or args.form == "plain")
    plain = run_form(case, args, args.precision or "fp64", args.guess or "warm", args.precond or "none",
                     args.weights, "plain" if not single else "form")
    other = None
    if not single:
        other = run_form(case, args, "mixed", "learned", "mg", WEIGHTS[args.workload], "learned+mixed")
    flow = {"C1": "taylor_green", "C2": "cylinder", "C4": "sphere", "C6": "flapping"}[case.name[:2]]
    key = f"{flow}_{case.n[0]}_{plain['precision']}"
    prec_text = PRECISIONS[plain["precision"]][4]
    config = {"workload": workload_name(case, plain["dps"]) + f" ({prec_text})",
              "forms": "plain FP64 (value) and learned+mixed (learned_mixed)" if other else "one form",
              **{k: plain[k] for k in ("dps", "precision", "initial_guess", "preconditioner", "stage_shape",
                                       "autotuned", "step_graphs", "ppe_iters_per_step", "max_true_rel_res",
                                       "graph_fallbacks")}}
    if "error_vs_plain_fp64" in plain:
        config["error_vs_plain_fp64"] = plain["error_vs_plain_fp64"]
    out = {"metric": METRIC, "value": plain["value"], "unit": "DP-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": plain["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": plain["dtype"], "data": "synthetic",
           "config": config, "roofline": roofline_of(plain, case, key)}
    if other:
        lm = {k: other[k] for k in ("value", "ms_per_step", "dtype", "ppe_iters_per_step", "max_true_rel_res",
                                    "error_vs_plain_fp64", "stage_shape", "graph_fallbacks", "weights")}
        lm["form"] = ("learned initial guess; Bi-CGSTAB with FP64 vectors and inner products whose matrix "
                      "products read the FP32 copy of the matrix (difference form), right-preconditioned by one "
                      "FP32 multigrid V-cycle (Galerkin levels built every solve); the FP64 residual confirms "
                      "the tolerance and restarts a run that missed it")
        lm["speedup_vs_plain"] = other["value"] / plain["value"]
        lm["stages"] = other.get("stages")
        out["learned_mixed"] = lm
    if not args.no_cpu_baseline:
        if case.dim == 2 and case.n_cells <= 1 << 18:
            log(f"timing the CPU oracle on {args.cpu_steps} steps")
            out["cpu_baseline"] = cpu_baseline_full_steps(case, args.cpu_steps)
        else:
            log("timing the CPU oracle on bounded samples of one step")
            out["cpu_baseline"] = cpu_baseline_sampled(case, plain["ppe_iters_per_step"])
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# measurement aids
# ---------------------------------------------------------------------------

def copy_rate(nbytes, reps=10):
    """Device-to-device copy of nbytes (read + write), timed by events: the
    measured streaming rate the stage kernels are compared with."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    assert torch.equal(dst[:: 1 << 16], src[:: 1 << 16])
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / s / 1e9


def sweep_size(n, iters, precision):
    """Stage kernels of the 2D Bi-CGSTAB on a periodic n x n mesh (jittered
    DPs, every DP inner, quadratic MLS Laplacian, one DP pinned), a seeded
    right-hand side and `iters` iterations (tolerance out of reach); every
    stage launch timed by HIP events on the solve stream."""
    import numpy as np
    import torch

    from paper_2404_17542_amd import configs, inputs
    from paper_2404_17542_amd import mcd as M
    case = configs.c1_taylor_green(n=n, steps=1)
    ctx = M.Context.from_case(case)
    f64 = dict(dtype=torch.float64, device="cuda")
    pos = torch.tensor(inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed), **f64)
    role = torch.full((case.n_cells,), M.ROLE_INNER, dtype=torch.int8, device="cuda")
    normal = torch.zeros_like(pos)
    ctx.build_stencils(0, pos, role, normal, case.bc_pressure, pin_first=True)
    rng = np.random.Generator(np.random.PCG64(n))
    rhs = torch.tensor(rng.standard_normal(case.n_cells), **f64)
    p = torch.zeros_like(rhs)
    prec = {"fp64": M.PREC_FP64, "mixed": M.PREC_FP32_MATRIX}[precision]
    mb = 8 if precision == "fp64" else 4
    ctx.solve_ppe(0, rhs, p, tol=1e-30, max_iter=iters, precision=prec, fp64_below=0.0, raise_on_fail=False)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    p.zero_()
    info = ctx.solve_ppe(0, rhs, p, tol=1e-30, max_iter=iters, precision=prec, fp64_below=0.0,
                         raise_on_fail=False)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    n_unk = case.n_cells - 1
    sb, pb = stage_bytes(n_unk, 2, mb, 8, "S", mb == 8), stage_bytes(n_unk, 2, mb, 8, "P", mb == 8)
    s_us = prof["s_ms"] / max(prof["s_n"], 1) * 1e3
    p_us = prof["p_ms"] / max(prof["p_n"], 1) * 1e3
    out = {"n": n, "unknowns": n_unk, "precision": precision, "iterations": info["iterations"],
           "s_launches": prof["s_n"], "s_avg_us": s_us, "s_bytes": sb, "s_GBs": sb / s_us / 1e3,
           "p_launches": prof["p_n"], "p_avg_us": p_us, "p_bytes": pb, "p_GBs": pb / p_us / 1e3,
           "shape": ctx.get_shape()}
    ctx.close()
    del ctx, pos, role, normal, rhs, p
    gc.collect()
    torch.cuda.empty_cache()
    return out


def bench_sweep(args):
    import torch

    from paper_2404_17542_amd import mcd
    torch.cuda.set_device(0)
    mcd.load()
    res = []
    for s in args.sizes.split(","):
        r = sweep_size(int(s), args.sweep_iters, args.precision or "fp64")
        r["copy_GBs"] = copy_rate(r["s_bytes"])
        for k in ("s", "p"):
            r[f"{k}_frac"] = r[f"{k}_GBs"] / HBM_PEAK_GBS
            r[f"{k}_frac_of_copy"] = r[f"{k}_GBs"] / r["copy_GBs"]
        log(f"{r['n']}^2 {r['precision']}: S {r['s_avg_us']:.1f} us {r['s_GBs']:.0f} GB/s "
            f"({100 * r['s_frac']:.0f} % of peak), P {r['p_avg_us']:.1f} us {r['p_GBs']:.0f} GB/s "
            f"({100 * r['p_frac']:.0f} %), copy of the S-stage bytes {r['copy_GBs']:.0f} GB/s")
        res.append(r)
    print(json.dumps(res), flush=True)


def bench_copy(args):
    """Plain device-to-device copies of a known size, for calibrating hardware
    byte counters (divide the known bytes by what a counter reports for these
    dispatches)."""
    import torch
    n = args.mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:: 1 << 16], src[:: 1 << 16])
    print(f"copied {args.mib} MiB x {args.reps} (read {args.mib} MiB and write {args.mib} MiB per dispatch)",
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["step", "sweep", "copy"], default="step")
    ap.add_argument("--workload", choices=["sphere", "cylinder", "tgv", "flapping", "manufactured"],
                    default="sphere",
                    help="sphere: 128^3 moving sphere (default line); cylinder: 1024^2 oscillating cylinder; "
                         "tgv: 512^2 periodic Taylor-Green; flapping: 512^2 hovering elliptic wing")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--form", choices=["metric", "plain"], default="metric",
                    help="metric: plain FP64 and learned+mixed (workloads with a trained network); plain: only "
                         "the plain FP64 form")
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default=None)
    ap.add_argument("--guess", choices=["warm", "zero", "learned"], default=None,
                    help="PPE initial guess: previous pressure, zero, or the learned correction")
    ap.add_argument("--weights", default=None, help="network weights for --guess learned")
    ap.add_argument("--precond", choices=["none", "jacobi", "mg"], default=None,
                    help="none: the plain method; jacobi: diagonal right preconditioning; mg: one FP32 multigrid "
                         "V-cycle as right preconditioner (FP64 outer iteration)")
    ap.add_argument("--no-step-graph", action="store_true",
                    help="issue the calls around the PPE solve one by one instead of as recorded HIP graphs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default stage-kernel shape instead of timing the candidates after warm-up")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=3,
                    help="steps after the timed region whose stage kernels are timed one by one")
    ap.add_argument("--sizes", default="1024,2048,4096,8192", help="--mode sweep: mesh sizes")
    ap.add_argument("--sweep-iters", type=int, default=64, help="--mode sweep: iterations per size")
    ap.add_argument("--mib", type=int, default=1024, help="--mode copy: bytes copied per dispatch, in MiB")
    ap.add_argument("--reps", type=int, default=5, help="--mode copy: dispatches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is not built.",
              file=sys.stderr)
        sys.exit(2)
    if args.mode == "sweep":
        return bench_sweep(args)
    if args.mode == "copy":
        return bench_copy(args)
    if args.workload == "manufactured":
        return bench_manufactured(args)
    if args.guess == "learned" and not args.weights:
        args.weights = WEIGHTS.get(args.workload)
        if args.weights is None:
            raise SystemExit("--guess learned needs --weights (written by paper_2404_17542_amd.learned)")
    return bench_step(args)


if __name__ == "__main__":
    main()
