"""Learned PPE initial guess: data set, training and evaluation on the GPU.

Not part of the MCD method.  A U-Net on the background mesh (libmcd's
BF16-MFMA kernels, see mcd_model_* in mcd.h) corrects the solver's warm
start: guess = P^k + s rms(r) h(r, P^k, roles), where r is the PPE residual
of P^k under the weights and right-hand side of step k+1.  The Bi-CGSTAB
solve still runs to the same tolerance, so the guess changes the iteration
count and never the accepted solution.

Data set: C2-shaped trajectories (configs.c3_cylinder_variant: seeded
amplitude, frequency and DP jitter), or C4-shaped ones for the 3D network
(configs.c4_sphere_variant), run with the plain method and the warm start.
After a spin-up, every step k -> k+1 gives one sample (r, P^k, roles,
P^{k+1}); P^{k+1} is the converged FP64 solution.

Everything here sequences libmcd calls; samples stay in device memory.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import configs
from . import mcd as M
from .sim import GpuSim

DEFAULT_CHANNELS = (16, 32, 64, 128)


@dataclass
class Sample:
    resid: torch.Tensor     # PPE residual of p_prev (f64 [Nc])
    p_prev: torch.Tensor    # warm start P^k
    p_next: torch.Tensor    # converged P^{k+1}
    role: torch.Tensor      # roles at k+1 (i8 [Nc])


def unknown_mask(role, bc):
    unk = role == M.ROLE_INNER
    for bid, typ in bc.items():
        if typ == M.BC_NEUMANN:
            unk |= role == bid
    return unk


VARIANTS = {"cylinder": configs.c3_cylinder_variant, "sphere": configs.c4_sphere_variant}
BASE_CASES = {"cylinder": configs.c2_oscillating_cylinder, "sphere": configs.c4_moving_sphere}


def collect(seeds, n, n_spin, n_save, log=print, flow="cylinder"):
    """Samples of the trajectories `seeds` (plain FP64 method, warm start)."""
    out = []
    for seed in seeds:
        case = VARIANTS[flow](seed, n=n)
        sim = GpuSim(case, update_info=False)
        t0 = time.perf_counter()
        iters = []
        for k in range(n_spin + n_save):
            pset, bodies_new, upd = sim.prepare()
            keep = k >= n_spin
            if keep:
                r = torch.empty_like(sim.P)
                sim.ctx.ppe_residual(pset, sim.rhs, sim.P, r, sim.fP)
                p_prev = sim.P.clone()
            info = sim.solve(pset)
            iters.append(info["iterations"])
            if keep:
                out.append(Sample(r, p_prev, sim.P.clone(), sim.role.clone()))
            sim.finish(pset, bodies_new, info, upd)
        torch.cuda.synchronize()
        m = case.body.motion
        log(f"collect seed {seed}: A={m.amplitude:.3f} f={m.freq:.3f} steps={n_spin + n_save} "
            f"mean iters={np.mean(iters):.0f} ({time.perf_counter() - t0:.1f} s)")
        sim.ctx.close()
    return out


def output_scale(samples, bc):
    """Median over samples of rms(P^{k+1} - P^k) / rms(r) on unknown cells."""
    ratios = []
    for s in samples:
        unk = unknown_mask(s.role, bc)
        dr = torch.linalg.vector_norm(s.resid[unk]).item()
        dp = torch.linalg.vector_norm((s.p_next - s.p_prev)[unk]).item()
        if dr > 0 and dp > 0:
            ratios.append(dp / dr)
    return float(np.median(ratios)) if ratios else 1.0


def lr_at(step, total, lr, warmup=50):
    """Linear warm-up, then cosine decay to lr / 20."""
    if step < warmup:
        return lr * (step + 1) / warmup
    f = (step - warmup) / max(1, total - warmup)
    return lr / 20 + (lr - lr / 20) * 0.5 * (1 + math.cos(math.pi * min(1.0, f)))


def train(model, samples, bc, epochs, lr, seed=0, log=print, log_every=200):
    """Adam over the samples in a seeded random order; returns the loss log."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = epochs * len(samples)
    hist, step = [], 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        run = []
        for i in order:
            s = samples[i]
            want = step % 10 == 0
            loss = model.train_step(s.resid, s.p_prev, s.p_next, s.role, bc, lr_at(step, total, lr), want_loss=want)
            if want:
                run.append(loss)
            if step % log_every == 0:
                log(f"train step {step}/{total} epoch {ep} loss {loss if want else float('nan'):.4g} "
                    f"({time.perf_counter() - t0:.1f} s)")
            step += 1
        hist.append(float(np.mean(run)) if run else float("nan"))
    torch.cuda.synchronize()
    return hist


def eval_loss(model, samples, bc):
    """Mean loss over samples (gradient only, no update)."""
    return float(np.mean([model.train_step(s.resid, s.p_prev, s.p_next, s.role, bc, 0.0) for s in samples]))


def evaluate(model, seeds, n, n_spin, n_eval, modes=("zero", "warm", "learned"), precision=M.PREC_FP64,
             log=print, flow="cylinder"):
    """Held-out trajectories: at every evaluated step each mode solves the
    same PPE from its own guess; the trajectory advances with the warm-start
    solution.  A mode is a guess ('zero', 'warm', 'learned'), optionally with
    '+jacobi' for the Jacobi-preconditioned solve.  Returns per-mode iteration
    counts, initial relative residuals and solve times (ms, guess included)."""
    if "warm" not in modes:
        raise ValueError("evaluation advances with the warm-start solution; include 'warm'")
    res = {m: {"iters": [], "rel0": [], "ms": []} for m in modes}
    for seed in seeds:
        case = VARIANTS[flow](seed, n=n)
        sim = GpuSim(case, precision=precision, update_info=False, model=model)
        r = torch.empty_like(sim.P)
        for k in range(n_spin + n_eval):
            pset, bodies_new, upd = sim.prepare()
            if k < n_spin:
                info = sim.solve(pset)
                sim.finish(pset, bodies_new, info, upd)
                continue
            p_k = sim.P.clone()
            order = [m for m in modes if m != "warm"] + (["warm"] if "warm" in modes else [])
            for mode in order:
                base, _, pre = mode.partition("+")
                precond = {"": M.PRECOND_NONE, "jacobi": M.PRECOND_JACOBI}[pre]
                sim.P.copy_(p_k)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                flag = sim.initial_guess(pset, base)
                info = sim.solve(pset, flag, precond)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                if flag == M.GUESS_ZERO:
                    rel0 = 1.0
                else:
                    # residual of the guess itself: re-form it from P^k (cheap)
                    g = p_k.clone()
                    if base == "learned":
                        sim.ctx.ppe_residual(pset, sim.rhs, g, r, sim.fP)
                        model.infer(r, g, sim.role, case.bc_pressure, g)
                    nr, nb = sim.ctx.ppe_residual(pset, sim.rhs, g, r, sim.fP)
                    rel0 = nr / nb if nb > 0 else 0.0
                res[mode]["iters"].append(info["iterations"])
                res[mode]["rel0"].append(rel0)
                res[mode]["ms"].append(ms)
            sim.finish(pset, bodies_new, info, upd)
        log(f"eval seed {seed}: " + ", ".join(
            f"{m} {np.mean(res[m]['iters'][-n_eval:]):.0f} it" for m in modes))
        sim.ctx.close()
    return res


def summarize(res):
    out = {}
    for m, d in res.items():
        it = np.asarray(d["iters"], dtype=float)
        out[m] = {"mean_iters": float(it.mean()), "median_iters": float(np.median(it)),
                  "mean_rel0": float(np.exp(np.mean(np.log(np.maximum(d["rel0"], 1e-300))))),
                  "mean_ms": float(np.mean(d["ms"])), "solves": int(it.size)}
    if "warm" in out and "learned" in out:
        w = np.asarray(res["warm"]["iters"], float)
        lr = np.asarray(res["learned"]["iters"], float)
        out["learned_vs_warm_iter_ratio"] = float(lr.sum() / w.sum())
        out["learned_fewer_iters_fraction"] = float(np.mean(lr < w))
    if "zero" in out and "learned" in out:
        out["learned_vs_zero_iter_ratio"] = float(np.sum(res["learned"]["iters"]) / np.sum(res["zero"]["iters"]))
    return out


def save_weights(path, model, scale, n, meta=None):
    np.savez(path, theta=model.get_params(), channels=np.asarray(model.channels, np.int64),
             scale=np.float64(scale), n=np.int64(n), meta=json.dumps(meta or {}))


def load_model(ctx, path):
    """Model on ctx from a weights file written by save_weights."""
    z = np.load(path, allow_pickle=False)
    model = M.Model(ctx, tuple(int(c) for c in z["channels"]))
    model.set_params(z["theta"])
    model.set_output_scale(float(z["scale"]))
    return model


def init_theta(channels, seed, dim=2):
    """He-normal weights with a zero head: the untrained guess is the warm start."""
    from .inputs import he_normal_params
    shapes, prev = [], 16
    for c in channels:
        shapes += [(prev, c), (c, c)]
        prev = c
    for l in range(len(channels) - 2, -1, -1):
        shapes += [(channels[l] + channels[l + 1], channels[l]), (channels[l], channels[l])]
    shapes.append((channels[0], 1))
    taps = 3 ** dim
    theta = he_normal_params(shapes, seed, taps=taps)
    theta[-(taps * channels[0] + 1):] = 0.0
    return theta


def _seeds(spec):
    a, _, b = spec.partition("-")
    return list(range(int(a), int(b) + 1)) if b else [int(a)]


def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the learned PPE initial guess")
    ap.add_argument("--flow", choices=sorted(VARIANTS), default="cylinder",
                    help="cylinder: 2D network on C2-shaped flows; sphere: 3D network on C4-shaped flows")
    ap.add_argument("--n", type=int, default=None, help="mesh cells per axis (default 1024 in 2D, 128 in 3D)")
    ap.add_argument("--channels", default="16,32,64,128")
    ap.add_argument("--train-seeds", default="1000-1019")
    ap.add_argument("--test-seeds", default="2000-2004")
    ap.add_argument("--spin", type=int, default=20)
    ap.add_argument("--save", type=int, default=100)
    ap.add_argument("--eval-steps", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="weights file (.npz)")
    ap.add_argument("--weights", default=None, help="skip training: evaluate this weights file")
    ap.add_argument("--json", default=None, help="write the summary here")
    ap.add_argument("--modes", default="zero,warm,learned",
                    help="evaluated starts, comma-separated; '+jacobi' adds the Jacobi preconditioner")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the learned guess runs on the GPU only")
    M.load()
    ch = tuple(int(c) for c in a.channels.split(","))
    if a.n is None:
        a.n = 1024 if a.flow == "cylinder" else 128
    base = BASE_CASES[a.flow](n=a.n)
    bc = base.bc_pressure
    ctx = M.Context.from_case(base)
    summary = {"flow": a.flow, "n": a.n, "channels": ch}
    if a.weights:
        model = load_model(ctx, a.weights)
    else:
        t0 = time.perf_counter()
        data = collect(_seeds(a.train_seeds), a.n, a.spin, a.save, flow=a.flow)
        summary["collect_s"] = time.perf_counter() - t0
        summary["samples"] = len(data)
        hold = data[-max(1, len(data) // 20):]
        train_set = data[:len(data) - len(hold)]
        scale = output_scale(train_set, bc)
        model = M.Model(ctx, ch)
        model.set_params(init_theta(ch, a.seed, dim=base.dim))
        model.set_output_scale(scale)
        summary["output_scale"] = scale
        summary["val_loss_before"] = eval_loss(model, hold, bc)
        t0 = time.perf_counter()
        summary["train_loss"] = train(model, train_set, bc, a.epochs, a.lr, seed=a.seed)
        summary["train_s"] = time.perf_counter() - t0
        summary["val_loss_after"] = eval_loss(model, hold, bc)
        print(f"val loss {summary['val_loss_before']:.4g} -> {summary['val_loss_after']:.4g}", flush=True)
        if a.out:
            save_weights(a.out, model, scale, a.n, {"flow": a.flow, "train_seeds": a.train_seeds,
                                                    "epochs": a.epochs, "lr": a.lr})
        del data, train_set, hold
    res = evaluate(model, _seeds(a.test_seeds), a.n, a.spin, a.eval_steps, modes=tuple(a.modes.split(",")),
                   flow=a.flow)
    summary["eval"] = summarize(res)
    print(json.dumps(summary), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(summary, f, indent=1)
    return summary


if __name__ == "__main__":
    main()
