"""Bandwidth sweep of the Bi-CGSTAB stage kernels on operators larger than
the on-chip caches.

Periodic n x n meshes (jittered DPs, every DP inner, the quadratic MLS
Laplacian of the cos^2 weight, one DP pinned), a seeded right-hand side and
a fixed number of iterations (the tolerance is set out of reach).  Every
stage launch is timed by HIP events on the solve stream (mcd_profile); the
achieved rate is the stage's algorithmic bytes per launch divided by its
average duration:
  S-stage (s = r - alpha v, t = A s): 9 matrix planes + r, v, r_hat read,
          s, t written;
  P-stage (r, x and p updates, v = A p): 9 matrix planes + 10 vector streams.
Everything runs through libmcd's C ABI.

    python -m paper_2404_17542_amd.stage_sweep --sizes 1024,2048,4096,8192 --iters 64
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import configs, inputs
from . import mcd as M

HBM_PEAK_GBS = 8000.0


def stage_bytes(n_unknown, matrix_bytes, vector_bytes):
    s = n_unknown * (9 * matrix_bytes + 5 * vector_bytes)
    p = n_unknown * (9 * matrix_bytes + 10 * vector_bytes)
    return s, p


def run(n, iters, precision="fp64", log=print):
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
    # one untimed solve (graph capture, first-touch), then the timed one
    ctx.solve_ppe(0, rhs, p, tol=1e-30, max_iter=iters, precision=prec, fp64_below=0.0, raise_on_fail=False)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    p.zero_()
    info = ctx.solve_ppe(0, rhs, p, tol=1e-30, max_iter=iters, precision=prec, fp64_below=0.0,
                         raise_on_fail=False)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    n_unk = case.n_cells - 1
    sb, pb = stage_bytes(n_unk, mb, 8)
    s_us = prof["s_ms"] / max(prof["s_n"], 1) * 1e3
    p_us = prof["p_ms"] / max(prof["p_n"], 1) * 1e3
    out = {"n": n, "unknowns": n_unk, "precision": precision, "iterations": info["iterations"],
           "s_launches": prof["s_n"], "s_avg_us": s_us, "s_bytes": sb, "s_GBs": sb / s_us / 1e3,
           "p_launches": prof["p_n"], "p_avg_us": p_us, "p_bytes": pb, "p_GBs": pb / p_us / 1e3,
           "shape": ctx.get_shape()}
    out["s_frac"] = out["s_GBs"] / HBM_PEAK_GBS
    out["p_frac"] = out["p_GBs"] / HBM_PEAK_GBS
    log(f"{n}^2 {precision}: S {s_us:.1f} us {out['s_GBs']:.0f} GB/s ({100 * out['s_frac']:.0f} %), "
        f"P {p_us:.1f} us {out['p_GBs']:.0f} GB/s ({100 * out['p_frac']:.0f} %)")
    ctx.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--sizes", default="1024,2048,4096,8192")
    ap.add_argument("--iters", type=int, default=64)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the sweep runs on the GPU")
    M.load()
    res = [run(int(s), a.iters, a.precision, log=lambda m: print(m, file=sys.stderr, flush=True))
           for s in a.sizes.split(",")]
    print(json.dumps(res), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
