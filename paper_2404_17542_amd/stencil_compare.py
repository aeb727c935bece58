"""The 3x3 against the 9x9 MLS support on the pressure solve (Sec. 4, flow
past stationary cylinders, and its table of PPE iterations and execution
time), on synthetic flows: the DPs of a case after its initial
arrangement, one seeded right-hand side, Bi-CGSTAB from zero to 1e-8.

Both supports run through the same code (mcd_ppe_wide: weight build and
assembly, then a Bi-CGSTAB with host-formed scalars), so their times compare
the supports, not two solvers; the production 3x3 solve (mcd_solve_ppe,
fused stage kernels) on the same problem is reported beside them.

    python -m paper_2404_17542_amd.stencil_compare --cases cylinder:1024,taylor_green:512
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import configs, inputs
from . import mcd as M

SETS = {"cylinder": configs.c2_oscillating_cylinder, "taylor_green": configs.c1_taylor_green,
        "flapping": configs.c6_flapping_ellipse}


def run(which, n, log=print):
    from .sim import GpuSim
    case = SETS[which](n=n)
    sim = GpuSim(case, update_info=False)
    ctx = sim.ctx
    f64 = dict(dtype=torch.float64, device="cuda")
    rng = np.random.Generator(np.random.PCG64(n))
    rhs = rng.standard_normal(case.n_cells)
    if case.pin_first:
        rhs -= rhs.mean()
    rhs_d = torch.tensor(rhs, **f64)
    zero = torch.zeros(case.n_cells, **f64)
    out = {"case": which, "n": n}
    for half, re in ((1, case.re_over_l0), (4, 3.5)):
        p = zero.clone()
        ctx.ppe_wide(half, re, sim.pos, sim.role, sim.normal, case.bc_pressure, rhs_d, p, zero,
                     pin_first=case.pin_first)            # first call allocates; time the second
        p.zero_()
        info = ctx.ppe_wide(half, re, sim.pos, sim.role, sim.normal, case.bc_pressure, rhs_d, p, zero,
                            pin_first=case.pin_first)
        out[f"{2 * half + 1}x{2 * half + 1}"] = info
        log(f"{which} {n}^2 {2 * half + 1}x{2 * half + 1} (r_e {re} l0): {info['iterations']} iterations, "
            f"build {info['build_ms']:.2f} ms, solve {info['solve_ms']:.1f} ms")
    # the production 3x3 solve on the same operator and right-hand side
    pset = sim.tuning_set()
    p = zero.clone()
    ctx.solve_ppe(pset, rhs_d, p, zero, tol=case.tol, guess=M.GUESS_ZERO)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    p.zero_()
    torch.cuda.synchronize()
    ev[0].record()
    info = ctx.solve_ppe(pset, rhs_d, p, zero, tol=case.tol, guess=M.GUESS_ZERO)
    ev[1].record()
    torch.cuda.synchronize()
    out["3x3 production"] = {"iterations": info["iterations"], "solve_ms": ev[0].elapsed_time(ev[1]),
                             "true_rel_residual": info["true_rel_residual"]}
    log(f"{which} {n}^2 3x3 production solve: {info['iterations']} iterations, {out['3x3 production']['solve_ms']:.1f} ms")
    w3, w9 = out["3x3"], out["9x9"]
    out["ratio_iterations_9_over_3"] = w9["iterations"] / max(w3["iterations"], 1)
    out["ratio_time_9_over_3"] = (w9["build_ms"] + w9["solve_ms"]) / (w3["build_ms"] + w3["solve_ms"])
    ctx.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--cases", default="taylor_green:512,cylinder:1024")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the comparison runs on the GPU")
    M.load()
    res = []
    for item in a.cases.split(","):
        which, n = item.split(":")
        res.append(run(which, int(n), log=lambda m: print(m, file=sys.stderr, flush=True)))
    print(json.dumps(res), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
