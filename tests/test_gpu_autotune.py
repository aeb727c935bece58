"""Autotuner of the Krylov stage kernels' launch shape (block count, 3D brick
depth), through the C ABI: every candidate shape solves the same PPE to the
tolerance (on the oracle's assembled operator in 3D, where bricks are ragged),
a fixed shape is run-to-run bit-identical, the tuner applies the candidate it
reports, and shapes outside the limits are rejected.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mcd_oracle as O
from paper_2404_17542_amd import configs, inputs
from gpu_helpers import bits_equal, np_, oracle_bodies

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_17542_amd import mcd
    mcd.load()
    return mcd


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_autotune_2d_every_shape_solves(M):
    """Taylor-Green 512^2 (512 tiles of 64 x 8): four block counts."""
    from paper_2404_17542_amd.sim import GpuSim
    case = configs.c1_taylor_green(n=512, steps=1)
    sim = GpuSim(case, update_info=False)
    pset, bodies_new, upd = sim.prepare()
    ctx = sim.ctx
    res = ctx.autotune(pset, iters=16)
    cands = res["candidates"]
    print(res)
    assert [c["grid"] for c in cands] == [128, 256, 384, 512]
    assert all(c["depth"] == 1 and c["us_per_iter"] > 0 for c in cands)
    k = res["chosen"]
    assert 0 <= k < len(cands)
    best = min(c["us_per_iter"] for c in cands)
    assert cands[k]["us_per_iter"] <= 1.02 * best
    assert res["shape"] == {"grid": cands[k]["grid"], "depth": 1, "blocks": cands[k]["grid"]}
    p0 = sim.P.clone()
    r = torch.empty_like(sim.P)
    sols = {}
    for c in cands:
        ctx.set_shape(c["grid"])
        assert ctx.get_shape()["blocks"] == c["grid"]
        for rep in range(2 if c["grid"] == 384 else 1):
            sim.P.copy_(p0)
            info = sim.solve(pset)
            assert info["converged"] and info["true_rel_residual"] <= 1e-8, (c, info)
            nr, nb = ctx.ppe_residual(pset, sim.rhs, sim.P, r, sim.fP)
            assert nr / nb <= 1e-8 * (1 + 1e-6), c
            if rep == 1:      # the same shape again: bit-identical
                assert bits_equal(np_(sim.P), sols[c["grid"]])
            sols[c["grid"]] = np_(sim.P).copy()
    ref = sols[512]
    for g, q in sols.items():
        assert np.linalg.norm(q - ref) / np.linalg.norm(ref) < 1e-5, g


def test_autotune_3d_brick_depths_on_the_oracle_operator(M):
    """Moving sphere 24^3: brick depths 4, 8, 16 (the last ragged: 16 + 8
    planes); each solves to 1e-8 on the oracle's assembled operator."""
    case = configs.c4_moving_sphere(n=24)
    m = O.Mesh.from_case(case)
    consts = O.RelaxConsts.make(case.l0, case.kappa, case.eps_relax, case.band_over_l0)
    ob = oracle_bodies(case, 0.0)
    pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
    up = O.update_dps(m, consts, ob, pos, O.roles(m, ob), 100)
    pos, role, nrm = up.pos, up.role, up.normal
    rng = np.random.default_rng(7)
    rhs = rng.standard_normal(m.Nc)
    f = np.where(role == 2, rng.standard_normal(m.Nc), 0.0)
    g = np.zeros(m.Nc)
    ctx = M.Context.from_case(case)
    ctx.build_stencils(2, _dev(pos), _dev(role, torch.int8), _dev(nrm), case.bc_pressure)
    st = O.mls_build(m, pos, role, nrm, case.bc_pressure, case.re_over_l0 * case.l0, case.l0, case.weight)
    A, b, uidx = O.ppe_system(m, st, role, case.bc_pressure, rhs, g, f)
    res = ctx.autotune(2, iters=8)
    depths = sorted({c["depth"] for c in res["candidates"]})
    assert depths == [4, 8, 16], res
    assert res["shape"]["depth"] == res["candidates"][res["chosen"]]["depth"]
    sols = []
    for depth in (4, 8, 16):
        for grid in (512, 2):      # every brick its own block; several bricks per block
            ctx.set_shape(grid, depth)
            p = _dev(g)
            info = ctx.solve_ppe(2, _dev(rhs), p, _dev(f))
            assert info["converged"] and info["true_rel_residual"] <= 1e-8, (depth, grid, info)
            pg = np_(p)
            assert np.linalg.norm(b - A @ pg[uidx]) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6), (depth, grid)
            sols.append(pg[uidx])
    for q in sols[1:]:
        assert np.linalg.norm(q - sols[0]) / np.linalg.norm(sols[0]) < 1e-5


def test_shape_limits(M):
    case3 = configs.c4_moving_sphere(n=16)
    ctx3 = M.Context.from_case(case3)
    for grid, depth in ((0, 8), (513, 8), (512, 0), (512, 17)):
        with pytest.raises(M.McdError) as e:
            ctx3.set_shape(grid, depth)
        assert e.value.status == 1
    ctx3.set_shape(100, 16)
    assert ctx3.get_shape() == {"grid": 100, "depth": 16, "blocks": 1 * 2 * 1}
    case2 = configs.c1_taylor_green(n=64, steps=1)
    ctx2 = M.Context.from_case(case2)
    with pytest.raises(M.McdError):
        ctx2.set_shape(512, 2)          # 2D has no brick depth
    with pytest.raises(M.McdError):
        ctx2.autotune(0)                # set not built
    ctx2.set_shape(512)
    assert ctx2.get_shape() == {"grid": 512, "depth": 1, "blocks": 1 * 8}
