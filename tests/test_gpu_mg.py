"""The multigrid preconditioner on the GPU (FP32 V-cycle, Galerkin levels
built per solve) against the oracle's definition, and the FP64 Bi-CGSTAB
that it preconditions.  Bars: one V-cycle applied to the same vector equals
the oracle's (FP64) V-cycle to 1e-4 relative (the GPU cycle runs in FP32);
preconditioned solves reach 1e-8 on the GPU's operator and on the oracle's
assembled operator in a handful of iterations."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mcd_oracle as O
from paper_2404_17542_amd import configs, inputs
from gpu_helpers import np_, oracle_bodies

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


CASES = {
    "cylinder128": lambda: configs.c2_oscillating_cylinder(n=128),
    "sphere24": lambda: configs.c4_moving_sphere(n=24),
    "sphere20": lambda: configs.c4_moving_sphere(n=20),          # odd coarse sizes (10 -> 5 -> 3)
    "taylor_green64": lambda: configs.c1_taylor_green(n=64),     # periodic, pinned DP
    "manufactured32": lambda: configs.c0_manufactured(32),       # Dirichlet walls, Gaussian weight
}


def _arranged(case):
    m = O.Mesh.from_case(case)
    consts = O.RelaxConsts.make(case.l0, case.kappa, case.eps_relax, case.band_over_l0)
    pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
    ob = oracle_bodies(case, 0.0)
    up = O.update_dps(m, consts, ob, pos, O.roles(m, ob), 100 if ob else 0)
    if not ob:
        up.pos = O.project_walls(m, pos)
    return m, up.pos, up.role, up.normal


def _problem(M, name):
    case = CASES[name]()
    m, pos, role, nrm = _arranged(case)
    ctx = M.Context.from_case(case)
    ctx.build_stencils(2, _dev(pos), _dev(role, torch.int8), _dev(nrm), case.bc_pressure, case.pin_first)
    st = O.mls_build(m, pos, role, nrm, case.bc_pressure, case.re_over_l0 * case.l0, case.rs_over_l0 * case.l0,
                     case.weight)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(m.Nc)
    f = np.where(role >= 2, rng.standard_normal(m.Nc), 0.0)
    g = np.zeros(m.Nc)
    A, b, uidx = O.ppe_system(m, st, role, case.bc_pressure, rhs, g, f, case.pin_first)
    return case, m, ctx, A, b, uidx, rhs, f, g


@pytest.mark.parametrize("name", sorted(CASES))
def test_vcycle_matches_the_oracle(M, name):
    case, m, ctx, A, b, uidx, rhs, f, g = _problem(M, name)
    levels = O.mg_levels(m, A, uidx)
    rng = np.random.default_rng(9)
    v = np.zeros(m.Nc)
    v[uidx] = rng.standard_normal(len(uidx))
    want = O.mg_vcycle(levels, v)
    out = torch.zeros(m.Nc, dtype=torch.float64, device="cuda")
    nlev = ctx.mg_apply(2, _dev(v), out)
    got = np_(out)
    assert nlev == len(levels)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"{name}: {nlev} levels, V-cycle relative difference {rel:.2e}")
    assert rel <= 1e-4, rel
    unk = np.zeros(m.Nc, dtype=bool)
    unk[uidx] = True
    assert np.all(got[~unk] == 0.0)


@pytest.mark.parametrize("name", sorted(CASES))
def test_preconditioned_solve_reaches_the_tolerance(M, name):
    case, m, ctx, A, b, uidx, rhs, f, g = _problem(M, name)
    p = _dev(g)
    info = ctx.solve_ppe(2, _dev(rhs), p, _dev(f), precond=M.PRECOND_MG)
    plain = ctx.solve_ppe(2, _dev(rhs), _dev(g), _dev(f))
    res = np.linalg.norm(b - A @ np_(p)[uidx]) / np.linalg.norm(b)
    print(f"{name}: MG {info['iterations']} iterations, plain {plain['iterations']}, oracle-operator residual "
          f"{res:.2e}")
    assert info["converged"] and info["true_rel_residual"] <= 1e-8
    assert res <= 1e-8
    assert info["iterations"] <= 12 and info["iterations"] < plain["iterations"]


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_products_reach_the_tolerance(M, name):
    """The mixed form: products with the FP32 difference-form matrix, FP64
    vectors, the FP32 V-cycle; the tolerance holds on the oracle's FP64
    operator."""
    case, m, ctx, A, b, uidx, rhs, f, g = _problem(M, name)
    p = _dev(g)
    info = ctx.solve_ppe(2, _dev(rhs), p, _dev(f), precision=M.PREC_FP32_MATRIX, precond=M.PRECOND_MG)
    res = np.linalg.norm(b - A @ np_(p)[uidx]) / np.linalg.norm(b)
    print(f"{name}: MG with FP32 products {info['iterations']} iterations, {info['restarts']} restarts, "
          f"oracle-operator residual {res:.2e}")
    assert info["converged"] and info["true_rel_residual"] <= 1e-8
    assert res <= 1e-8
    assert info["iterations"] <= 16


@pytest.mark.parametrize("precision", ["fp64", "fp32_matrix"])
def test_non_finite_rhs_is_reported_and_p_kept(M, precision):
    """A non-finite right-hand side: the multigrid solve reads the b_eff
    check back with its first residual, reports MCD_ERR_ARG and leaves p as
    it was; a later solve on the same context works."""
    case, m, ctx, A, b, uidx, rhs, f, g = _problem(M, "cylinder128")
    prec = {"fp64": M.PREC_FP64, "fp32_matrix": M.PREC_FP32_MATRIX}[precision]
    bad = rhs.copy()
    bad[uidx[len(uidx) // 2]] = np.inf
    p0 = np.random.default_rng(9).standard_normal(m.Nc)
    p = _dev(p0)
    with pytest.raises(M.McdError) as e:
        ctx.solve_ppe(2, _dev(bad), p, _dev(f), precision=prec, precond=M.PRECOND_MG)
    assert e.value.status == 1
    assert np.array_equal(np_(p).view(np.int64), p0.view(np.int64))
    info = ctx.solve_ppe(2, _dev(rhs), p, _dev(f), precision=prec, precond=M.PRECOND_MG)
    assert info["converged"] and info["true_rel_residual"] <= 1e-8


def test_unusable_mesh_and_precision_are_refused(M):
    case, m, ctx, A, b, uidx, rhs, f, g = _problem(M, "cylinder128")
    with pytest.raises(M.McdError) as e:
        ctx.solve_ppe(2, _dev(rhs), _dev(g), _dev(f), precision=M.PREC_FP32_REFINE, precond=M.PRECOND_MG)
    assert e.value.status == 1
    odd = configs.c1_taylor_green(n=62)          # periodic 62 -> 31 (odd): no coarse level
    c2 = M.Context.from_case(odd)
    mo, pos, role, nrm = _arranged(odd)
    c2.build_stencils(0, _dev(pos), _dev(role, torch.int8), _dev(nrm), {}, True)
    with pytest.raises(M.McdError) as e:
        c2.solve_ppe(0, _dev(np.ones(mo.Nc)), _dev(np.zeros(mo.Nc)), precond=M.PRECOND_MG)
    assert e.value.status == 1
