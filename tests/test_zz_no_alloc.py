"""The allocation-free residual entry point (mcd_ppe_residual_noalloc)
against mcd_ppe_residual through the C ABI: the same r and norms, bit for
bit, on two calls in a row, the second on a smaller mesh (the shared
per-device scratch keeps the first call's contents and must not leak into
the second), and the same error on a non-finite right-hand side."""
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


def _problem(M, case, seed):
    m = O.Mesh.from_case(case)
    ob = oracle_bodies(case, 0.0)
    pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
    consts = O.RelaxConsts.make(case.l0, case.kappa, case.eps_relax, case.band_over_l0)
    up = O.update_dps(m, consts, ob, pos, O.roles(m, ob), 50 if ob else 0)
    ctx = M.Context.from_case(case)
    ctx.build_stencils(2, _dev(up.pos), _dev(up.role, torch.int8), _dev(up.normal), case.bc_pressure,
                       case.pin_first)
    rng = np.random.default_rng(seed)
    rhs = rng.standard_normal(m.Nc)
    p = rng.standard_normal(m.Nc)
    f = np.where(up.role >= 2, rng.standard_normal(m.Nc), 0.0)
    return ctx, _dev(rhs), _dev(p), _dev(f), m.Nc


def _both(ctx, rhs, p, f, n):
    r0 = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    r1 = torch.full((n,), -3.0, dtype=torch.float64, device="cuda")
    n0 = ctx.ppe_residual(2, rhs, p, r0, f)
    n1 = ctx.ppe_residual_noalloc(2, rhs, p, r1, f)
    return np_(r0), np_(r1), n0, n1


def test_noalloc_residual_matches_the_allocating_one(M):
    assert 0 < M.load().mcd_noalloc_scratch_bytes() <= 1 << 16
    big = _problem(M, configs.c2_oscillating_cylinder(n=256), 1)
    small = _problem(M, configs.c4_moving_sphere(n=24), 2)       # smaller mesh, other dimension
    for ctx, rhs, p, f, n in (big, small):
        r0, r1, n0, n1 = _both(ctx, rhs, p, f, n)
        assert bits_equal(r0, r1)
        assert n0 == n1 and n0[0] > 0 and n0[1] > 0
    # the first problem again after the smaller one: nothing left over
    ctx, rhs, p, f, n = big
    r0, r1, n0, n1 = _both(ctx, rhs, p, f, n)
    assert bits_equal(r0, r1) and n0 == n1
    # without Neumann data, and the same error on a non-finite right-hand side
    r = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert ctx.ppe_residual_noalloc(2, rhs, p, r) == ctx.ppe_residual(2, rhs, p, r)
    bad_unknown = rhs * float("nan")             # non-finite at every (so at some unknown) row
    with pytest.raises(M.McdError) as e0:
        ctx.ppe_residual(2, bad_unknown, p, r, f)
    with pytest.raises(M.McdError) as e1:
        ctx.ppe_residual_noalloc(2, bad_unknown, p, r, f)
    assert e0.value.status == e1.value.status == 1
    with pytest.raises(M.McdError):
        ctx.ppe_residual_noalloc(3, rhs, p, r, f)            # unbuilt set
