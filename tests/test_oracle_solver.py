"""Pins of the oracle's PPE solve and time step (Sec. 3.3): dense direct
solves, the manufactured solution's convergence order, the Taylor-Green
decay, and the remap's exactness on quadratics."""
import math

import numpy as np
import pytest

from oracle import mcd_oracle as O
from oracle.sim import OracleSim
from paper_2404_17542_amd import configs, inputs


def _c0(n):
    case = configs.c0_manufactured(n)
    m = O.Mesh.from_case(case)
    pos = O.project_walls(m, inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed))
    role = O.roles(m, [])
    st = O.mls_build(m, pos, role, np.zeros_like(pos), case.bc_pressure, case.re_over_l0 * case.l0,
                     case.l0, case.weight)
    return case, m, pos, role, st


@pytest.mark.parametrize("n", [16, 32])
def test_bicgstab_matches_dense_solve(n):
    case, m, pos, role, st = _c0(n)
    rhs = inputs.manufactured_rhs(pos)
    g = np.where(role == O.INNER, 0.0, inputs.manufactured_pressure(pos))
    p, info, (A, b, uidx) = O.solve_ppe(m, st, role, case.bc_pressure, rhs, g, None, 1e-12)
    dense = np.linalg.solve(A.toarray(), b)
    assert info.converged and info.true_rel_residual <= 1e-12
    np.testing.assert_allclose(p[uidx], dense, rtol=0, atol=1e-10 * np.abs(dense).max())
    # the operator applied through the weights equals the assembled matrix
    Phi = O.poly_coeffs(m, st, p)
    lap = O.lap_from_phi(Phi, st.rs, 2)
    np.testing.assert_allclose(lap[uidx], rhs[uidx], rtol=0, atol=1e-9 * np.abs(rhs).max())


def test_jacobi_on_a_diagonal_system_takes_one_iteration():
    """Right preconditioning with M = diag(A) makes A M^-1 = I on a diagonal
    matrix: one iteration gives x = b / d exactly (to rounding), while the
    plain method needs several (distinct eigenvalues)."""
    import scipy.sparse as sp
    rng = np.random.Generator(np.random.PCG64(11))
    d = rng.uniform(0.5, 50.0, 40)
    A = sp.diags(d).tocsr()
    b = rng.standard_normal(40)
    x, info = O.bicgstab(A, b, np.zeros(40), 1e-12, minv=O.jacobi_inverse_diagonal(A))
    assert info.iterations == 1
    np.testing.assert_allclose(x, b / d, rtol=1e-14)
    _, plain = O.bicgstab(A, b, np.zeros(40), 1e-12)
    assert plain.iterations > 3


def test_jacobi_is_the_column_scaled_plain_solve():
    """Bi-CGSTAB right-preconditioned by D equals plain Bi-CGSTAB on A D^-1
    with x = D^-1 y, iteration for iteration (up to rounding, which Bi-CGSTAB
    amplifies after a few dozen iterations; compared over the first 12), and
    the preconditioned PPE solve reaches the dense solution."""
    case, m, pos, role, st = _c0(32)
    rhs = inputs.manufactured_rhs(pos)
    g = np.where(role == O.INNER, 0.0, inputs.manufactured_pressure(pos))
    p, info, (A, b, uidx) = O.solve_ppe(m, st, role, case.bc_pressure, rhs, g, None, 1e-10, precond="jacobi")
    assert info.converged and info.true_rel_residual <= 1e-10
    dense = np.linalg.solve(A.toarray(), b)
    np.testing.assert_allclose(p[uidx], dense, rtol=0, atol=1e-8 * np.abs(dense).max())
    minv = O.jacobi_inverse_diagonal(A)
    assert np.all(minv < 0)          # the MLS Laplacian's diagonal is negative
    import scipy.sparse as sp
    x12, _ = O.bicgstab(A, b, np.zeros(len(b)), 1e-30, max_iter=12, minv=minv)
    y12, _ = O.bicgstab((A @ sp.diags(minv)).tocsr(), b, np.zeros(len(b)), 1e-30, max_iter=12)
    np.testing.assert_allclose(minv * y12, x12, rtol=0, atol=1e-12 * np.abs(x12).max())
    # a left-preconditioned or unpreconditioned loop takes other iterates
    xp, _ = O.bicgstab(A, b, np.zeros(len(b)), 1e-30, max_iter=12)
    assert np.abs(xp - x12).max() > 1e-6 * np.abs(x12).max()


def test_manufactured_convergence_order():
    """p = sin 2 pi x sin 2 pi y: the RMS error of the jittered quadratic MLS
    Poisson solve falls at order >= 1.5 between the two finest meshes."""
    errs = []
    for n in (16, 32, 64):
        case, m, pos, role, st = _c0(n)
        rhs = inputs.manufactured_rhs(pos)
        g = np.where(role == O.INNER, 0.0, inputs.manufactured_pressure(pos))
        p, info, _ = O.solve_ppe(m, st, role, case.bc_pressure, rhs, g, None, 1e-10)
        assert info.converged
        err = p - inputs.manufactured_pressure(pos)
        errs.append(math.sqrt(np.mean(err[role == O.INNER] ** 2)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] >= 1.5, orders


def test_mixed_refinement_reaches_fp64_tolerance():
    case, m, pos, role, st = _c0(32)
    rhs = inputs.manufactured_rhs(pos)
    g = np.where(role == O.INNER, 0.0, inputs.manufactured_pressure(pos))
    p64, i64, _ = O.solve_ppe(m, st, role, case.bc_pressure, rhs, g, None, 1e-8)
    pm, im = O.solve_ppe_mixed(m, st, role, case.bc_pressure, rhs, g, None, 1e-8)
    assert im.converged and im.true_rel_residual <= 1e-8 and im.restarts >= 2
    assert np.linalg.norm(pm - p64) / np.linalg.norm(p64) < 1e-7
    # without refinement, scipy's Bi-CGSTAB entirely in FP32 (checked on the
    # FP64 operator) stalls far above the tolerance
    from scipy.sparse.linalg import bicgstab
    A, beff, uidx = O.ppe_system(m, st, role, case.bc_pressure, rhs, g, None)
    nb = np.linalg.norm(beff)
    x32, _ = bicgstab(A.astype(np.float32), (beff / nb).astype(np.float32), rtol=1e-12, maxiter=2000)
    assert x32.dtype == np.float32
    rel32 = np.linalg.norm(beff - A @ (x32.astype(np.float64) * nb)) / nb
    assert rel32 > 1e-7, rel32


def test_fp32_matrix_with_residual_replacement():
    """FP32-stored matrix in the products, FP64 vectors: the replacement
    brings the FP64 residual to 1e-8, about as fast as FP64; without it the
    recursion converges to the solution of the rounded matrix, whose FP64
    residual stalls above the tolerance."""
    case, m, pos, role, st = _c0(48)
    rhs = inputs.manufactured_rhs(pos)
    g = np.where(role == O.INNER, 0.0, inputs.manufactured_pressure(pos))
    p64, i64, _ = O.solve_ppe(m, st, role, case.bc_pressure, rhs, g, None, 1e-8)
    pm, im = O.solve_ppe_fp32_matrix(m, st, role, case.bc_pressure, rhs, g, None, 1e-8)
    assert im.converged and im.true_rel_residual <= 1e-8 and im.refinements >= 2
    assert np.linalg.norm(pm - p64) / np.linalg.norm(p64) < 1e-7
    assert im.iterations <= 1.5 * i64.iterations + 10, (im.iterations, i64.iterations)
    # the FP32 operator in difference form against a plain per-entry rounding:
    # on a smooth field its product error is orders of magnitude smaller,
    # because the rounded stencil rows still sum to zero
    A, beff, uidx = O.ppe_system(m, st, role, case.bc_pressure, rhs, g, None)
    xs = p64[uidx]
    exact = A @ xs
    e_diff = np.linalg.norm(O.fp32_operator(A, np.float64)(xs) - exact)
    e_plain = np.linalg.norm(A.astype(np.float32).astype(np.float64) @ xs - exact)
    assert e_diff < 0.1 * e_plain, (e_diff, e_plain)
    # and on a constant field (A x is the row sum: zero on inner rows, what
    # remains is the FP32 rounding of the rows next to Dirichlet DPs)
    one = np.ones(len(uidx))
    e_diff = np.linalg.norm(O.fp32_operator(A, np.float64)(one) - A @ one)
    e_plain = np.linalg.norm(A.astype(np.float32).astype(np.float64) @ one - A @ one)
    assert e_diff < 0.1 * e_plain, (e_diff, e_plain)


def test_remap_identity_and_quadratic_exactness():
    n, l0 = 12, 0.1
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0, (True, True))
    pos = inputs.jittered_positions(m.n, m.origin, l0, seed=3)
    role = np.full(m.Nc, O.INNER, np.int8)
    st = O.mls_build(m, pos, role, np.zeros_like(pos), {}, 2.5 * l0, l0)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((2, m.Nc))
    out, _ = O.remap_velocity(m, st, u, pos, pos, role, role, [], [])
    assert np.array_equal(out, u)
    # a quadratic field (away from the periodic seam) is shifted exactly
    cf = rng.standard_normal(6)

    def q(p):
        return cf[0] + cf[1] * p[0] + cf[2] * p[1] + cf[3] * p[0] ** 2 + cf[4] * p[0] * p[1] + cf[5] * p[1] ** 2
    mnp = O.Mesh(2, (n, n), (0.0, 0.0), l0)
    stq = O.mls_build(mnp, pos, role, np.zeros_like(pos), {}, 2.5 * l0, l0)
    shift = 0.3 * l0 * rng.uniform(-1, 1, (2, m.Nc))
    ijk = m.ijk(np.arange(m.Nc))
    ins = np.all((ijk > 0) & (ijk < n - 1), axis=0)
    uq = np.stack([q(pos), q(pos)])
    out, _ = O.remap_velocity(mnp, stq, uq, pos, pos + shift, role, role, [], [])
    np.testing.assert_allclose(out[0, ins], q(pos + shift)[ins], rtol=0, atol=1e-12)


def _tgv_decay_ratio(n, t_end):
    case = configs.c1_taylor_green(n, steps=1)
    steps = int(round(t_end / case.dt))
    sim = OracleSim(case)
    ke0 = sim.kinetic_energy()
    for _ in range(steps):
        rec = sim.step()
        assert rec["converged"]
    ana = math.exp(-4 * case.nu * steps * case.dt)
    return (1 - sim.kinetic_energy() / ke0) / (1 - ana)


def test_taylor_green_decay_converges_first_order():
    """KE(t)/KE(0) of the Taylor-Green vortex decays as exp(-4 nu t); the
    scheme's excess dissipation (first-order MOC, Sec. 3.3) must shrink about
    linearly with the mesh spacing at fixed time."""
    t_end = 20 * configs.c1_taylor_green(64).dt
    r64 = _tgv_decay_ratio(64, t_end)
    r128 = _tgv_decay_ratio(128, t_end)
    assert 1.0 < r128 < r64 < 1.5
    assert (r128 - 1.0) < 0.65 * (r64 - 1.0)


def test_two_body_steps():
    """Two cylinders (ids 2 and 3) on 64^2: each step converges, every body
    DP carries its own body's velocity, and the velocity field stays
    bounded by a few times the peak body speed."""
    case = configs.c2_two_cylinders(n=64, steps=3)
    sim = OracleSim(case)
    for _ in range(3):
        rec = sim.step()
        assert rec["converged"] and rec["rel_res"] <= 1e-8
    for b in sim.bodies:
        sel = sim.role == b.body_id
        assert sel.sum() > 5
        for a in range(2):
            assert np.all(sim.u[a, sel] == b.velocity[a])
    assert np.isfinite(sim.u).all() and np.abs(sim.u).max() < 5 * 2 * math.pi * 0.15


def test_rotating_body_velocity_and_neumann_closed_forms():
    """Rigid rotation of a circle (Eqs. velocity_moving_boundary,
    dvdt_moving_boundary): the rotational part of V at a body point is
    tangential with |V - V_trans| = |omega| |r|; at constant omega the
    acceleration is centripetal, so -dV/dt . n = omega^2 |r| + (-dV_trans/dt . n)
    for n = r/|r|, and an angular acceleration adds nothing along n."""
    case = configs.c2_oscillating_cylinder(n=64)
    m = O.Mesh.from_case(case)
    rng = np.random.default_rng(3)
    ang = rng.uniform(0, 2 * math.pi, m.Nc)
    rad = 0.5 * (1 + 0.1 * rng.uniform(-1, 1, m.Nc))
    c = (0.3, -0.2)
    pos = np.stack([c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang)])
    normal = np.stack([np.cos(ang), np.sin(ang)])
    role = np.full(m.Nc, 2, dtype=np.int8)
    w, vt, dv = 1.7, (0.4, -0.9), (2.0, 0.5)
    b = O.BodyState(c, 0.5, 2, vt, (0.0, 0.0, w))
    V = O.body_point_velocity(b, pos)
    rel = [V[0] - vt[0], V[1] - vt[1]]
    r = pos - np.array(c)[:, None]
    np.testing.assert_allclose(rel[0] * r[0] + rel[1] * r[1], 0.0, atol=1e-14)
    np.testing.assert_allclose(np.hypot(*rel), abs(w) * np.hypot(*r), rtol=1e-14)
    f = O.neumann_pressure_data(m, role, normal, [b], {2: (0.0, 0.0)}, {2: (0.0, 0.0, 0.0)}, pos=pos)
    np.testing.assert_allclose(f, w * w * rad, rtol=1e-13)
    f2 = O.neumann_pressure_data(m, role, normal, [b], {2: dv}, {2: (0.0, 0.0, -3.1)}, pos=pos)
    np.testing.assert_allclose(f2, w * w * rad - (dv[0] * normal[0] + dv[1] * normal[1]), rtol=1e-12, atol=1e-13)
    # a rotating body without positions is an error, a still one is not
    with pytest.raises(ValueError):
        O.neumann_pressure_data(m, role, normal, [b], {2: dv}, None)
    O.neumann_pressure_data(m, role, normal, [O.BodyState(c, 0.5, 2, vt)], {2: dv}, None)


def test_rotating_cylinder_steps():
    """Spinning cylinder on 64^2: steps converge and every body DP carries
    V_trans + omega x r of its own position."""
    case = configs.c2_rotating_cylinder(n=64, steps=3)
    sim = OracleSim(case)
    for _ in range(3):
        rec = sim.step()
        assert rec["converged"] and rec["rel_res"] <= 1e-8
    b = sim.bodies[0]
    assert b.omega[2] != 0.0
    sel = sim.role == b.body_id
    r = sim.pos[:, sel] - np.array(b.centre)[:, None]
    np.testing.assert_allclose(sim.u[0, sel], b.velocity[0] - b.omega[2] * r[1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(sim.u[1, sel], b.velocity[1] + b.omega[2] * r[0], rtol=0, atol=1e-15)
