"""Pins of the oracle's multigrid preconditioner (the preconditioner of the
mixed-precision form; not from the paper): the transfer operators'
defining properties, the Galerkin coarse operators' row sums, the V-cycle's
error contraction, the exact coarsest solve, and mesh-independent
iteration counts of the preconditioned Bi-CGSTAB to 1e-8 (the solution is
the plain method's)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mcd_oracle as O
from oracle.sim import OracleSim
from paper_2404_17542_amd import configs


def _ppe(case):
    o = OracleSim(case)
    o.step()
    A, b, uidx = o.last_ppe
    return o.mesh, A, b, uidx


def _precond(mesh, levels, uidx):
    def minv(q):
        full = np.zeros(mesh.Nc)
        full[uidx] = q
        return O.mg_vcycle(levels, full)[uidx]
    return minv


def test_transfers_partition_unity_and_mean():
    """P interpolates constants exactly at unknown fine cells (rows sum to
    1), has zero rows elsewhere, reaches only unknown coarse cells, and R
    averages the 2^dim children of each coarse cell."""
    case = configs.c2_oscillating_cylinder(n=64, steps=1)
    mesh, A, b, uidx = _ppe(case)
    levels = O.mg_levels(mesh, A, uidx)
    assert len(levels) >= 3
    for fine, coarse in zip(levels[:-1], levels[1:]):
        rs = np.asarray(fine.P.sum(axis=1)).ravel()
        assert np.allclose(rs[fine.unknown], 1.0, atol=1e-14)
        assert np.all(rs[~fine.unknown] == 0.0)
        cols = fine.P.tocoo().col
        assert np.all(coarse.unknown[cols])
        assert np.all(fine.P.data > 0)
        rr = np.asarray(fine.R.sum(axis=1)).ravel()
        assert np.allclose(rr, 1.0)            # even sizes: every coarse cell has 2^dim children
        assert coarse.unknown.sum() <= fine.unknown.sum()


def test_galerkin_keeps_zero_row_sums_on_a_periodic_laplacian():
    """With every cell unknown on a periodic mesh, the MLS Laplacian kills
    constants (A 1 = 0), so every Galerkin level does: A_c 1 = R A P 1 =
    R A 1 = 0, and the coarse stencils stay within the 3^dim block."""
    case = configs.c1_taylor_green(n=64, steps=1)
    m = O.Mesh.from_case(case)
    from paper_2404_17542_amd import inputs
    pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
    role = np.full(m.Nc, O.INNER, np.int8)
    st = O.mls_build(m, pos, role, np.zeros_like(pos), {}, case.re_over_l0 * case.l0, case.l0)
    A, _, uidx = O.ppe_system(m, st, role, {}, np.zeros(m.Nc), np.zeros(m.Nc), None)
    levels = O.mg_levels(m, A, uidx)
    for lev in levels:
        one = np.ones(lev.A.shape[0])
        scale = abs(lev.A).max()
        assert np.abs(lev.A @ one).max() <= 1e-12 * scale * 9
        assert lev.A.getnnz(axis=1).max() <= 9


def test_vcycle_contracts_the_error():
    """The V-cycle is a convergent iteration on the Dirichlet Poisson matrix
    (manufactured case): ||(I - M^-1 A) e|| < 0.5 ||e|| for random e."""
    case = configs.c0_manufactured(32)
    m = O.Mesh.from_case(case)
    from paper_2404_17542_amd import inputs
    pos = O.project_walls(m, inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed))
    role = O.roles(m, [])
    st = O.mls_build(m, pos, role, np.zeros_like(pos), case.bc_pressure, case.re_over_l0 * case.l0, case.l0,
                     case.weight)
    A, _, uidx = O.ppe_system(m, st, role, case.bc_pressure, np.zeros(m.Nc), np.zeros(m.Nc), None)
    levels = O.mg_levels(m, A, uidx)
    minv = _precond(m, levels, uidx)
    rng = np.random.default_rng(3)
    for _ in range(4):
        e = rng.standard_normal(len(uidx))
        assert np.linalg.norm(e - minv(A @ e)) < 0.5 * np.linalg.norm(e)


def test_coarsest_level_is_an_exact_solve():
    """A mesh of at most 64 cells is its own coarsest level: the V-cycle is
    A^-1 (to rounding)."""
    case = configs.c0_manufactured(8)
    m = O.Mesh.from_case(case)
    from paper_2404_17542_amd import inputs
    pos = O.project_walls(m, inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed))
    role = O.roles(m, [])
    st = O.mls_build(m, pos, role, np.zeros_like(pos), case.bc_pressure, case.re_over_l0 * case.l0, case.l0,
                     case.weight)
    A, _, uidx = O.ppe_system(m, st, role, case.bc_pressure, np.zeros(m.Nc), np.zeros(m.Nc), None)
    levels = O.mg_levels(m, A, uidx)
    assert len(levels) == 1
    b = np.random.default_rng(1).standard_normal(len(uidx))
    x = _precond(m, levels, uidx)(b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("which", ["cylinder", "taylor_green", "sphere"])
def test_preconditioned_iterations_do_not_grow_with_the_mesh(which):
    """MG-preconditioned Bi-CGSTAB reaches 1e-8 in a handful of iterations,
    about the same on a mesh twice as fine, while the plain method's count
    grows; both reach the same solution."""
    make = {"cylinder": lambda n: configs.c2_oscillating_cylinder(n=n, steps=1),
            "taylor_green": lambda n: configs.c1_taylor_green(n=n, steps=1),
            "sphere": lambda n: configs.c4_moving_sphere(n=n, steps=1)}[which]
    sizes = (16, 32) if which == "sphere" else (64, 128)
    counts, plain = [], []
    for n in sizes:
        mesh, A, b, uidx = _ppe(make(n))
        levels = O.mg_levels(mesh, A, uidx)
        x, info = O.bicgstab(A, b, np.zeros(len(uidx)), 1e-8, minv=_precond(mesh, levels, uidx))
        x0, info0 = O.bicgstab(A, b, np.zeros(len(uidx)), 1e-8)
        assert info.converged and info0.converged
        assert np.linalg.norm(x - x0) <= 1e-5 * np.linalg.norm(x0)
        counts.append(info.iterations)
        plain.append(info0.iterations)
    assert max(counts) <= 10, counts
    assert counts[1] <= counts[0] + 2, counts
    assert plain[1] > 1.5 * plain[0] and plain[1] > 3 * counts[1], (plain, counts)
