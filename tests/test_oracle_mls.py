"""Pins of the oracle's MLS weights (Sec. 3.2) against facts fixed by the
mathematics: the hand-derived regular-grid closed form, exact reproduction of
quadratics (with and without Neumann data), and an independent weighted
least-squares solve by QR/SVD."""
import json
import os

import numpy as np
import pytest

from oracle import mcd_oracle as O
from paper_2404_17542_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _regular(dim, n=6):
    m = O.Mesh(dim, (n,) * dim, (0.0,) * dim, 1.0, (True,) * dim)
    pos = inputs.cell_centroids(m.n, m.origin, m.l0)
    role = np.full(m.Nc, O.INNER, np.int8)
    return m, pos, role


def test_regular_grid_closed_form():
    g = json.load(open(os.path.join(GOLD, "regular_grid_weights.json")))
    m, pos, role = _regular(2)
    st = O.mls_build(m, pos, role, np.zeros_like(pos), {}, 2.5, 1.0, "cos2")
    lc = O.lap_coefficients(m, st)
    c = 14
    for s, off in enumerate(m.offsets):
        nz = sum(1 for v in off if v)
        want = g["lap_centre"] if nz == 0 else (g["lap_edge"] if nz == 1 else g["lap_diag"])
        assert lc[s, c] == pytest.approx(want, rel=1e-13, abs=1e-15)
        # d/dx = Phi_0 / r_s
        wdx = 0.0 if off[0] == 0 else off[0] * (g["dx_edge"] if nz == 1 else g["dx_diag"])
        if s != m.centre:
            assert st.phi[0, s, c] == pytest.approx(wdx, rel=1e-13, abs=1e-15)
    assert st.phi[0, m.centre, c] == pytest.approx(0.0, abs=1e-15)


def _random_quadratic(rng, dim):
    nb = 1 + dim + dim * (dim + 1) // 2
    cf = rng.standard_normal(nb)

    def f(p):
        out = cf[0] + sum(cf[1 + a] * p[a] for a in range(dim))
        k = 1 + dim
        for a in range(dim):
            for b in range(a, dim):
                out = out + cf[k] * p[a] * p[b]
                k += 1
        return out

    def grad(p):
        g = []
        for a in range(dim):
            v = cf[1 + a] + 0 * p[0]
            k = 1 + dim
            for i in range(dim):
                for j in range(i, dim):
                    if i == a:
                        v = v + cf[k] * p[j]
                    if j == a:
                        v = v + cf[k] * p[i]
                    k += 1
            g.append(v)
        return np.stack(g)

    def lap():
        k = 1 + dim
        s = 0.0
        for i in range(dim):
            for j in range(i, dim):
                if i == j:
                    s += 2 * cf[k]
                k += 1
        return s
    return f, grad, lap


@pytest.mark.parametrize("dim,kind", [(2, "cos2"), (2, "gauss"), (3, "cos2")])
def test_quadratic_reproduction_interior(dim, kind):
    n = 10 if dim == 2 else 6
    l0 = 0.1
    m = O.Mesh(dim, (n,) * dim, (0.0,) * dim, l0, (False,) * dim)
    pos = inputs.jittered_positions(m.n, m.origin, l0, seed=11)
    role = np.full(m.Nc, O.INNER, np.int8)
    ijk = m.ijk(np.arange(m.Nc))
    interior = np.all((ijk > 0) & (ijk < n - 1), axis=0)
    idx = np.nonzero(interior)[0]
    st = O.mls_build(m, pos, role, np.zeros_like(pos), {}, 2.5 * l0, l0, kind, idx=idx)
    rng = np.random.default_rng(3)
    f, grad, lap = _random_quadratic(rng, dim)
    Phi = O.poly_coeffs(m, st, f(pos))
    g = O.grad_from_phi(Phi, l0, dim)
    np.testing.assert_allclose(g, grad(pos[:, idx]), rtol=0, atol=1e-11)
    np.testing.assert_allclose(O.lap_from_phi(Phi, l0, dim), lap(), rtol=0, atol=1e-9)
    # weights sum to zero per derivative op (centre slot)
    assert np.abs(st.phi[:, : m.S].sum(axis=1)).max() < 1e-11


def test_quadratic_reproduction_with_neumann_rows():
    """Boundary DPs of a circle with exact Neumann data n . grad f."""
    dim, n, l0 = 2, 24, 1.0 / 24
    m = O.Mesh(dim, (n, n), (0.0, 0.0), l0, (False, False))
    body = O.BodyState((0.5, 0.5), 0.23, 2)
    role = O.roles(m, [body])
    pos = inputs.jittered_positions(m.n, m.origin, l0, seed=5)
    consts = O.RelaxConsts.make(l0)
    up = O.update_dps(m, consts, [body], pos, role, 200)
    pos, role, nrm = up.pos, up.role, up.normal
    rng = np.random.default_rng(9)
    f, grad, lap = _random_quadratic(rng, dim)
    fneu = np.sum(nrm * grad(pos), axis=0)
    ijk = m.ijk(np.arange(m.Nc))
    interior = np.all((ijk > 0) & (ijk < n - 1), axis=0) & (role != O.VOID)
    idx = np.nonzero(interior)[0]
    st = O.mls_build(m, pos, role, nrm, {2: O.NEUMANN}, 2.5 * l0, l0, "cos2", idx=idx)
    ok = ~st.singular
    assert ok.sum() > 0.9 * len(idx)
    assert (st.kind == 2).any()
    Phi = O.poly_coeffs(m, st, f(pos), fneu)
    g = O.grad_from_phi(Phi, l0, dim)
    np.testing.assert_allclose(g[:, ok], grad(pos[:, idx])[:, ok], rtol=0, atol=1e-9)
    np.testing.assert_allclose(O.lap_from_phi(Phi, l0, dim)[ok], lap(), rtol=0, atol=1e-7)


def test_weights_match_independent_least_squares():
    """The chi_c = 1 fit is a weighted linear least-squares problem; solving it
    with numpy's SVD-based lstsq must give the same Phi as the Cholesky path."""
    dim, n, l0 = 2, 12, 0.5
    m = O.Mesh(dim, (n, n), (0.0, 0.0), l0, (False, False))
    body = O.BodyState((3.0, 3.0), 1.1, 2)
    role = O.roles(m, [body])
    pos = inputs.jittered_positions(m.n, m.origin, l0, seed=21)
    up = O.update_dps(m, O.RelaxConsts.make(l0), [body], pos, role, 100)
    pos, role, nrm = up.pos, up.role, up.normal
    rng = np.random.default_rng(2)
    fld = rng.standard_normal(m.Nc)
    fneu = rng.standard_normal(m.Nc)
    bc = {2: O.NEUMANN}
    idx = np.array([c for c in range(m.Nc) if role[c] != O.VOID
                    and all(0 < v < n - 1 for v in m.ijk(np.array([c]))[:, 0])])
    st = O.mls_build(m, pos, role, nrm, bc, 2.5 * l0, l0, "cos2", idx=idx)
    Phi = O.poly_coeffs(m, st, fld, fneu)
    checked = 0
    for k, c in enumerate(idx):
        if st.singular[k]:
            continue
        i, j = c % n, c // n
        A, y = [], []
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                q = (i + di) + n * (j + dj)
                r = role[q]
                if r == O.VOID:
                    continue
                X, Y = (pos[0, q] - pos[0, c]) / l0, (pos[1, q] - pos[1, c]) / l0
                dist = np.hypot(pos[0, q] - pos[0, c], pos[1, q] - pos[1, c])
                w = np.cos(np.pi * dist / (2 * 2.5 * l0)) ** 2 if dist <= 2.5 * l0 else 0.0
                sw = np.sqrt(w)
                if r == 2:       # Neumann row: (n . grad p) . Phi = r_s f
                    nx, ny = nrm[0, q], nrm[1, q]
                    A.append(sw * np.array([nx, ny, nx * X, nx * Y + ny * X, ny * Y]))
                    y.append(sw * l0 * fneu[q])
                elif q != c:     # value row: p . Phi = phi_j - phi_c
                    A.append(sw * np.array([X, Y, X * X / 2, X * Y, Y * Y / 2]))
                    y.append(sw * (fld[q] - fld[c]))
        sol = np.linalg.lstsq(np.array(A), np.array(y), rcond=None)[0]
        np.testing.assert_allclose(Phi[:, k], sol, rtol=1e-9, atol=1e-9)
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("kind", ["cos2", "gauss"])
def test_quadratic_reproduction_on_the_9x9_support(kind):
    """The widened support (Sec. 4: 9x9 cells, r_e = 3.5 l0) still reproduces
    quadratics exactly: gradient and Laplacian of a random quadratic at
    interior DPs, weights summing to zero."""
    n, l0 = 16, 0.1
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0, (False, False)).with_stencil_half(4)
    assert m.S == 81 and m.offsets[m.centre] == (0, 0) and len(m.spring_offsets) == 9
    pos = inputs.jittered_positions(m.n, m.origin, l0, seed=12)
    role = np.full(m.Nc, O.INNER, np.int8)
    ijk = m.ijk(np.arange(m.Nc))
    idx = np.nonzero(np.all((ijk > 3) & (ijk < n - 4), axis=0))[0]
    st = O.mls_build(m, pos, role, np.zeros_like(pos), {}, 3.5 * l0, l0, kind, idx=idx)
    rng = np.random.default_rng(4)
    f, grad, lap = _random_quadratic(rng, 2)
    Phi = O.poly_coeffs(m, st, f(pos))
    np.testing.assert_allclose(O.grad_from_phi(Phi, l0, 2), grad(pos[:, idx]), rtol=0, atol=1e-10)
    np.testing.assert_allclose(O.lap_from_phi(Phi, l0, 2), lap(), rtol=0, atol=1e-8)
    assert np.abs(st.phi[:, : m.S].sum(axis=1)).max() < 1e-10
    # r_e = 3.5 l0 reaches about 37 of the 81 cells; the rest carry zero weight
    nz = (np.abs(st.phi[2, : m.S]) + np.abs(st.phi[4, : m.S]) > 0).sum(axis=0)
    assert 30 <= nz.min() and nz.max() <= 50


def test_series_weight_functions_match_the_library():
    """The MLS weight's cosine and exponential are series evaluations (same
    bits everywhere); on their ranges they agree with the C library: cos to
    2.5e-16 absolute (about one ulp of 1) on [0, pi/2], exp(-t) to 2e-15
    relative on [0, 4]."""
    import math
    x = np.linspace(0.0, math.pi / 2, 20001)
    got = O.fit_cos(x)
    want = np.array([math.cos(v) for v in x])
    assert np.max(np.abs(got - want)) <= 2.5e-16
    t = np.linspace(0.0, 4.0, 20001)
    got = O.series_exp_neg(t)
    want = np.array([math.exp(-v) for v in t])
    assert np.max(np.abs(got / want - 1.0)) <= 2e-15
    # the weight itself: cos^2 vanishes at r = re, is 1 at r = 0 and 1/2 at re/2
    w = O.weight(np.array([0.0, 1.25, 2.5, 2.6]), 2.5, "cos2")
    assert w[0] == 1.0 and abs(w[1] - 0.5) <= 2.5e-16 and abs(w[2]) <= 1e-31 and w[3] == 0.0
