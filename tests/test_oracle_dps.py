"""Pins of the oracle's masking and DP arrangement (Sec. 2.2-2.4)."""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import mcd_oracle as O
from paper_2404_17542_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _brute_roles(n, origin, l0, centre, radius, walls):
    """Pure-Python vertex counting with psi = hypot(v - c) - R >= 0."""
    dim = len(n)
    out = []
    for c in range(int(np.prod(n))):
        ijk, r = [], c
        for a in range(dim):
            ijk.append(r % n[a])
            r //= n[a]
        cnt = 0
        for v in range(2 ** dim):
            vx = [origin[a] + (ijk[a] + ((v >> a) & 1)) * l0 for a in range(dim)]
            psi = math.sqrt(sum((vx[a] - centre[a]) ** 2 for a in range(dim))) - radius
            cnt += psi >= 0
        full = 2 ** dim
        role = -1 if cnt == full else (2 if cnt >= full // 2 else 0)
        if walls and any(ijk[a] in (0, n[a] - 1) for a in range(dim)):
            role = 1
        out.append(role)
    return np.array(out, dtype=np.int8)


@settings(max_examples=25, deadline=None)
@given(n=st.integers(4, 12), cx=st.floats(0.2, 0.8), cy=st.floats(0.2, 0.8), rad=st.floats(0.05, 0.4),
       walls=st.booleans())
def test_roles_brute_force_2d(n, cx, cy, rad, walls):
    l0 = 1.0 / n
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0, walls=walls)
    got = O.roles(m, [O.BodyState((cx, cy), rad, 2)])
    want = _brute_roles((n, n), (0.0, 0.0), l0, (cx, cy), rad, walls)
    # |v-c|^2 >= R^2 and hypot(v-c) - R >= 0 can differ only on exact ties
    assert np.mean(got == want) == 1.0


@settings(max_examples=8, deadline=None)
@given(n=st.integers(4, 7), rad=st.floats(0.1, 0.4))
def test_roles_brute_force_3d(n, rad):
    l0 = 1.0 / n
    m = O.Mesh(3, (n, n, n), (0.0,) * 3, l0, walls=True)
    got = O.roles(m, [O.BodyState((0.47, 0.52, 0.5), rad, 2)])
    want = _brute_roles((n, n, n), (0.0,) * 3, l0, (0.47, 0.52, 0.5), rad, True)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("key", ["cylinder_1024", "sphere_128"])
def test_role_counts_at_t0(key):
    g = json.load(open(os.path.join(GOLD, "role_counts_t0.json")))[key]
    dim = len(g["n"])
    m = O.Mesh(dim, g["n"], g["origin"], g["l0"], walls=True)
    r = O.roles(m, [O.BodyState(tuple(g["centre"]), g["radius"], 2)])
    assert int((r == O.INNER).sum()) == g["inner"]
    assert int((r == 2).sum()) == g["body"]
    assert int((r == O.VOID).sum()) == g["void"]
    assert int((r == 1).sum()) == g["wall"]


def test_no_edge_adjacent_inner_void():
    """An inner cell shares two vertices with psi >= 0 with each edge
    neighbour, so no edge neighbour of an inner cell can be void."""
    n = 64
    m = O.Mesh(2, (n, n), (0.0, 0.0), 1.0 / n)
    r = O.roles(m, [O.BodyState((0.51, 0.43), 0.27, 2)]).reshape(n, n)
    inner, void = r == O.INNER, r == O.VOID
    assert not (inner[:, 1:] & void[:, :-1]).any() and not (inner[:, :-1] & void[:, 1:]).any()
    assert not (inner[1:, :] & void[:-1, :]).any() and not (inner[:-1, :] & void[1:, :]).any()


def test_spring_hand_example():
    """One edge neighbour at 0.8 l0: the spring is compressed by 0.2 and the
    DP moves by kappa l0 (1 - 0.8) = 0.04 l0 away from it (Eqs.
    dimensionless_force_function, 1st_intermed_position)."""
    l0 = 1.0
    m = O.Mesh(2, (3, 3), (0.0, 0.0), l0)
    role = np.zeros(9, np.int8)
    role[4] = O.INNER
    role[5] = O.INNER
    pos = inputs.cell_centroids(m.n, m.origin, l0)
    pos[0, 4] = 1.6
    pos[0, 5] = 2.4          # distance 0.8
    consts = O.RelaxConsts.make(l0)
    out, mx = O.relax_sweep(m, consts, [], role, np.array([4]), pos)
    assert out[0, 4] == pytest.approx(1.6 - 0.04, abs=1e-15)
    assert out[1, 4] == pos[1, 4]
    assert mx == pytest.approx(0.04, abs=1e-15)


def test_regular_grid_is_a_fixed_point():
    n = 10
    m = O.Mesh(2, (n, n), (0.0, 0.0), 0.1, (True, True))
    pos = inputs.cell_centroids(m.n, m.origin, m.l0)
    role = np.full(m.Nc, O.INNER, np.int8)
    out, mx = O.relax_sweep(m, O.RelaxConsts.make(0.1), [], role, np.arange(m.Nc), pos)
    assert mx < 1e-15


def test_update_invariants_cylinder():
    """Every DP ends inside its closed cell; band boundary DPs end on the
    circle unless the mesh constraint clamped them; the clamp is idempotent."""
    n = 96
    l0 = 8.0 / n
    m = O.Mesh(2, (n, n), (-4.0, -4.0), l0, walls=True)
    body = O.BodyState((0.13, -0.07), 0.5, 2)
    pos = inputs.jittered_positions(m.n, m.origin, l0, seed=2)
    role0 = O.roles(m, [body])
    consts = O.RelaxConsts.make(l0)
    up = O.update_dps(m, consts, [body], pos, role0, 300)
    ijk = m.ijk(np.arange(m.Nc))
    for a in range(2):
        lo = m.origin[a] + ijk[a] * l0
        hi = m.origin[a] + (ijk[a] + 1) * l0
        assert np.all(up.pos[a] >= lo) and np.all(up.pos[a] <= hi)
    bnd = np.nonzero(up.role == 2)[0]
    psi = np.hypot(up.pos[0, bnd] - body.centre[0], up.pos[1, bnd] - body.centre[1]) - body.radius
    on_edge = np.zeros(len(bnd), bool)
    for a in range(2):
        lo = m.origin[a] + ijk[a, bnd] * l0
        hi = m.origin[a] + (ijk[a, bnd] + 1) * l0
        on_edge |= (up.pos[a, bnd] == lo) | (up.pos[a, bnd] == hi)
    assert np.all(np.abs(psi[~on_edge]) <= 1e-12 * l0 * 10)
    assert on_edge.mean() < 0.5
    # wall DPs on the walls
    w = np.nonzero(up.role == 1)[0]
    wi = m.ijk(w)
    assert np.all(up.pos[0, w][wi[0] == 0] == -4.0)
    # a second update at the same body position moves nothing already converged
    again = O.update_dps(m, consts, [body], up.pos, up.role, 1)
    assert np.array_equal(again.role, up.role)
    assert np.abs(again.pos - up.pos).max() < 0.05 * l0


def test_transition_codes():
    prev = np.array([0, 0, -1, -1, 2, 2, 0, -1, 2], np.int8)
    new = np.array([0, -1, 0, -1, 0, -1, 2, 2, 2], np.int8)
    assert list(O.transition_codes(prev, new)) == [0, 1, 3, 4, 6, 7, 2, 5, 8]


def _perturbed_regular_3d(kappa, sweeps):
    n = 8
    m = O.Mesh(3, (n, n, n), (0.0,) * 3, 1.0, (True,) * 3)
    pos = inputs.cell_centroids(m.n, m.origin, 1.0)
    rng = np.random.default_rng(0)
    pos = pos + 0.05 * rng.uniform(-1, 1, pos.shape)
    role = np.full(m.Nc, O.INNER, np.int8)
    consts = O.RelaxConsts.make(1.0, kappa)
    mxs = []
    for _ in range(sweeps):
        pos, mx = O.relax_sweep(m, consts, [], role, np.arange(m.Nc), pos)
        mxs.append(mx)
    return mxs


def test_relaxation_stability_3d_reading():
    """Reading for 3D: with the 26 springs of the 3x3x3 block the explicit
    step is stable for kappa = 1/10 (perturbations of a regular grid decay)
    and unstable for the 2D value 1/5 (they grow until the mesh clamp)."""
    stable = _perturbed_regular_3d(0.1, 30)
    assert stable[-1] < 0.2 * stable[0]
    unstable = _perturbed_regular_3d(0.2, 30)
    assert max(unstable[5:]) > 2 * unstable[0]


# ---------------------------------------------------------------------------
# Boundary-fitted arrangement (Sec. 4, Eqs. dp_arrng_boundary-fit_x** and
# dp_arrng_beta)
# ---------------------------------------------------------------------------

def test_fit_cos_is_the_cosine():
    x = np.linspace(-np.pi, np.pi, 20001)
    assert np.abs(O.fit_cos(x) - np.cos(x)).max() < 1e-10
    assert O.fit_cos(0.0) == 1.0 and abs(O.fit_cos(np.pi) + 1.0) < 1e-10


def test_boundary_fitted_step_of_an_inner_dp():
    """DPs at the centroids of a regular grid feel no spring force, so one
    sweep moves an inner DP (whose neighbours are all inner) by exactly
    beta psi towards the body with beta = alpha/2 (1 + cos(pi psi / r_e)) for
    psi < r_e, and not at all for psi >= r_e; alpha = 0 is the original
    algorithm bit for bit."""
    n, l0 = 64, 1.0 / 64
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0)
    body = O.BodyState((0.5 + 0.3 * l0, 0.5 - 0.2 * l0), 10 * l0, 2)
    pos = inputs.cell_centroids(m.n, m.origin, l0)
    role = O.roles(m, [body])
    band = O.band_cells(m, [body], role, 5.0 * l0)
    alpha, re_l0 = 0.03, 3.0          # r_e below the 5 l0 band: band DPs beyond r_e stay
    fit = O.RelaxConsts.make(l0, fit_alpha=alpha, fit_re_over_l0=re_l0)
    out, _ = O.relax_sweep(m, fit, [body], role, band, pos)
    out0, _ = O.relax_sweep(m, O.RelaxConsts.make(l0), [body], role, band, pos)
    out00, _ = O.relax_sweep(m, O.RelaxConsts.make(l0, fit_alpha=0.0), [body], role, band, pos)
    assert np.array_equal(out0, out00)
    ijk = m.ijk(band)
    checked = far = 0
    for k, c in enumerate(band):
        if role[c] != O.INNER:
            continue
        nb = [(ijk[0][k] + dx) + n * (ijk[1][k] + dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
        if any(role[j] != O.INNER for j in nb):
            continue                       # a boundary neighbour exerts a spring force
        d = pos[:, c] - np.array(body.centre)
        r = np.hypot(d[0], d[1])
        psi = r - body.radius
        moved = out[:, c] - out0[:, c]
        if psi >= re_l0 * l0:
            assert np.all(moved == 0.0)
            far += 1
            continue
        beta = alpha / 2 * (1 + np.cos(np.pi * psi / (re_l0 * l0)))
        # fit_cos is the cosine to 1e-10 (absolute), which bounds beta's error
        np.testing.assert_allclose(moved, -beta * psi * d / r, rtol=0, atol=alpha * psi * 1e-10 + 1e-16)
        checked += 1
    assert checked > 20 and far > 0


# ---------------------------------------------------------------------------
# several bodies (Sec. 2.2-2.4 applied per body; nearest-body readings)
# ---------------------------------------------------------------------------

def test_two_separated_bodies_arrange_as_each_alone():
    """Bodies whose bands are far apart: with a fixed sweep count (eps = 0)
    the two-body roles and positions are, bit for bit, the union of the
    single-body results; each body's cells carry its own id."""
    from paper_2404_17542_amd import configs
    case = configs.c2_oscillating_cylinder(n=64)
    m = O.Mesh.from_case(case)
    consts = O.RelaxConsts.make(case.l0, case.kappa, 0.0, case.band_over_l0)
    A = O.BodyState((-2.0, 0.3), 0.6, 2)
    B = O.BodyState((1.9, -0.2), 0.45, 3)
    pos0 = inputs.jittered_positions(case.n, case.origin, case.l0, 3)

    def arrange(bodies):
        return O.update_dps(m, consts, bodies, pos0, O.roles(m, bodies), 40)

    ua, ub, uab = arrange([A]), arrange([B]), arrange([B, A])      # order of the list is irrelevant
    assert uab.sweeps == ua.sweeps == ub.sweeps == 40
    assert np.array_equal(uab.role, np.where(ua.role != O.INNER, ua.role, ub.role))
    assert (uab.role == 2).sum() > 10 and (uab.role == 3).sum() > 10
    moved_a = np.any(ua.pos != pos0, axis=0)
    assert np.array_equal(uab.pos.view(np.int64), np.where(moved_a[None], ua.pos, ub.pos).view(np.int64))
    for up, b in ((ua, A), (ub, B)):
        sel = up.role == b.body_id
        assert np.array_equal(uab.normal[:, sel], up.normal[:, sel])


def test_boundary_cell_takes_the_nearest_body_id():
    """Two circles a few cells apart: every body-boundary cell carries the id
    of the body with the smallest |psi| at its centroid (lower id on ties),
    by brute force over the cells."""
    n, l0 = 48, 1.0 / 48
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0)
    A = O.BodyState((0.3, 0.5), 0.17, 2)
    B = O.BodyState((0.68, 0.47), 0.16, 3)       # surface gap ~ 2.5 l0
    role = O.roles(m, [A, B])
    checked = 0
    for c in range(m.Nc):
        if role[c] in (O.INNER, O.VOID):
            continue
        i, j = c % n, c // n
        x, y = (i + 0.5) * l0, (j + 0.5) * l0
        pa = abs(math.hypot(x - A.centre[0], y - A.centre[1]) - A.radius)
        pb = abs(math.hypot(x - B.centre[0], y - B.centre[1]) - B.radius)
        assert role[c] == (3 if pb < pa else 2), c
        checked += 1
    assert checked > 40 and (role == 3).sum() > 15


def test_boundary_fitted_step_toward_the_nearest_body():
    """The boundary-fitted move of an inner DP between two bodies goes
    towards the body of smaller psi at the DP (lower id on ties):
    x -= beta psi (x - c)/|x - c| of that body (DPs at grid centroids feel
    no spring force)."""
    n, l0 = 64, 1.0 / 64
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0)
    A = O.BodyState((0.3 + 0.2 * l0, 0.5), 9 * l0, 2)
    B = O.BodyState((0.7 - 0.1 * l0, 0.5 + 0.3 * l0), 8 * l0, 3)
    bodies = [A, B]
    pos = inputs.cell_centroids(m.n, m.origin, l0)
    role = O.roles(m, bodies)
    band = O.band_cells(m, bodies, role, 5.0 * l0)
    alpha, re_l0 = 0.03, 8.0
    fit = O.RelaxConsts.make(l0, fit_alpha=alpha, fit_re_over_l0=re_l0)
    out, _ = O.relax_sweep(m, fit, bodies, role, band, pos)
    out0, _ = O.relax_sweep(m, O.RelaxConsts.make(l0), bodies, role, band, pos)
    ijk = m.ijk(band)
    toward = {2: 0, 3: 0}
    for k, c in enumerate(band):
        if role[c] != O.INNER:
            continue
        nb = [(ijk[0][k] + dx) + n * (ijk[1][k] + dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
        if any(role[j] != O.INNER for j in nb):
            continue
        psis = []
        for b in bodies:
            d = pos[:, c] - np.array(b.centre)
            psis.append(np.hypot(d[0], d[1]) - b.radius)
        b = bodies[int(psis[1] < psis[0])]
        d = pos[:, c] - np.array(b.centre)
        r = np.hypot(d[0], d[1])
        psi = r - b.radius
        if psi >= re_l0 * l0:
            continue
        beta = alpha / 2 * (1 + np.cos(np.pi * psi / (re_l0 * l0)))
        np.testing.assert_allclose(out[:, c] - out0[:, c], -beta * psi * d / r, rtol=0,
                                   atol=alpha * psi * 1e-10 + 1e-16)
        toward[b.body_id] += 1
    assert toward[2] > 20 and toward[3] > 20
