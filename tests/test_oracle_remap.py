"""Pins of the oracle's remap for DPs that enter the fluid (Appendix A,
Eq. A.2, with the shifted support of Sec. 3.4).

A DP that was on the body boundary at step k and is inner at step k+1 takes
its value from the step-k fit of the neighbouring cell c' one cell further
into the fluid: c' = c + sign(x^k - x_b) per axis for a circle (psi grows
away from the centre).  The expected values here come from an independent
weighted least-squares fit (numpy lstsq) of c' 's 3x3 block, written from
the definition of the chi_c = 1 quadratic MLS, not from the oracle's
Cholesky; c' comes from integer cell arithmetic and the geometry.  A
flipped shift sign, a wrong c' or a missing fallback fails one of these.
"""
import math

import numpy as np

from oracle import mcd_oracle as O
from paper_2404_17542_amd import inputs

N, L0 = 32, 1.0 / 16.0
RE, RS = 2.5 * L0, L0
BODY = 2
BC_U = {BODY: O.DIRICHLET}          # velocity set: no-slip body (value rows)
XB_K = (1.0, 1.0)                   # body centre at step k
XB_K1 = (1.0 + 0.3 * L0, 1.0 - 0.2 * L0)   # and at step k+1
R = 0.4


def _cubic(p):
    """A cubic velocity component in cell units: a quadratic fit cannot
    reproduce it, so the fitted value depends on which block was fitted."""
    x = (p[0] - 1.0) / L0
    y = (p[1] - 1.0) / L0
    return 0.3 + 0.2 * x - 0.1 * y + 0.05 * x * x - 0.04 * x * y + 0.03 * y * y + 0.02 * x ** 3 - 0.015 * x * y * y


def _quadratic(p):
    x = (p[0] - 1.0) / L0
    y = (p[1] - 1.0) / L0
    return -0.2 + 0.1 * x + 0.25 * y - 0.07 * x * x + 0.05 * x * y + 0.04 * y * y


def _two_steps():
    """Positions and roles at steps k and k+1 of a circle that moves by
    (0.3, -0.2) l0, arranged by the oracle's DP update."""
    m = O.Mesh(2, (N, N), (0.0, 0.0), L0)
    consts = O.RelaxConsts.make(L0)
    bk = [O.BodyState(XB_K, R, BODY, (0.0, 0.0))]
    bk1 = [O.BodyState(XB_K1, R, BODY, (0.0, 0.0))]
    pos0 = inputs.jittered_positions(m.n, m.origin, L0, seed=21)
    up_k = O.update_dps(m, consts, bk, pos0, O.roles(m, bk), 200)
    up_k1 = O.update_dps(m, consts, bk1, up_k.pos, up_k.role, 20)
    return m, bk, bk1, up_k, up_k1


def _lstsq_value(m, pos_k, role_k, u, centre, x_eval):
    """chi_c = 1 quadratic MLS at `centre` over its 3x3 block at step k
    (value rows: inner and no-slip body DPs other than the centre; cos^2
    weight), solved as a weighted least-squares problem, evaluated at x_eval."""
    ci, cj = centre % N, centre // N
    xc = pos_k[:, centre]
    rows, rhs = [], []
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            i, j = ci + di, cj + dj
            if (di, dj) == (0, 0) or not (0 <= i < N and 0 <= j < N):
                continue
            c = i + N * j
            if role_k[c] not in (O.INNER, BODY):
                continue
            dx, dy = pos_k[0, c] - xc[0], pos_k[1, c] - xc[1]
            r = math.hypot(dx, dy)
            if r > RE:
                continue
            w = math.cos(math.pi * r / (2.0 * RE)) ** 2
            X, Y = dx / RS, dy / RS
            sw = math.sqrt(w)
            rows.append([sw * X, sw * Y, sw * X * X / 2, sw * X * Y, sw * Y * Y / 2])
            rhs.append(sw * (u[c] - u[centre]))
    A = np.array(rows)
    assert A.shape[0] >= 5 and np.linalg.matrix_rank(A) == 5
    phi = np.linalg.lstsq(A, np.array(rhs), rcond=None)[0]
    X, Y = (x_eval[0] - xc[0]) / RS, (x_eval[1] - xc[1]) / RS
    return u[centre] + phi @ np.array([X, Y, X * X / 2, X * Y, Y * Y / 2])


def _expected_source(m, pos_k, c):
    """Cell c' = c + sign(x^k - x_b) per axis, in integer cell arithmetic."""
    ci, cj = c % N, c // N
    sx = int(pos_k[0, c] > XB_K[0]) - int(pos_k[0, c] < XB_K[0])
    sy = int(pos_k[1, c] > XB_K[1]) - int(pos_k[1, c] < XB_K[1])
    return (ci + sx) + N * (cj + sy)


def _centroid_dist(c):
    ci, cj = c % N, c // N
    return math.hypot((ci + 0.5) * L0 - XB_K[0], (cj + 0.5) * L0 - XB_K[1])


def test_entering_dps_take_the_shifted_fit_into_the_fluid():
    """Every DP that goes boundary -> inner reads the step-k fit of
    c' = c + sign(x^k - x_b): a cell farther from the body than c, inner at
    step k; with a cubic field its value equals the independent fit of c'
    's block evaluated at x^{k+1} (and differs from the fit of c's own
    block, so the test sees which block was used)."""
    m, bk, bk1, up_k, up_k1 = _two_steps()
    entering = np.nonzero((up_k.role == BODY) & (up_k1.role == O.INNER))[0]
    assert len(entering) >= 4
    st_k = O.mls_build(m, up_k.pos, up_k.role, up_k.normal, BC_U, RE, RS)
    u = np.zeros((2, m.Nc))
    u[0] = _cubic(up_k.pos)
    u[1] = _quadratic(up_k.pos)
    out, stats = O.remap_velocity(m, st_k, u, up_k.pos, up_k1.pos, up_k.role, up_k1.role, bk, bk1)
    assert stats["fallback"] == 0 and stats["shifted"] == len(entering)
    for c in entering:
        cp = _expected_source(m, up_k.pos, c)
        assert stats["src"][c] == cp
        assert _centroid_dist(cp) > _centroid_dist(c)          # into the fluid
        assert up_k.role[cp] == O.INNER
        want = _lstsq_value(m, up_k.pos, up_k.role, u[0], cp, up_k1.pos[:, c])
        own = _lstsq_value(m, up_k.pos, up_k.role, u[0], c, up_k1.pos[:, c])
        assert abs(out[0, c] - want) <= 1e-11, (c, out[0, c], want)
        assert abs(own - want) > 1e-6            # the two blocks are distinguishable
        # the quadratic component is reproduced exactly at x^{k+1}
        assert abs(out[1, c] - _quadratic(up_k1.pos[:, c])) <= 1e-11


def test_flipped_shift_would_point_into_the_body():
    """The opposite shift c - sign(x^k - x_b) lands on a cell that is not
    inner at step k (void or on the body) for every entering DP: the
    direction is what makes the shifted support usable."""
    m, bk, bk1, up_k, up_k1 = _two_steps()
    entering = np.nonzero((up_k.role == BODY) & (up_k1.role == O.INNER))[0]
    for c in entering:
        cp = _expected_source(m, up_k.pos, c)
        flipped = 2 * c - cp
        assert up_k.role[flipped] != O.INNER
        assert _centroid_dist(flipped) < _centroid_dist(c)


def test_entering_dp_falls_back_to_its_own_fit_when_c_prime_was_not_inner():
    """Hand-built: one entering DP's c' is marked as a body DP at step k.
    The remap then uses the DP's own step-k fit (counted as a fallback), and
    the value equals the independent fit of its own block."""
    m, bk, bk1, up_k, up_k1 = _two_steps()
    entering = np.nonzero((up_k.role == BODY) & (up_k1.role == O.INNER))[0]
    role_k = up_k.role.copy()
    u = np.zeros((2, m.Nc))
    u[0] = _cubic(up_k.pos)
    u[1] = _quadratic(up_k.pos)
    chosen = None
    for c in entering:
        cp = _expected_source(m, up_k.pos, c)
        trial = role_k.copy()
        trial[cp] = BODY
        try:
            _lstsq_value(m, up_k.pos, trial, u[0], c, up_k1.pos[:, c])
        except AssertionError:
            continue                      # own block too thin for a fit
        chosen, role_k = c, trial
        break
    assert chosen is not None
    st_k = O.mls_build(m, up_k.pos, role_k, up_k.normal, BC_U, RE, RS)
    assert not st_k.singular[chosen]
    out, stats = O.remap_velocity(m, st_k, u, up_k.pos, up_k1.pos, role_k, up_k1.role, bk, bk1)
    assert stats["fallback"] >= 1
    assert stats["src"][chosen] == chosen
    want = _lstsq_value(m, up_k.pos, role_k, u[0], chosen, up_k1.pos[:, chosen])
    assert abs(out[0, chosen] - want) <= 1e-11
    # the other entering DPs still take their shifted fits
    for c in entering:
        if c != chosen and role_k[_expected_source(m, up_k.pos, c)] == O.INNER:
            assert stats["src"][c] == _expected_source(m, up_k.pos, c)


def test_dp_entering_the_body_boundary_takes_the_body_velocity():
    """inner -> boundary: the no-slip body velocity V_b^{k+1}."""
    m, bk, bk1, up_k, up_k1 = _two_steps()
    bk1 = [O.BodyState(XB_K1, R, BODY, (0.7, -0.4))]
    st_k = O.mls_build(m, up_k.pos, up_k.role, up_k.normal, BC_U, RE, RS)
    u = np.stack([_cubic(up_k.pos), _quadratic(up_k.pos)])
    out, _ = O.remap_velocity(m, st_k, u, up_k.pos, up_k1.pos, up_k.role, up_k1.role, bk, bk1)
    onto = np.nonzero((up_k.role == O.INNER) & (up_k1.role == BODY))[0]
    assert len(onto) >= 1
    assert np.all(out[0, onto] == 0.7) and np.all(out[1, onto] == -0.4)
    assert np.all(out[:, up_k1.role == O.VOID] == 0.0)
