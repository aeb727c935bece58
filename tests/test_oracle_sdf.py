"""Pins of the discrete-SDF body (Sec. 2.5: an SDF sampled on its own grid,
read through the chi_c = 1 MLS of Sec. 3.2 at the body's posture) and of
the ellipse SDF generator used as its input."""
import math

import numpy as np
import pytest

from oracle import mcd_oracle as O
from paper_2404_17542_amd import inputs


def _body(values, origin, h, centre=(0.0, 0.0), theta=0.0, radius=1.0, far=1e9, kind="cos2", re=2.5):
    g = O.SdfGrid(np.asarray(values, dtype=np.float64), origin, h, re, kind, far)
    return O.BodyState(centre, radius, 2, (0.0, 0.0), (0.0, 0.0, 0.0), theta, g)


def _grid(n, h, f):
    o = (-(n // 2) * h, -(n // 2) * h)
    ax0 = o[0] + h * np.arange(n)
    X, Y = np.meshgrid(ax0, ax0)
    return f(X, Y), o


@pytest.mark.parametrize("kind", ["cos2", "gauss"])
def test_quadratics_are_reproduced_at_any_posture(kind):
    """A quadratic sampled on the grid is reproduced exactly (psi and its
    gradient) at any point and posture: the chi_c = 1 quadratic fit is exact
    for quadratics."""
    rng = np.random.default_rng(1)
    cq = rng.standard_normal(6)

    def q(X, Y):
        return cq[0] + cq[1] * X + cq[2] * Y + cq[3] * X * X + cq[4] * X * Y + cq[5] * Y * Y

    h = 0.05
    vals, o = _grid(41, h, q)
    c, th = (0.3, -0.7), 0.83
    b = _body(vals, o, h, c, th, kind=kind)
    K = 400
    xi = rng.uniform(-0.8, 0.8, (2, K))
    x = np.stack([c[0] + math.cos(th) * xi[0] - math.sin(th) * xi[1],
                  c[1] + math.sin(th) * xi[0] + math.cos(th) * xi[1]])
    psi, g = O.sdf_eval(b, x)
    np.testing.assert_allclose(psi, q(xi[0], xi[1]), rtol=0, atol=1e-12)
    gx = cq[1] + 2 * cq[3] * xi[0] + cq[4] * xi[1]
    gy = cq[2] + cq[4] * xi[0] + 2 * cq[5] * xi[1]
    np.testing.assert_allclose(g[0], math.cos(th) * gx - math.sin(th) * gy, rtol=0, atol=1e-10)
    np.testing.assert_allclose(g[1], math.sin(th) * gx + math.cos(th) * gy, rtol=0, atol=1e-10)


def test_discrete_circle_converges_at_third_order():
    """A circle given as a sampled SDF: psi at random points approaches
    |x - c| - R with an error that falls about 8x per halving of h (the
    quadratic fit's third-order truncation), and grad psi is close to the
    radial unit vector."""
    R = 0.5
    rng = np.random.default_rng(2)
    ang = rng.uniform(0, 2 * math.pi, 500)
    rad = rng.uniform(0.3, 0.8, 500)
    c = (0.1, 0.2)
    x = np.stack([c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang)])
    errs = []
    for h in (0.04, 0.02, 0.01):
        n = int(round(2.0 / h)) + 1
        vals, o = _grid(n, h, lambda X, Y: np.hypot(X, Y) - R)
        b = _body(vals, o, h, c, theta=0.4)
        psi, g = O.sdf_eval(b, x)
        errs.append(np.abs(psi - (rad - R)).max())
        assert np.abs(g[0] - np.cos(ang)).max() < 50 * h * h and np.abs(g[1] - np.sin(ang)).max() < 50 * h * h
    assert errs[0] / errs[1] > 5.0 and errs[1] / errs[2] > 5.0, errs


def test_far_points_take_the_bounding_disc():
    vals, o = _grid(21, 0.1, lambda X, Y: np.hypot(X, Y) - 0.5)
    b = _body(vals, o, 0.1, (1.0, 2.0), theta=1.0, radius=0.6, far=0.8)
    x = np.array([[1.0 + 0.9, 1.0, 1.0 - 0.5], [2.0, 2.0 + 2.5, 2.0 - 0.7]])
    psi, g = O.sdf_eval(b, x)
    r = np.hypot(x[0] - 1.0, x[1] - 2.0)
    np.testing.assert_array_equal(psi, r - 0.6)
    np.testing.assert_allclose(g[0], (x[0] - 1.0) / r)


def test_posture_rotates_the_shape():
    """The ellipse's SDF grid at posture theta gives, at x, the ellipse
    distance at R(-theta)(x - c) (within the interpolation error where the
    distance is smooth: in the fluid and within 2h inside the surface; the
    kink of the interior distance on the focal segment is not resolved); a quarter
    turn swaps the axes."""
    a, bb, h = 0.5, 0.125, 0.0125
    vals, o, h = inputs.ellipse_sdf_grid(a, bb, h, 0.9)
    c, th = (0.2, -0.1), 0.6
    body = _body(vals, o, h, c, th, radius=a)
    rng = np.random.default_rng(3)
    xi = rng.uniform(-0.7, 0.7, (2, 2000))
    x = np.stack([c[0] + math.cos(th) * xi[0] - math.sin(th) * xi[1],
                  c[1] + math.sin(th) * xi[0] + math.cos(th) * xi[1]])
    psi, _ = O.sdf_eval(body, x)
    exact = inputs.ellipse_distance(a, bb, xi[0], xi[1])
    fluid = exact >= 0.0
    assert fluid.sum() > 1500
    # largest near the tips, whose radius of curvature b^2/a is only 2.5 h
    assert np.abs(psi - exact)[fluid].max() < 0.01 * h
    near = (exact < 0.0) & (exact > -2 * h)
    assert np.abs(psi - exact)[near].max() < 0.05 * h
    q = _body(vals, o, h, (0.0, 0.0), 0.5 * math.pi, radius=a)
    pts = np.array([[0.0, 0.0, 0.3], [0.6, -0.6, 0.0]])
    psi_q, _ = O.sdf_eval(q, pts)
    np.testing.assert_allclose(psi_q, [0.1, 0.1, 0.3 - bb], atol=1e-3 * h)


def test_discrete_circle_roles_match_the_analytic_circle():
    """Masks from a sampled circle SDF equal the analytic circle's except
    where a vertex lies within the interpolation error of the surface."""
    n, l0 = 64, 1.0 / 64
    m = O.Mesh(2, (n, n), (0.0, 0.0), l0)
    c, R = (0.5 + 0.3 * l0, 0.5 - 0.2 * l0), 10.3 * l0
    h = 0.5 * l0
    vals, o = _grid(161, h, lambda X, Y: np.hypot(X, Y) - R)
    sb = _body(vals, o, h, c, theta=0.3, radius=R, far=O.sdf_far_radius(R, l0, 5.0))
    ab = O.BodyState(c, R, 2)
    rs, ra = O.roles(m, [sb]), O.roles(m, [ab])
    diff = np.nonzero(rs != ra)[0]
    ijk = m.ijk(np.arange(m.Nc))
    near = np.zeros(m.Nc, dtype=bool)
    for v in range(4):
        vx = m.origin[0] + (ijk[0] + (v & 1)) * l0
        vy = m.origin[1] + (ijk[1] + (v >> 1)) * l0
        near |= np.abs(np.hypot(vx - c[0], vy - c[1]) - R) < 1e-3 * h
    assert np.all(near[diff]), diff
    assert (ra == 2).sum() > 40
    np.testing.assert_array_equal(O.band_cells(m, [sb], rs, 5 * l0), O.band_cells(m, [ab], ra, 5 * l0))


def test_ellipse_distance_closed_forms():
    """On the axes the distance is closed-form; elsewhere it matches a
    dense sampling of the boundary."""
    a, b = 0.5, 0.125
    d = inputs.ellipse_distance(a, b, np.array([0.7, 0.0, -0.9, 0.0]), np.array([0.0, 0.3, 0.0, -0.05]))
    np.testing.assert_allclose(d, [0.2, 0.175, 0.4, -0.075], atol=1e-15)
    rng = np.random.default_rng(4)
    P = rng.uniform(-0.8, 0.8, (2, 200))
    t = np.linspace(0, 2 * np.pi, 400001)
    E = np.stack([a * np.cos(t), b * np.sin(t)])
    bf = np.array([np.min(np.hypot(E[0] - p[0], E[1] - p[1])) for p in P.T])
    d = inputs.ellipse_distance(a, b, P[0], P[1])
    np.testing.assert_allclose(np.abs(d), bf, atol=5e-9)
    inside = (P[0] / a) ** 2 + (P[1] / b) ** 2 < 1
    assert np.all((d < 0) == inside)


@pytest.mark.parametrize("kind,re", [("cos2", 2.5), ("gauss", 2.5), ("cos2", 1.6)])
def test_closed_form_equals_the_weighted_least_squares_fit(kind, re):
    """The closed-form Phi of the symmetric 3x3 support equals a direct
    weighted least-squares solve (numpy lstsq of sqrt(w) p . Phi = sqrt(w)
    dpsi over the eight nodes) for random node values."""
    rng = np.random.default_rng(5)
    vals = rng.standard_normal((7, 7))
    h = 0.1
    b = _body(vals, (-0.3, -0.3), h, kind=kind, re=re)
    pts = np.stack([rng.uniform(-0.15, 0.15, 50), rng.uniform(-0.15, 0.15, 50)])
    psi, g = O.sdf_eval(b, pts)
    for k in range(pts.shape[1]):
        q = (pts[:, k] - np.array([-0.3, -0.3])) / h
        i, j = int(np.floor(q[0] + 0.5)), int(np.floor(q[1] + 0.5))
        rows, rhs = [], []
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                if di == 0 and dj == 0:
                    continue
                w = float(O.weight(np.hypot(di, dj), re, kind))
                rows.append(math.sqrt(w) * np.array([di, dj, 0.5 * di * di, di * dj, 0.5 * dj * dj]))
                rhs.append(math.sqrt(w) * (vals[j + dj, i + di] - vals[j, i]))
        phi = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
        s = q - np.array([i, j])
        ref = vals[j, i] + phi @ np.array([s[0], s[1], 0.5 * s[0] ** 2, s[0] * s[1], 0.5 * s[1] ** 2])
        gref = np.array([phi[0] + s[0] * phi[2] + s[1] * phi[3], phi[1] + s[0] * phi[3] + s[1] * phi[4]]) / h
        assert abs(psi[k] - ref) < 1e-12
        assert abs(g[0][k] - gref[0]) < 1e-10 and abs(g[1][k] - gref[1]) < 1e-10


# ---------------------------------------------------------------------------
# 3D (the same rule over the 3x3x3 nodes, posture about an axis)
# ---------------------------------------------------------------------------

def _body3(values, origin, h, centre=(0.0, 0.0, 0.0), theta=0.0, axis=(0.0, 0.0, 1.0), radius=1.0, far=1e9,
           kind="cos2", re=2.5):
    g = O.SdfGrid(np.asarray(values, dtype=np.float64), origin, h, re, kind, far)
    return O.BodyState(centre, radius, 2, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), theta, g, axis)


def _grid3(n, h, f):
    o = (-(n // 2) * h,) * 3
    ax = o[0] + h * np.arange(n)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    return f(X, Y, Z), o


def test_posture_matrix_is_the_rotation_about_the_axis():
    rng = np.random.default_rng(6)
    a = rng.standard_normal(3)
    a /= np.linalg.norm(a)
    th = 0.77
    R = np.array(O.posture_matrix(th, a)).reshape(3, 3)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-15)
    assert abs(np.linalg.det(R) - 1.0) < 1e-14
    np.testing.assert_allclose(R @ a, a, atol=1e-15)
    u = np.cross(a, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    assert abs(float(u @ (R @ u)) - math.cos(th)) < 1e-14        # turns by theta in the plane normal to a
    Rz = np.array(O.posture_matrix(th, (0.0, 0.0, 1.0))).reshape(3, 3)
    np.testing.assert_allclose(Rz[:2, :2], [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]], atol=0)


@pytest.mark.parametrize("kind", ["cos2", "gauss"])
def test_quadratics_are_reproduced_in_3d(kind):
    rng = np.random.default_rng(7)
    cq = rng.standard_normal(10)

    def q(X, Y, Z):
        return (cq[0] + cq[1] * X + cq[2] * Y + cq[3] * Z + cq[4] * X * X + cq[5] * Y * Y + cq[6] * Z * Z
                + cq[7] * X * Y + cq[8] * Y * Z + cq[9] * Z * X)

    h = 0.1
    vals, o = _grid3(17, h, q)
    a = np.array([0.3, -0.5, 0.8])
    a /= np.linalg.norm(a)
    c, th = (0.2, -0.1, 0.3), 1.1
    b = _body3(vals, o, h, c, th, tuple(a), kind=kind)
    R = np.array(O.posture_matrix(th, a)).reshape(3, 3)
    xi = rng.uniform(-0.55, 0.55, (3, 300))
    x = np.array(c)[:, None] + R @ xi
    psi, g = O.sdf_eval(b, x)
    np.testing.assert_allclose(psi, q(*xi), rtol=0, atol=1e-12)
    gxi = np.stack([cq[1] + 2 * cq[4] * xi[0] + cq[7] * xi[1] + cq[9] * xi[2],
                    cq[2] + 2 * cq[5] * xi[1] + cq[7] * xi[0] + cq[8] * xi[2],
                    cq[3] + 2 * cq[6] * xi[2] + cq[8] * xi[1] + cq[9] * xi[0]])
    np.testing.assert_allclose(np.array(g), R @ gxi, rtol=0, atol=1e-10)


def test_3d_closed_form_equals_the_weighted_least_squares_fit():
    rng = np.random.default_rng(8)
    vals = rng.standard_normal((6, 6, 6))
    h, re = 0.1, 2.5
    b = _body3(vals, (-0.25, -0.25, -0.25), h, re=re)
    pts = rng.uniform(-0.1, 0.1, (3, 30))
    psi, g = O.sdf_eval(b, pts)
    for k in range(pts.shape[1]):
        q = (pts[:, k] + 0.25) / h
        i, j, l = (int(np.floor(v + 0.5)) for v in q)
        rows, rhs = [], []
        for dk in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    if di == dj == dk == 0:
                        continue
                    w = float(O.weight(math.sqrt(di * di + dj * dj + dk * dk), re, "cos2"))
                    rows.append(math.sqrt(w) * np.array([di, dj, dk, 0.5 * di * di, 0.5 * dj * dj, 0.5 * dk * dk,
                                                         di * dj, dj * dk, dk * di]))
                    rhs.append(math.sqrt(w) * (vals[l + dk, j + dj, i + di] - vals[l, j, i]))
        phi = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
        s = q - np.array([i, j, l])
        p = np.array([s[0], s[1], s[2], 0.5 * s[0] ** 2, 0.5 * s[1] ** 2, 0.5 * s[2] ** 2, s[0] * s[1], s[1] * s[2],
                      s[2] * s[0]])
        assert abs(psi[k] - (vals[l, j, i] + phi @ p)) < 1e-12


def test_3d_sampled_sphere_converges_and_capsule_sdf_closed_forms():
    R0 = 0.4
    rng = np.random.default_rng(9)
    d = rng.standard_normal((3, 300))
    d /= np.linalg.norm(d, axis=0)
    rad = rng.uniform(0.3, 0.6, 300)
    x = d * rad
    errs = []
    for h in (0.05, 0.025):
        n = int(round(1.6 / h)) + 1
        vals, o = _grid3(n, h, lambda X, Y, Z: np.sqrt(X * X + Y * Y + Z * Z) - R0)
        psi, _ = O.sdf_eval(_body3(vals, o, h, theta=0.3, axis=(0.0, 0.6, 0.8)), x)
        errs.append(np.abs(psi - (rad - R0)).max())
    assert errs[0] / errs[1] > 5.0, errs
    vals, o, h = inputs.capsule_sdf_grid(0.12, 0.06, 0.01, 0.3)
    ax = o[0] + h * np.arange(vals.shape[0])
    i0 = int(np.argmin(np.abs(ax)))
    assert abs(vals[i0, i0, i0] + 0.06) < 1e-15                       # centre: -radius
    i1 = int(np.argmin(np.abs(ax - 0.2)))
    assert abs(vals[i0, i0, i1] - (ax[i1] - 0.12 - 0.06)) < 1e-15      # beyond the cap along x
    assert abs(vals[i1, i0, i0] - (ax[i1] - 0.06)) < 1e-15             # off the axis along z
