"""Pins of the oracle's fluid-force evaluation (Sec. 3.4): closed forms for
fields the quadratic MLS reconstructs exactly, so that only the surface
quadrature (the dGamma elements and the DP normals) is approximate.

* linear pressure P = a + c y, u = 0:  F = -oint P n = (0, -c pi R^2)
  (Archimedes), to the accuracy of the surface polygon through the
  boundary DPs (measured 2.2e-4 at 256^2 and 1.2e-4 at 512^2: boundary DPs
  clamped onto a cell edge sit up to 0.05 l0 off the circle);
* u = (y^2, 0), P = 0:  F = mu oint (grad u + grad u^T) n = mu (2 pi R^2, 0);
* rigid rotation and uniform pressure: no force beyond the quadrature error;
* the diamond angle orders points like the polar angle.
"""
import math

import numpy as np
import pytest

from oracle import mcd_oracle as O
from paper_2404_17542_amd import configs, inputs


def _arranged_cylinder(n):
    case = configs.c2_oscillating_cylinder(n=n)
    m = O.Mesh.from_case(case)
    consts = O.RelaxConsts.make(case.l0, case.kappa, case.eps_relax, case.band_over_l0)
    b = case.body
    body = O.BodyState(centre=b.motion.centre(0.0), radius=b.radius, body_id=b.body_id)
    pos = inputs.jittered_positions(case.n, case.origin, case.l0, case.jitter_seed)
    up = O.update_dps(m, consts, [body], pos, O.roles(m, [body]), 100)
    return case, m, body, up.pos, up.role, up.normal


def _force(case, m, body, pos, role, nrm, u, p, f, mu):
    re, rs = case.re_over_l0 * case.l0, case.rs_over_l0 * case.l0
    F, cnt = O.fluid_force(m, pos, role, nrm, [body], case.bc_velocity, case.bc_pressure, u, p, f, re, rs, mu,
                           case.weight)
    return F[0], cnt[0]


def test_linear_pressure_gives_archimedes_force():
    c, a = 3.0, 0.7
    errs = []
    for n in (256, 512):
        case, m, body, pos, role, nrm = _arranged_cylinder(n)
        p = a + c * pos[1]
        f = np.where(role == body.body_id, c * nrm[1], 0.0)        # dP/dn at the body
        u = np.zeros((2, m.Nc))
        F, (nb, nfb) = _force(case, m, body, pos, role, nrm, u, p, f, 0.01)
        exact = -c * math.pi * body.radius ** 2
        assert nb > 50 and nfb == 0
        assert abs(F[0]) < 1e-2 * abs(exact)
        errs.append(abs(F[1] - exact) / abs(exact))
    assert max(errs) < 1e-3, errs


def test_quadratic_shear_gives_the_viscous_force():
    mu = 0.05
    case, m, body, pos, role, nrm = _arranged_cylinder(512)
    u = np.stack([pos[1] ** 2, np.zeros(m.Nc)])
    F, _ = _force(case, m, body, pos, role, nrm, u, np.zeros(m.Nc), np.zeros(m.Nc), mu)
    exact = 2 * mu * math.pi * body.radius ** 2
    assert abs(F[0] - exact) / exact < 1e-3, (F, exact)      # measured 1.3e-4
    assert abs(F[1]) < 1e-3 * exact


def test_rigid_rotation_and_uniform_pressure_give_no_force():
    case, m, body, pos, role, nrm = _arranged_cylinder(256)
    xc, yc = body.centre
    u = np.stack([-(pos[1] - yc), pos[0] - xc]) * 2.0
    p = np.full(m.Nc, 5.0)
    F, _ = _force(case, m, body, pos, role, nrm, u, p, np.zeros(m.Nc), 0.1)
    # -P oint n dGamma with P = 5 over a perimeter of pi: quadrature-level only
    assert np.abs(F).max() < 1e-2 * 5.0 * math.pi * 2 * body.radius


def test_diamond_angle_is_monotone_in_the_polar_angle():
    th = np.linspace(0, 2 * np.pi, 1001)[:-1]
    d = O.diamond_angle(np.cos(th), np.sin(th))
    assert np.all(np.diff(d) > 0) and d[0] == 0.0 and d[-1] < 4.0
    assert O.diamond_angle(np.array([0.0]), np.array([1.0]))[0] == 1.0
    assert O.diamond_angle(np.array([-1.0]), np.array([0.0]))[0] == 2.0
    assert O.diamond_angle(np.array([0.0]), np.array([-1.0]))[0] == 3.0
