"""Host logic of the learned-guess trajectory variants: seeded amplitude and
frequency in their ranges, Re = 100 kept, and the CFL number of the base
flow never exceeded."""
import math

import pytest

from paper_2404_17542_amd import configs


@pytest.mark.parametrize("variant,base", [(configs.c3_cylinder_variant, configs.c2_oscillating_cylinder),
                                          (configs.c4_sphere_variant, configs.c4_moving_sphere)])
def test_variants(variant, base):
    b = base(n=64)
    diam = 2 * b.body.radius
    cfl_base = 2 * math.pi * b.body.motion.freq * b.body.motion.amplitude * b.dt / b.l0
    seen = set()
    for seed in range(1000, 1020):
        c = variant(seed, n=64)
        m = c.body.motion
        assert 0.1 * diam <= m.amplitude <= 0.4 * diam and 0.5 <= m.freq <= 2.0
        u = 2 * math.pi * m.freq * m.amplitude
        assert u * diam / c.nu == pytest.approx(100.0)
        assert u * c.dt / c.l0 <= cfl_base * (1 + 1e-12)
        assert c.jitter_seed == seed and c.dim == b.dim and c.n == b.n
        assert variant(seed, n=64) == c
        seen.add((m.amplitude, m.freq))
    assert len(seen) == 20


def test_two_cylinders_case():
    """Distinct body ids with a boundary condition each, the phase-shifted
    oscillation of the second body (c(0) = c0 + A e_y), a surface gap that
    stays positive over a period, and overlapping 5 l0 bands on 128^2."""
    c = configs.c2_two_cylinders(n=128)
    A, B = c.rigid_bodies
    assert (A.body_id, B.body_id) == (configs.BODY_ID, configs.BODY_ID + 1)
    for bc in (c.bc_pressure, c.bc_velocity):
        assert set(bc) == {configs.WALL_ID, A.body_id, B.body_id}
    assert B.motion.centre(0.0) == (0.5, 0.15)
    assert abs(B.motion.velocity(0.0)[1]) < 1e-15
    gaps = []
    for k in range(200):
        t = k / 200.0
        ca, cb = A.motion.centre(t), B.motion.centre(t)
        gaps.append(math.dist(ca, cb) - A.radius - B.radius)
    assert 0.35 < min(gaps) < max(gaps) < 2 * c.band_over_l0 * c.l0 + 0.1
    assert min(gaps) < 2 * c.band_over_l0 * c.l0
    assert configs.c2_oscillating_cylinder(n=128).rigid_bodies == (configs.c2_oscillating_cylinder(n=128).body,)
    assert configs.c1_taylor_green(n=64).rigid_bodies == ()


def test_prescribed_motions_differentiate_consistently():
    """velocity and omega are the time derivatives of centre and theta
    (central differences), for the oscillation with spin and the flapping
    wing; the wing's stroke runs along beta and its period is pi a0."""
    from paper_2404_17542_amd.inputs import FlappingMotion, Oscillation
    motions = [Oscillation((0.1, 0.2), 0.15, 1.3, 1, 0.4, spin_amplitude=0.3, spin_freq=0.7, theta0=0.2),
               FlappingMotion((0.0, 0.0), 2.5, math.pi / 3, math.pi / 4, 0.3)]
    h = 1e-6
    for mo in motions:
        for t in (0.0, 0.37, 1.9):
            c1, c0 = mo.centre(t + h), mo.centre(t - h)
            for a in range(2):
                assert abs((c1[a] - c0[a]) / (2 * h) - mo.velocity(t)[a]) < 1e-7
            assert abs((mo.theta(t + h) - mo.theta(t - h)) / (2 * h) - mo.omega(t)) < 1e-7
            assert mo.omega_vector(t) == (0.0, 0.0, mo.omega(t))
    wing = motions[1]
    T = math.pi * wing.a0
    for t in (0.0, 0.8, 2.1):
        assert all(abs(u - v) < 1e-12 for u, v in zip(wing.centre(t), wing.centre(t + T)))
        c = wing.centre(t)
        assert abs(c[1] * math.cos(wing.beta) - c[0] * math.sin(wing.beta)) < 1e-12
