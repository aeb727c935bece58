"""Workload definitions (data only): mesh, DP jitter seed, bodies, physics constants.

Role ids: the outer ring (2D) / shell (3D) of cells is the wall boundary with
id WALL_ID; the moving rigid body has id BODY_ID (further bodies take the ids
after it).  Per-field boundary
conditions are given per id (Dirichlet or Neumann) for the pressure set and
the velocity set.
"""
from __future__ import annotations

import math

import numpy as np
from dataclasses import dataclass, field, replace
from typing import Optional

from .inputs import FlappingMotion, Oscillation, capsule_sdf_grid, ellipse_sdf_grid

WALL_ID = 1
BODY_ID = 2

DIRICHLET = 0
NEUMANN = 1


@dataclass(frozen=True)
class Body:
    """A rigid circle (2D) or sphere (3D) with prescribed motion; with
    `ellipse` = (a, b), a >= b, a 2D ellipse given to the method as a
    discrete SDF (Sec. 2.5) on its own grid of spacing sdf_h_over_l0 * l0,
    major axis along the body-frame x axis, and `radius` = a bounds it."""
    radius: float
    motion: object
    body_id: int = BODY_ID
    ellipse: Optional[tuple] = None
    capsule: Optional[tuple] = None      # 3D: (half length, radius), axis along body-frame x
    sdf_h_over_l0: float = 0.5

    def sdf_grid(self, l0, band_over_l0):
        """(values, origin, h) of the body's discrete SDF, covering the ball of
        radius R + (band + 2) l0 with its inner nodes, or None."""
        if self.ellipse is None and self.capsule is None:
            return None
        h = self.sdf_h_over_l0 * l0
        reach = self.radius + (band_over_l0 + 2.0) * l0 + h
        if self.capsule is not None:
            return capsule_sdf_grid(self.capsule[0], self.capsule[1], h, reach)
        return ellipse_sdf_grid(self.ellipse[0], self.ellipse[1], h, reach)

    def posture_axis(self):
        return tuple(getattr(self.motion, "spin_axis", (0.0, 0.0, 1.0)))


@dataclass(frozen=True)
class Case:
    name: str
    dim: int
    n: tuple
    origin: tuple
    l0: float
    periodic: tuple
    walls: bool
    jitter_seed: int
    weight: str = "cos2"          # "cos2" (paper) or "gauss"
    re_over_l0: float = 2.5
    rs_over_l0: float = 1.0
    kappa: float = 0.2
    band_over_l0: float = 5.0
    n_relax: int = 20
    n_relax_init: int = 500
    eps_relax: float = 1e-6
    fit_alpha: float = 0.0        # boundary-fitted arrangement (Sec. 4): 0 = original, paper example 0.03
    fit_re_over_l0: float = 5.0   # its radius r_e / l0
    body: Optional[Body] = None
    more_bodies: tuple = ()       # further bodies (distinct ids), after `body`
    nu: float = 0.0
    dt: float = 0.0
    steps: int = 1
    tol: float = 1e-8
    # boundary condition per role id for the pressure and the velocity sets
    bc_pressure: dict = field(default_factory=dict)
    bc_velocity: dict = field(default_factory=dict)
    pin_first: bool = False

    @property
    def rigid_bodies(self):
        """Every body of the case: `body` first, then `more_bodies`."""
        return ((self.body,) if self.body is not None else ()) + tuple(self.more_bodies)

    @property
    def n_cells(self):
        out = 1
        for m in self.n:
            out *= m
        return out

    def scaled(self, n, **kw):
        """Same case on a different mesh size (domain kept, l0 rescaled)."""
        length = self.n[0] * self.l0
        return replace(self, n=tuple(n), l0=length / n[0], **kw)


def c0_manufactured(n=32):
    """Unit square, n x n mesh, Dirichlet ring, Gaussian weight, one solve."""
    return Case(name=f"C0-manufactured-{n}", dim=2, n=(n, n), origin=(0.0, 0.0), l0=1.0 / n,
                periodic=(False, False), walls=True, jitter_seed=0, weight="gauss",
                bc_pressure={1: DIRICHLET}, bc_velocity={1: DIRICHLET})


def c1_taylor_green(n=512, steps=100):
    """Periodic [0, 2pi]^2 Taylor-Green vortex, nu = 0.01, dt = 0.2 l0."""
    l0 = 2 * math.pi / n
    return Case(name=f"C1-taylor-green-{n}", dim=2, n=(n, n), origin=(0.0, 0.0), l0=l0,
                periodic=(True, True), walls=False, jitter_seed=1, weight="cos2",
                nu=0.01, dt=0.2 * l0, steps=steps, pin_first=True)


def c2_oscillating_cylinder(n=1024, steps=50):
    """[-4, 4]^2, cylinder D = 1 with x(t) = 0.2 sin(2 pi t), Re = 100."""
    amp, freq, diam = 0.2, 1.0, 1.0
    u_max = 2 * math.pi * freq * amp
    l0 = 8.0 / n
    return Case(name=f"C2-oscillating-cylinder-{n}", dim=2, n=(n, n), origin=(-4.0, -4.0), l0=l0,
                periodic=(False, False), walls=True, jitter_seed=2, weight="cos2",
                body=Body(radius=0.5 * diam, motion=Oscillation((0.0, 0.0), amp, freq, 0)),
                nu=u_max * diam / 100.0, dt=(1.0 / 800.0) * (1024.0 / n), steps=steps,
                bc_pressure={1: DIRICHLET, 2: NEUMANN}, bc_velocity={1: NEUMANN, 2: DIRICHLET})


def c2_rotating_cylinder(n=256, steps=50):
    """C2 with a rotational oscillation added: posture theta(t) = 0.3 sin(2 pi t),
    so the no-slip velocity V_trans + omega x r has a tangential part of
    peak omega R = 0.94 (Eqs. velocity_moving_boundary, dvdt_moving_boundary)."""
    base = c2_oscillating_cylinder(n=n, steps=steps)
    mot = base.body.motion
    return replace(base, name=f"C2-rotating-cylinder-{n}", jitter_seed=6,
                   body=Body(radius=base.body.radius,
                             motion=Oscillation(mot.c0, mot.amplitude, mot.freq, 0, spin_amplitude=0.3,
                                                spin_freq=1.0)))


def c6_flapping_ellipse(n=512, steps=50):
    """Hovering elliptic wing (Sec. 4, flapping wing): chord 1, aspect ratio 4
    (semi-axes 0.5, 0.125), box [-10, 6]^2 (16 chords, 6 from the origin to
    the upper and right walls), stroke plane at beta = pi/3 with
    a(t) = a0/2 (1 + cos(2t/a0)), a0 = 2.5, posture theta(t) =
    pi/4 (1 - sin(2t/a0)); no slip on the wing and the walls.  Re = 100 on
    the peak translational speed 1 and the chord.  dt = pi/600 at 512^2
    (scaled with the mesh).  The wing is a discrete SDF."""
    l0 = 16.0 / n
    wing = Body(radius=0.5, motion=FlappingMotion((0.0, 0.0), 2.5, math.pi / 3, math.pi / 4),
                ellipse=(0.5, 0.125))
    return Case(name=f"C6-flapping-ellipse-{n}", dim=2, n=(n, n), origin=(-10.0, -10.0), l0=l0,
                periodic=(False, False), walls=True, jitter_seed=7, weight="cos2", body=wing,
                nu=0.01, dt=(math.pi / 600.0) * (512.0 / n), steps=steps,
                bc_pressure={1: DIRICHLET, 2: NEUMANN}, bc_velocity={1: DIRICHLET, 2: DIRICHLET})


def c2_two_cylinders(n=256, steps=50):
    """[-4, 4]^2 with two cylinders whose relaxation bands overlap: D = 1 at
    (-0.9, 0) with x(t) = 0.15 sin(2 pi t) (id 2) and D = 0.7 at (0.5, 0)
    with y(t) = 0.15 sin(2 pi t + pi/2) (id 3); the surface gap is 0.55 at
    rest and 0.4 at the closest, so on a 128^2 mesh the 5 l0 bands overlap.  Re = 100 on the first cylinder's peak speed and diameter; walls
    and bodies as in C2."""
    amp, freq, diam = 0.15, 1.0, 1.0
    u_max = 2 * math.pi * freq * amp
    base = c2_oscillating_cylinder(n=n, steps=steps)
    return replace(base, name=f"C2-two-cylinders-{n}", jitter_seed=5,
                   body=Body(radius=0.5 * diam, motion=Oscillation((-0.9, 0.0), amp, freq, 0)),
                   more_bodies=(Body(radius=0.35, motion=Oscillation((0.5, 0.0), amp, freq, 1, 0.5 * math.pi),
                                     body_id=BODY_ID + 1),),
                   nu=u_max * diam / 100.0,
                   bc_pressure={1: DIRICHLET, 2: NEUMANN, 3: NEUMANN},
                   bc_velocity={1: NEUMANN, 2: DIRICHLET, 3: DIRICHLET})


def c3_cylinder_variant(seed, n=1024, steps=120):
    """A C2-shaped trajectory for the learned-guess data set: amplitude
    A ~ U[0.1, 0.4] D and frequency f ~ U[0.5, 2] drawn from PCG64(seed),
    Re = 100 kept (nu follows the peak body speed), the DP jitter seeded by
    `seed`, and the step shortened where the body is faster than in C2 so
    that the CFL number stays that of C2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    diam = 1.0
    amp = float(rng.uniform(0.1, 0.4)) * diam
    freq = float(rng.uniform(0.5, 2.0))
    u_max = 2 * math.pi * freq * amp
    u_ref = 2 * math.pi * 1.0 * 0.2
    base = c2_oscillating_cylinder(n=n, steps=steps)
    return replace(base, name=f"C3-cylinder-{n}-seed{seed}", jitter_seed=int(seed),
                   body=Body(radius=0.5 * diam, motion=Oscillation((0.0, 0.0), amp, freq, 0)),
                   nu=u_max * diam / 100.0, dt=base.dt * min(1.0, u_ref / u_max))


def c4_moving_sphere(n=128, steps=20):
    """[0, 1]^3, sphere D = 0.25 at the centre with x(t) = 0.05 sin(2 pi t), Re = 100."""
    diam = 0.25
    amp, freq = 0.2 * diam, 1.0
    u_max = 2 * math.pi * freq * amp
    l0 = 1.0 / n
    # kappa = 1/10: with the 26 springs of the 3x3x3 block the explicit step
    # of the 2D value 1/5 is unstable (kappa * lambda_max ~ 2.5 > 2); 1/10
    # gives the 2D contraction per sweep (reading for 3D)
    return Case(name=f"C4-moving-sphere-{n}", dim=3, n=(n, n, n), origin=(0.0, 0.0, 0.0), l0=l0,
                periodic=(False, False, False), walls=True, jitter_seed=4, weight="cos2", kappa=0.1,
                body=Body(radius=0.5 * diam, motion=Oscillation((0.5, 0.5, 0.5), amp, freq, 0)),
                nu=u_max * diam / 100.0, dt=(1.0 / 200.0) * (128.0 / n), steps=steps,
                bc_pressure={1: DIRICHLET, 2: NEUMANN}, bc_velocity={1: NEUMANN, 2: DIRICHLET})


def c4_two_spinning_spheres(n=32, steps=20):
    """[0, 1]^3 with two spheres whose 5 l0 bands overlap on 32^3: R = 0.12
    at (0.3, 0.5, 0.5), x(t) = 0.03 sin(2 pi t), spinning about y with
    angle 0.4 sin(2 pi t) (id 2); R = 0.1 at (0.7, 0.5, 0.5), z(t) =
    0.03 sin(2 pi t + pi/2), spinning about (1, 1, 1)/sqrt(3) with angle
    0.6 sin(4 pi t) (id 3).  Walls and boundary conditions as in C4."""
    base = c4_moving_sphere(n=n, steps=steps)
    k = 1.0 / math.sqrt(3.0)
    a = Body(radius=0.12, motion=Oscillation((0.3, 0.5, 0.5), 0.03, 1.0, 0, spin_amplitude=0.4, spin_freq=1.0,
                                             spin_axis=(0.0, 1.0, 0.0)))
    b = Body(radius=0.1, motion=Oscillation((0.7, 0.5, 0.5), 0.03, 1.0, 2, 0.5 * math.pi, spin_amplitude=0.6,
                                            spin_freq=2.0, spin_axis=(k, k, k)), body_id=BODY_ID + 1)
    return replace(base, name=f"C4-two-spinning-spheres-{n}", jitter_seed=8, body=a, more_bodies=(b,),
                   bc_pressure={1: DIRICHLET, 2: NEUMANN, 3: NEUMANN},
                   bc_velocity={1: NEUMANN, 2: DIRICHLET, 3: DIRICHLET})


def c4_spinning_capsule(n=32, steps=20):
    """[0, 1]^3 with a capsule (half length 0.12, radius 0.06; a discrete SDF
    on a grid of spacing l0/2) at (0.5, 0.5, 0.5) + 0.03 sin(2 pi t) e_x,
    turning about the axis (0, 0.6, 0.8) with angle 0.5 + 0.4 sin(2 pi t).
    Walls and boundary conditions as in C4."""
    base = c4_moving_sphere(n=n, steps=steps)
    body = Body(radius=0.18, motion=Oscillation((0.5, 0.5, 0.5), 0.03, 1.0, 0, spin_amplitude=0.4, spin_freq=1.0,
                                                theta0=0.5, spin_axis=(0.0, 0.6, 0.8)),
                capsule=(0.12, 0.06))
    return replace(base, name=f"C4-spinning-capsule-{n}", jitter_seed=9, body=body)


def c4_sphere_variant(seed, n=128, steps=60):
    """A C4-shaped trajectory for the 3D learned-guess data set: amplitude
    A ~ U[0.1, 0.4] D and frequency f ~ U[0.5, 2] drawn from PCG64(seed), as
    for the cylinder variants, Re = 100 kept, the DP jitter seeded by `seed`
    and the step shortened where the sphere is faster than in C4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = c4_moving_sphere(n=n, steps=steps)
    diam = 2 * base.body.radius
    amp = float(rng.uniform(0.1, 0.4)) * diam
    freq = float(rng.uniform(0.5, 2.0))
    u_max = 2 * math.pi * freq * amp
    u_ref = 2 * math.pi * 1.0 * 0.2 * diam
    return replace(base, name=f"C4-sphere-{n}-seed{seed}", jitter_seed=int(seed),
                   body=Body(radius=0.5 * diam, motion=Oscillation((0.5, 0.5, 0.5), amp, freq, 0)),
                   nu=u_max * diam / 100.0, dt=base.dt * min(1.0, u_ref / u_max))
