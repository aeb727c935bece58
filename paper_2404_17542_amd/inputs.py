"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module holds *data generation only*: cell geometry of the background
mesh, seeded jitter of the discrete points (DPs), analytic fields of the test
problems (manufactured Poisson solution, Taylor-Green vortex) and prescribed
rigid-body trajectories.  None of the MCD method's arithmetic (masking,
relaxation, MLS, Krylov) lives here, so importing it does not couple the
oracle to the GPU path.

Cell ordering everywhere: c = i + n0 * (j + n1 * k) (x fastest).
Per-DP vectors are structure-of-arrays, shape (dim, Nc).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def n_cells(n) -> int:
    return int(np.prod(np.asarray(n, dtype=np.int64)))


def cell_index_grid(n):
    """Integer cell coordinates (dim, Nc), x fastest."""
    dim = len(n)
    grids = np.meshgrid(*[np.arange(m, dtype=np.int64) for m in n], indexing="ij")
    # meshgrid(ij) gives axis-0 slowest; we want x (axis 0 of n) fastest.
    out = np.empty((dim, n_cells(n)), dtype=np.int64)
    for a in range(dim):
        out[a] = np.transpose(grids[a]).reshape(-1)
    return out


def cell_centroids(n, origin, l0):
    """Centroid of every background-mesh cell, (dim, Nc) float64."""
    ijk = cell_index_grid(n)
    dim = len(n)
    out = np.empty((dim, ijk.shape[1]), dtype=np.float64)
    for a in range(dim):
        out[a] = origin[a] + (ijk[a].astype(np.float64) + 0.5) * l0
    return out


def jittered_positions(n, origin, l0, seed, amp=0.2):
    """One DP per cell at the centroid plus uniform jitter of +-amp*l0 per axis.

    numpy PCG64(seed) draws U(-amp, amp) of shape (dim, Nc) in one call.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-amp, amp, size=(len(n), n_cells(n)))
    return cell_centroids(n, origin, l0) + l0 * u


# --------------------------------------------------------------------------
# Analytic fields of the synthetic workloads
# --------------------------------------------------------------------------

def manufactured_pressure(pos):
    """p = sin(2 pi x) sin(2 pi y) on the unit square."""
    return np.sin(2 * np.pi * pos[0]) * np.sin(2 * np.pi * pos[1])


def manufactured_rhs(pos):
    """Laplacian of manufactured_pressure: -8 pi^2 sin(2 pi x) sin(2 pi y)."""
    return -8.0 * np.pi ** 2 * manufactured_pressure(pos)


def tgv_velocity(pos, t, nu):
    """2D Taylor-Green vortex on [0, 2pi]^2: (sin x cos y, -cos x sin y) e^{-2 nu t}."""
    e = math.exp(-2.0 * nu * t)
    return np.stack([np.sin(pos[0]) * np.cos(pos[1]) * e,
                     -np.cos(pos[0]) * np.sin(pos[1]) * e])


def tgv_pressure(pos, t, nu):
    """p = (cos 2x + cos 2y) e^{-4 nu t} / 4."""
    return 0.25 * (np.cos(2 * pos[0]) + np.cos(2 * pos[1])) * math.exp(-4.0 * nu * t)


# --------------------------------------------------------------------------
# Prescribed rigid-body motion (translation only)
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Oscillation:
    """Body centre c(t) = c0 + A sin(2 pi f t + phase) e_axis; velocity is its
    derivative.  Optional spin about spin_axis (z in 2D): angle theta(t) =
    theta0 + S sin(2 pi f_s t), angular velocity omega(t) = d theta / dt
    (omega_vector: omega(t) spin_axis)."""
    c0: tuple
    amplitude: float
    freq: float
    axis: int = 0
    phase: float = 0.0
    spin_amplitude: float = 0.0
    spin_freq: float = 0.0
    theta0: float = 0.0
    spin_axis: tuple = (0.0, 0.0, 1.0)    # unit axis of the spin (z in 2D)

    def theta(self, t):
        return self.theta0 + self.spin_amplitude * math.sin(2 * math.pi * self.spin_freq * t)

    def omega(self, t):
        return 2 * math.pi * self.spin_freq * self.spin_amplitude * math.cos(2 * math.pi * self.spin_freq * t)

    def omega_vector(self, t):
        w = self.omega(t)
        return tuple(w * a for a in self.spin_axis)

    def centre(self, t):
        c = list(self.c0)
        c[self.axis] = self.c0[self.axis] + self.amplitude * math.sin(2 * math.pi * self.freq * t + self.phase)
        return tuple(float(v) for v in c)

    def velocity(self, t):
        v = [0.0] * len(self.c0)
        v[self.axis] = 2 * math.pi * self.freq * self.amplitude * math.cos(2 * math.pi * self.freq * t + self.phase)
        return tuple(v)


@dataclass(frozen=True)
class FlappingMotion:
    """Hovering-wing kinematics: the rotation centre moves along a stroke
    plane of elevation beta, c(t) = c0 + a(t) (cos beta, sin beta) with
    a(t) = a0/2 (1 + cos(2t/a0)), and the posture angle is
    theta(t) = theta_offset + theta0 (1 - sin(2t/a0 + phi)) (Sec. 4, flapping
    wing); velocity and omega are the time derivatives."""
    c0: tuple
    a0: float
    beta: float
    theta0: float
    phi: float = 0.0
    theta_offset: float = 0.0

    def centre(self, t):
        a = 0.5 * self.a0 * (1.0 + math.cos(2.0 * t / self.a0))
        return (self.c0[0] + a * math.cos(self.beta), self.c0[1] + a * math.sin(self.beta))

    def velocity(self, t):
        da = -math.sin(2.0 * t / self.a0)
        return (da * math.cos(self.beta), da * math.sin(self.beta))

    def theta(self, t):
        return self.theta_offset + self.theta0 * (1.0 - math.sin(2.0 * t / self.a0 + self.phi))

    def omega(self, t):
        return -self.theta0 * (2.0 / self.a0) * math.cos(2.0 * t / self.a0 + self.phi)

    def omega_vector(self, t):
        return (0.0, 0.0, self.omega(t))


def ellipse_distance(semi_a, semi_b, x, y):
    """Signed distance (> 0 outside) from points (x, y) to the ellipse
    x^2/a^2 + y^2/b^2 = 1, by Eberly's bisection on the closest-point
    parameter ("Distance from a Point to an Ellipse, an Ellipsoid, or a
    Hyperellipsoid", Geometric Tools), vectorised; a >= b."""
    assert semi_a >= semi_b > 0
    y0 = np.abs(np.asarray(x, dtype=np.float64))
    y1 = np.abs(np.asarray(y, dtype=np.float64))
    e0, e1 = float(semi_a), float(semi_b)
    z0, z1 = y0 / e0, y1 / e1
    g = z0 * z0 + z1 * z1 - 1.0
    r0 = (e0 / e1) ** 2
    # generic case y0 > 0, y1 > 0: root s of (r0 z0/(s + r0))^2 + (z1/(s + 1))^2 = 1
    n0 = r0 * z0
    lo = z1 - 1.0
    hi = np.where(g < 0, 0.0, np.sqrt(n0 * n0 + z1 * z1) - 1.0)
    for _ in range(160):
        sm = 0.5 * (lo + hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            gm = (n0 / (sm + r0)) ** 2 + (z1 / (sm + 1.0)) ** 2 - 1.0
        lo = np.where(gm > 0, sm, lo)
        hi = np.where(gm > 0, hi, sm)
    sbar = 0.5 * (lo + hi)
    with np.errstate(divide="ignore", invalid="ignore"):
        x0 = r0 * y0 / (sbar + r0)
        x1 = y1 / (sbar + 1.0)
    d_gen = np.sqrt((x0 - y0) ** 2 + (x1 - y1) ** 2)
    # y1 = 0: on the major axis
    num, den = e0 * y0, e0 * e0 - e1 * e1
    xde = np.minimum(num / den, 1.0)
    d_axis = np.where(num < den, np.sqrt((e0 * xde - y0) ** 2 + (e1 * np.sqrt(1.0 - xde * xde)) ** 2),
                      np.abs(y0 - e0))
    # y0 = 0, y1 > 0: on the minor axis
    d_minor = np.abs(y1 - e1)
    d = np.where(y1 > 0, np.where(y0 > 0, d_gen, d_minor), d_axis)
    d = np.where((y1 > 0) & (y0 > 0) & (g == 0), 0.0, d)
    return np.where(g < 0, -d, d)


def ellipse_sdf_grid(semi_a, semi_b, h, half_extent):
    """Discrete SDF of an ellipse centred at the origin of its frame, major
    axis along x: nodes -L + (i, j) h with L = half_extent rounded up to a
    multiple of h plus one node; returns (values [ny][nx], origin, h)."""
    m = int(math.ceil(half_extent / h)) + 1
    ax = -m * h + h * np.arange(2 * m + 1)
    X, Y = np.meshgrid(ax, ax)
    return ellipse_distance(semi_a, semi_b, X, Y), (-m * h, -m * h), h


def capsule_sdf_grid(half_length, radius, h, half_extent):
    """Discrete SDF of a capsule (the points within `radius` of the segment
    from (-half_length, 0, 0) to (half_length, 0, 0)) in its own frame: the
    exact distance |p - clamp(p_x, -L, L) e_x| - radius at the nodes
    -M h + (i, j, k) h, M = ceil(half_extent / h) + 1; returns
    (values [nz][ny][nx], origin, h)."""
    m = int(math.ceil(half_extent / h)) + 1
    ax = -m * h + h * np.arange(2 * m + 1)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    cx = np.clip(X, -half_length, half_length)
    vals = np.sqrt((X - cx) ** 2 + Y ** 2 + Z ** 2) - radius
    return vals, (-m * h, -m * h, -m * h), h


def he_normal_params(shapes, seed, taps=9):
    """Seeded initial network parameters: for each (cin, cout) convolution of
    `taps` taps (9 in 2D, 27 in 3D), weights N(0, 2 / (taps cin)) of shape
    [taps][cin][cout] then zero biases (flat FP32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for cin, cout in shapes:
        parts.append(rng.standard_normal(taps * cin * cout) * np.sqrt(2.0 / (taps * cin)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def random_unet_batch(rng_seed, shape, dtype=np.float32):
    """Seeded normal tensor for network tests (no method arithmetic)."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    return rng.standard_normal(shape).astype(dtype)
