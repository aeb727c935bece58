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
