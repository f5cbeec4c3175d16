"""The base pass queues the points within kFrontRadius (in M) of the screen
centre first, on the ground that every Kerr critical curve lies there: the
screen radius of the critical curve (spherical photon orbits mapped to a
distant observer's screen, Bardeen's relations) stays below it for every spin
and inclination, with room for the photon ring around it."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def front_radius():
    src = open(os.path.join(ROOT, "paper_2103_07417_amd", "csrc", "art_kernels.hip")).read()
    return float(re.search(r"constexpr double kFrontRadius = ([0-9.]+);", src).group(1))


def critical_curve_radii(a, inc_deg, n=20001):
    """Screen radii sqrt(alpha^2 + beta^2) of the critical curve (M = 1)."""
    if abs(a) < 1e-12:
        return np.array([math.sqrt(27.0)])
    aa = abs(a)
    r_pro = 2.0 * (1.0 + math.cos(2.0 / 3.0 * math.acos(-aa)))
    r_ret = 2.0 * (1.0 + math.cos(2.0 / 3.0 * math.acos(aa)))
    r = np.linspace(r_pro, r_ret, n)
    xi = -(r ** 3 - 3.0 * r ** 2 + a * a * r + a * a) / (a * (r - 1.0))
    eta = r ** 3 * (4.0 * a * a - r * (r - 3.0) ** 2) / (a * a * (r - 1.0) ** 2)
    th = math.radians(inc_deg)
    alpha = -xi / math.sin(th)
    b2 = eta + a * a * math.cos(th) ** 2 - xi ** 2 / math.tan(th) ** 2
    ok = b2 >= 0.0
    return np.sqrt(alpha[ok] ** 2 + b2[ok])


def test_schwarzschild_shadow_radius():
    # a -> 0 limit of the relations: the circle of radius sqrt(27) M
    rr = critical_curve_radii(1e-4, 60.0)
    assert abs(rr.min() - math.sqrt(27.0)) < 1e-3 and abs(rr.max() - math.sqrt(27.0)) < 1e-3


@pytest.mark.parametrize("a", [0.0, 0.5, -0.5, 0.94, -0.94, 0.998, -0.998])
@pytest.mark.parametrize("inc", [17.0, 60.0, 90.0, 163.0])
def test_critical_curve_within_front_radius(a, inc):
    rr = critical_curve_radii(a, inc)
    assert rr.size > 0
    # the photon ring sits within a few tenths of M of the curve
    assert rr.max() + 0.5 < front_radius(), (a, inc, rr.max())
    assert rr.min() > 2.0
