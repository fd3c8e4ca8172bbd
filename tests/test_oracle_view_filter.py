"""Pins of the oracle's view filter (Sec. III-A, Eq. 1): the triangulation
angle at sparse points seen by two keyframes, accepted when at least 20% of
the points lie within [6, 60] degrees. Closed forms: a point on the
perpendicular bisector of the baseline b at distance D from its midpoint
sees the baseline under 2 atan(b / 2D); points on the baseline's line
outside the segment see 0 degrees, inside it 180; the fraction rule is
checked on mixtures with a known count, including the boundary fraction and
the closed angle interval."""
import math

import numpy as np
import pytest

import oracle


def _bisector_point(ca, cb, D, rng):
    ca, cb = np.asarray(ca, float), np.asarray(cb, float)
    mid = 0.5 * (ca + cb)
    u = (cb - ca) / np.linalg.norm(cb - ca)
    v = rng.normal(size=3)
    v -= u * (u @ v)
    v /= np.linalg.norm(v)
    return mid + D * v


def test_bisector_angles_are_exact():
    rng = np.random.default_rng(0)
    ca, cb = [0.0, 0.0, 0.0], [1.0, 0.2, -0.3]
    b = np.linalg.norm(np.subtract(cb, ca))
    for deg in [1.0, 5.9, 6.1, 30.0, 59.9, 60.1, 120.0]:
        D = b / 2 / math.tan(math.radians(deg) / 2)
        p = _bisector_point(ca, cb, D, rng)
        acc, k, c = oracle.view_filter(ca, cb, [p], min_frac=1.0)
        assert c == 1
        assert k == (1 if 6.0 <= deg <= 60.0 else 0), deg
        assert acc == (k == 1)


def test_points_on_the_baseline_line():
    ca, cb = np.array([0.0, 0.0, 0.0]), np.array([2.0, 0.0, 0.0])
    outside = [ca - [1.0, 0, 0], cb + [3.0, 0, 0]]   # 0 degrees
    inside = [np.array([0.5, 0.0, 0.0])]            # 180 degrees
    at_centre = [ca.copy()]                         # no angle
    _, k, c = oracle.view_filter(ca, cb, outside + inside + at_centre, min_deg=0.0, max_deg=0.0)
    assert (k, c) == (2, 3)
    _, k, c = oracle.view_filter(ca, cb, inside, min_deg=180.0, max_deg=180.0)
    assert (k, c) == (1, 1)


@pytest.mark.parametrize("n_good,n_bad,accepted", [(20, 80, True), (19, 81, False), (0, 10, False),
                                                    (5, 0, True)])
def test_fraction_rule(n_good, n_bad, accepted):
    rng = np.random.default_rng(n_good * 7 + n_bad)
    ca, cb = [0.0, 0.0, 0.0], [0.0, 0.0, 1.0]
    pts = []
    for i in range(n_good):
        deg = rng.uniform(7.0, 59.0)
        pts.append(_bisector_point(ca, cb, 0.5 / math.tan(math.radians(deg) / 2), rng))
    for i in range(n_bad):
        deg = rng.uniform(0.5, 5.0) if i % 2 else rng.uniform(61.0, 170.0)
        pts.append(_bisector_point(ca, cb, 0.5 / math.tan(math.radians(deg) / 2), rng))
    acc, k, c = oracle.view_filter(ca, cb, pts)
    assert (k, c) == (n_good, n_good + n_bad)
    assert acc == accepted


def test_no_points_rejects():
    acc, k, c = oracle.view_filter([0, 0, 0], [1, 0, 0], np.zeros((0, 3)))
    assert (acc, k, c) == (False, 0, 0)
