"""Pins of the oracle's median post-filter (Sec. III-C, item 2: a depth
whose distance from the median of its window exceeds a threshold is dropped
from the map), against facts the oracle
does not compute itself: flat maps survive, an isolated outlier goes and its
neighbours stay, the decision at every pixel of random maps equals a brute
force with numpy's sort over the wrapped window, the window wraps across the
seam, and the threshold is inclusive."""
import numpy as np
import pytest

import oracle

P = dict(median_radius=2, median_rel=0.05, patch_size=3, patch_stride=1)


def _maps(d):
    H, W = d.shape
    n = np.zeros((3, H, W))
    n[2] = np.where(d > 0, -1.0, 0.0)
    c = np.where(d > 0, 0.5, 2.0)
    return n, c


def test_flat_map_is_unchanged():
    d = np.full((16, 32), 3.0)
    n, c = _maps(d)
    d2, n2, c2 = oracle.median_filter(d, n, c, P)
    assert np.array_equal(d2, d) and np.array_equal(n2, n) and np.array_equal(c2, c)


def test_isolated_outlier_is_removed_alone():
    d = np.full((16, 32), 3.0)
    d[8, 10] = 3.5
    n, c = _maps(d)
    d2, n2, c2 = oracle.median_filter(d, n, c, P)
    assert d2[8, 10] == 0 and c2[8, 10] == 2.0 and np.all(n2[:, 8, 10] == 0)
    keep = np.ones_like(d, dtype=bool)
    keep[8, 10] = False
    assert np.array_equal(d2[keep], d[keep])


def _brute(d, R, rel):
    H, W = d.shape
    drop = np.zeros_like(d, dtype=bool)
    for y in range(H):
        for x in range(W):
            if not d[y, x] > 0:
                continue
            rows = [yy for yy in range(y - R, y + R + 1) if 0 <= yy < H]
            cols = [(x + dx) % W for dx in range(-R, R + 1)]
            win = d[np.ix_(rows, cols)].ravel()
            win = np.sort(win[win > 0])
            m = win[(len(win) - 1) // 2]
            drop[y, x] = abs(d[y, x] - m) > rel * m
    return drop


@pytest.mark.parametrize("seed,R", [(0, 2), (1, 1), (2, 3)])
def test_random_maps_match_brute_force(seed, R):
    rng = np.random.default_rng(seed)
    H, W = 12, 24
    d = rng.uniform(2.0, 2.4, (H, W))
    d[rng.uniform(size=(H, W)) < 0.2] = 0.0       # holes
    d[rng.uniform(size=(H, W)) < 0.05] *= 1.5      # outliers
    n, c = _maps(d)
    params = dict(P, median_radius=R)
    d2, _, c2 = oracle.median_filter(d, n, c, params)
    drop = _brute(d, R, 0.05)
    assert drop.sum() > 3
    assert np.array_equal(d2 == 0, (d == 0) | drop)
    assert np.array_equal(d2[~drop], d[~drop])


def test_window_wraps_across_the_seam():
    d = np.full((10, 20), 4.0)
    d[:, 18:] = 9.0   # a strip at the right edge ...
    d[:, :2] = 9.0    # ... continued at the left edge: 4 columns wide across the seam
    n, c = _maps(d)
    d2, _, _ = oracle.median_filter(d, n, c, P)
    # with the wrap the strip's columns see 2-3 strip columns of 5: no drop
    # at the inner strip columns x = 19 and x = 0
    assert np.all(d2[2:8, 19] == 9.0) and np.all(d2[2:8, 0] == 9.0)


def test_threshold_is_inclusive():
    d = np.full((9, 18), 100.0)
    d[4, 4] = 105.0    # exactly 5% above the median: kept
    d[4, 12] = 105.5   # 5.5%: removed
    n, c = _maps(d)
    d2, _, _ = oracle.median_filter(d, n, c, P)
    assert d2[4, 4] == 105.0 and d2[4, 12] == 0.0


def test_radius_zero_is_off():
    d = np.random.default_rng(3).uniform(1, 5, (8, 16))
    n, c = _maps(d)
    d2, _, _ = oracle.median_filter(d, n, c, dict(P, median_radius=0))
    assert np.array_equal(d2, d)
