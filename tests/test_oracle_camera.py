"""Pins of the oracle's equirectangular camera model and sampler.

Closed forms: special directions (forward, right, left, back, poles), unit
bearings, project(unproject(x)) == x, and bilinear sampling against torch's
grid_sample on an independently wrap-padded copy of the image.
"""
import math

import numpy as np
import pytest
import torch

import oracle

W, H = 64, 32


def test_special_directions():
    # the image centre looks along +z
    assert np.allclose(oracle.unproject(W, H, W / 2 - 0.5, H / 2 - 0.5), [0, 0, 1], atol=1e-15)
    # a quarter turn to the right is +x, to the left -x
    assert np.allclose(oracle.unproject(W, H, 3 * W / 4 - 0.5, H / 2 - 0.5), [1, 0, 0], atol=1e-15)
    assert np.allclose(oracle.unproject(W, H, W / 4 - 0.5, H / 2 - 0.5), [-1, 0, 0], atol=1e-15)
    # the left edge of the first column looks backwards
    assert np.allclose(oracle.unproject(W, H, -0.5, H / 2 - 0.5), [0, 0, -1], atol=1e-15)
    # the top edge is the north pole (up is -y), the bottom edge the south pole
    assert np.allclose(oracle.unproject(W, H, 5.0, -0.5), [0, -1, 0], atol=1e-15)
    assert np.allclose(oracle.unproject(W, H, 5.0, H - 0.5), [0, 1, 0], atol=1e-15)
    # 45 degrees up, straight ahead
    b = oracle.unproject(W, H, W / 2 - 0.5, H / 4 - 0.5)
    assert np.allclose(b, [0, -math.sqrt(0.5), math.sqrt(0.5)], atol=1e-15)


def test_project_special_directions():
    assert np.allclose(oracle.project(W, H, [0, 0, 5]), (W / 2 - 0.5, H / 2 - 0.5), atol=1e-12)
    assert np.allclose(oracle.project(W, H, [2, 0, 0]), (3 * W / 4 - 0.5, H / 2 - 0.5), atol=1e-12)
    assert np.allclose(oracle.project(W, H, [0, -3, 0])[1], -0.5, atol=1e-12)
    assert np.allclose(oracle.project(W, H, [0, 3, 0])[1], H - 0.5, atol=1e-12)
    # scale invariance
    Y = np.array([0.3, -0.2, 0.7])
    assert np.allclose(oracle.project(W, H, Y), oracle.project(W, H, 7.5 * Y), atol=1e-12)


def test_bearings_are_unit_and_round_trip():
    rng = np.random.default_rng(1)
    pts = [(x, y) for y in range(H) for x in range(W)]
    pts += [(rng.uniform(-0.49, W - 0.51), rng.uniform(-0.49, H - 0.51)) for _ in range(2000)]
    for x, y in pts:
        b = oracle.unproject(W, H, x, y)
        assert abs(np.linalg.norm(b) - 1.0) < 1e-14
        u, v = oracle.project(W, H, b)
        assert abs(u - x) < 1e-9 and abs(v - y) < 1e-9


def test_bearing_matches_spherical_angles():
    # independent statement: the angle between two bearings is the great-circle
    # distance of their (lon, lat)
    rng = np.random.default_rng(2)
    for _ in range(500):
        x1, x2 = rng.uniform(0, W, 2)
        y1, y2 = rng.uniform(0, H - 1, 2)
        lon1, lon2 = 2 * math.pi * (x1 + 0.5) / W, 2 * math.pi * (x2 + 0.5) / W
        lat1, lat2 = math.pi / 2 - math.pi * (y1 + 0.5) / H, math.pi / 2 - math.pi * (y2 + 0.5) / H
        hav = math.sin((lat2 - lat1) / 2) ** 2 + math.cos(lat1) * math.cos(lat2) * math.sin((lon2 - lon1) / 2) ** 2
        ang = 2 * math.asin(min(1.0, math.sqrt(hav)))
        b1 = oracle.unproject(W, H, x1, y1)
        b2 = oracle.unproject(W, H, x2, y2)
        assert abs(math.atan2(np.linalg.norm(np.cross(b1, b2)), np.dot(b1, b2)) - ang) < 1e-12


def _grid_sample_wrapped(img, xs, ys):
    Hh, Ww = img.shape
    padded = np.concatenate([img[:, -1:], img, img[:, :1]], axis=1)  # one column each side
    t = torch.from_numpy(padded)[None, None]
    gx = (2.0 * (np.asarray(xs) + 1.0) + 1.0) / (Ww + 2) - 1.0
    gy = (2.0 * np.asarray(ys) + 1.0) / Hh - 1.0
    grid = torch.from_numpy(np.stack([gx, gy], axis=-1))[None, None]
    out = torch.nn.functional.grid_sample(t, grid, mode="bilinear", padding_mode="border",
                                          align_corners=False)
    return out[0, 0, 0].numpy()


def test_bilinear_matches_grid_sample_with_wrap():
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (H, W))
    xs = rng.uniform(-0.5, W - 0.5, 3000)
    ys = rng.uniform(-0.5, H - 0.5, 3000)
    # include the seam, the poles and exact pixel centres
    xs = np.concatenate([xs, [-0.5, W - 0.5, W - 0.75, -0.25, 0.0, 5.0]])
    ys = np.concatenate([ys, [3.0, 7.5, -0.5, H - 0.5, 0.0, H - 1.0]])
    ref = _grid_sample_wrapped(img, xs, ys)
    got = np.array([oracle.sample(img, x, y) for x, y in zip(xs, ys)])
    assert np.max(np.abs(got - ref)) < 1e-13


def test_sample_seam_and_centres():
    rng = np.random.default_rng(4)
    img = rng.uniform(0, 1, (H, W))
    # halfway across the seam is the mean of the last and first column
    assert oracle.sample(img, W - 0.5, 6.0) == pytest.approx(0.5 * (img[6, -1] + img[6, 0]), abs=1e-15)
    assert oracle.sample(img, -0.5, 6.0) == pytest.approx(0.5 * (img[6, -1] + img[6, 0]), abs=1e-15)
    # pixel centres return the pixel
    for x, y in [(0, 0), (W - 1, H - 1), (13, 7)]:
        assert oracle.sample(img, x, y) == img[y, x]
