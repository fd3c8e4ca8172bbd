"""Pins of the oracle's dense point-cloud fusion (Sec. III: four consistent
keyframes are buffered and duplicate points erased) and of its completeness
measure (coverage of a 720x360 panorama), against facts the oracle does not
compute itself: a map fused with itself keeps only the first copy; every
keep decision on rendered maps equals a brute force with numpy's unique over
voxel keys of points lifted independently; one huge voxel per octant keeps
exactly one point; coverage of a dense shell of points around the camera is complete,
of a half shell half."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import bearings


def _lift(d, pose):
    R, t = pose
    R = np.asarray(R, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    H, W = d.shape
    X = bearings(W, H) * d[None]
    return np.einsum("ji,jhw->ihw", R, X - t[:, None, None])


def _brute_keep(depths, poses, voxel):
    keys, order = [], []
    HW = depths[0].size
    for m, (d, pose) in enumerate(zip(depths, poses)):
        X = _lift(d, pose).reshape(3, -1)
        valid = d.ravel() > 0
        v = np.floor(X[:, valid] / voxel).astype(np.int64).T
        keys.append(v)
        order.append(m * HW + np.nonzero(valid)[0])
    keys = np.concatenate(keys)
    order = np.concatenate(order)
    srt = np.argsort(order)
    _, first = np.unique(keys[srt], axis=0, return_index=True)
    keep = np.zeros(len(depths) * HW, dtype=np.uint8)
    keep[order[srt][first]] = 1
    return keep.reshape(len(depths), *depths[0].shape)


@pytest.fixture(scope="module")
def hall():
    return synth.scaled("hall", 96, seed=0)


def test_self_fusion_keeps_the_first_copy(hall):
    d = hall.gt_depth[2].astype(np.float64)
    p = hall.poses[2]
    keep, n = oracle.fuse([d, d], [p, p], 0.05)
    assert n == keep.sum() and n > 100
    assert keep[1].sum() == 0
    assert np.array_equal(keep[0], _brute_keep([d], [p], 0.05)[0])


@pytest.mark.parametrize("voxel", [0.02, 0.1, 0.5])
def test_keep_masks_match_brute_force(hall, voxel):
    depths = [hall.gt_depth[k].astype(np.float64) for k in range(4)]
    poses = [hall.poses[k] for k in range(4)]
    keep, n = oracle.fuse(depths, poses, voxel)
    exp = _brute_keep(depths, poses, voxel)
    assert np.array_equal(keep, exp)
    assert n == exp.sum()


def test_huge_voxels_keep_one_point_per_octant(hall):
    # with a 1e6 m voxel a point's voxel is just the signs of its coordinates
    depths = [hall.gt_depth[k].astype(np.float64) for k in range(3)]
    poses = [hall.poses[k] for k in range(3)]
    keep, n = oracle.fuse(depths, poses, 1e6)
    seen = {}
    for m in range(3):
        X = _lift(depths[m], poses[m]).reshape(3, -1)
        for i in np.flatnonzero(depths[m].ravel() > 0):
            seen.setdefault(tuple(X[:, i] < 0), (m, i))
    assert n == len(seen) and 1 <= n <= 8
    for m, i in seen.values():
        assert keep[m].ravel()[i] == 1


def _shell(W, H, upper_only=False, r=3.0):
    """A camera at the origin and a map of a sphere of radius r around it."""
    d = np.full((H, W), r)
    if upper_only:
        d[H // 2:] = 0.0
    return d, (np.eye(3), np.zeros(3))


def test_coverage_of_shells():
    W, H = 1440, 720
    d, pose = _shell(W, H)
    c, cover = oracle.coverage([d], [pose], None, pose, 720, 360)
    assert c == 720 * 360
    d, pose = _shell(W, H, upper_only=True)
    c, cover = oracle.coverage([d], [pose], None, pose, 720, 360)
    assert c == 720 * 180
    assert cover[:180].all() and not cover[180:].any()
