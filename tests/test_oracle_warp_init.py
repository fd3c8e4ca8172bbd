"""Pins of the oracle's plane-map warping (Sec. III-B: the optimised plane
map of the preceding keyframe initialises the current one), checked against
facts the oracle does not compute itself:

* identical poses return the map unchanged;
* a yaw by a whole number of pixels is an exact column shift (longitude
  lam -> lam + alpha under a rotation about the vertical), with the normal
  rotated;
* planes of an analytic world plane arrive with the depth and normal a ray
  cast from the destination camera gives;
* where a nearer plane covers a wall in the destination view, the nearer
  plane wins (the z-buffer), and the wall elsewhere;
* a plane seen from behind by the destination camera yields nothing;
* warped ground-truth planes as the initialisation reach a given accuracy in
  fewer iterations than the random initialisation (the purpose of the step).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import bearings

PARAMS = dict(synth.BASE_PARAMS, patch_size=5, patch_stride=1, depth_min=0.1, depth_max=50.0)


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _pose(R, centre):
    R = np.asarray(R, dtype=np.float64)
    return R, -R @ np.asarray(centre, dtype=np.float64)


def _plane_map(W, H, pose, planes):
    """Ray-cast depth and camera-frame normal (facing the camera) of the
    nearest of `planes` = [(m, e, bounds)] with world plane m.X = e and
    optional bounds (lo, hi) on the world coordinates of the hit."""
    R, t = pose
    c = -R.T @ t
    b = bearings(W, H).reshape(3, -1)
    w = R.T @ b
    depth = np.full(W * H, np.inf)
    normal = np.zeros((3, W * H))
    for m, e, bounds in planes:
        m = np.asarray(m, dtype=np.float64)
        den = m @ w
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (e - m @ c) / den
        hit = np.isfinite(s) & (s > 0)
        if bounds is not None:
            P = c[:, None] + s[None, :] * w
            lo, hi = bounds
            hit &= np.all((P >= np.asarray(lo)[:, None]) & (P <= np.asarray(hi)[:, None]), axis=0)
        nearer = hit & (s < depth)
        depth[nearer] = s[nearer]
        n_cam = R @ m
        # facing the camera: n . b < 0
        sign = np.where((n_cam @ b) < 0, 1.0, -1.0)
        normal[:, nearer] = (n_cam[:, None] * sign[None, :])[:, nearer]
    depth[~np.isfinite(depth)] = 0.0
    return depth.reshape(H, W), normal.reshape(3, H, W)


def _band(H):
    r = (PARAMS["patch_size"] - 1) // 2
    m = np.zeros(H, dtype=bool)
    m[r:H - r] = True
    return m


def test_identity_pose_returns_the_map():
    W, H = 48, 24
    pose = _pose(_rot_y(0.3), [0.2, -1.0, 0.1])
    d, n = _plane_map(W, H, pose, [([0.0, 0.0, 1.0], 3.0, None), ([1.0, 0.0, 0.0], -2.5, None),
                                   ([0.0, 1.0, 0.0], 0.5, None)])
    dd, dn = oracle.warp_planes(d, n, pose, pose, PARAMS)
    band = _band(H)
    ok = (d[band] >= PARAMS["depth_min"]) & (d[band] <= PARAMS["depth_max"])
    assert ok.mean() > 0.5
    np.testing.assert_allclose(dd[band][ok], d[band][ok], rtol=1e-12)
    np.testing.assert_allclose(dn[:, band][:, ok], n[:, band][:, ok], atol=1e-12)
    # out of the depth range or outside the band: nothing
    assert np.all(dd[band][~ok] == 0) and np.all(dd[~band] == 0)


def test_yaw_by_whole_pixels_is_an_exact_shift():
    W, H = 64, 32
    k = 5
    alpha = 2 * math.pi * k / W
    src = _pose(np.eye(3), [0.0, 0.0, 0.0])
    dst = _pose(_rot_y(alpha), [0.0, 0.0, 0.0])
    rng = np.random.default_rng(0)
    d = rng.uniform(1.0, 10.0, (H, W))
    # normals facing the camera: the negated bearing, tilted a little
    b = bearings(W, H)
    n = -b + 0.2 * rng.normal(size=(3, H, W))
    n /= np.linalg.norm(n, axis=0)
    dd, dn = oracle.warp_planes(d, n, src, dst, PARAMS)
    band = _band(H)
    # longitude lam -> lam + alpha: column x -> x + k
    exp_d = np.roll(d, k, axis=1)
    exp_n = np.einsum("ij,jhw->ihw", _rot_y(alpha), np.roll(n, k, axis=2))
    np.testing.assert_allclose(dd[band], exp_d[band], rtol=1e-9)
    np.testing.assert_allclose(dn[:, band], exp_n[:, band], atol=1e-9)


def test_analytic_plane_arrives_exactly():
    W, H = 96, 48
    plane = ([0.3, -0.2, 1.0], 4.0, None)
    m = np.array(plane[0])
    plane = (m / np.linalg.norm(m), 4.0 / np.linalg.norm(m), None)
    A = _pose(_rot_y(0.1), [0.0, -1.2, 0.0])
    B = _pose(_rot_y(-0.25), [0.35, -1.1, 0.2])
    dA, nA = _plane_map(W, H, A, [plane])
    dB, nB = _plane_map(W, H, B, [plane])
    dd, dn = oracle.warp_planes(dA, nA, A, B, PARAMS)
    got = dd > 0
    assert np.all(dB[got] > 0)
    np.testing.assert_allclose(dd[got], dB[got], rtol=1e-9)
    np.testing.assert_allclose(dn[:, got], nB[:, got], atol=1e-9)
    band = _band(H)[:, None] & (dB > PARAMS["depth_min"]) & (dB < PARAMS["depth_max"])
    # a forward splat leaves a few holes where the view magnifies
    assert got[band].mean() > 0.75


@pytest.mark.parametrize("side", [1.0, -1.0])
def test_nearer_plane_wins_in_the_destination(side):
    # moving either way puts the hidden wall points after, then before, the
    # nearer plane in source pixel order; the baseline makes the strip of
    # wall that A sees beside the square and B sees behind it ~8 px wide
    W, H = 256, 128
    wall = ([0.0, 0.0, 1.0], 6.0, None)
    # a square 2 m in front of the wall
    patch = ([0.0, 0.0, 1.0], 3.0, ([-1.0, -2.5, 2.9], [1.0, -0.5, 3.1]))
    A = _pose(np.eye(3), [0.0, -1.5, 0.0])
    B = _pose(np.eye(3), [1.2 * side, -1.5, 0.2])
    dA, nA = _plane_map(W, H, A, [wall, patch])
    dB, nB = _plane_map(W, H, B, [wall, patch])
    dd, dn = oracle.warp_planes(dA, nA, A, B, PARAMS)
    # compare away from silhouettes: pixels whose 5x5 neighbourhood in B
    # sees one surface (the world z of the ray-cast hit names it)
    bB = bearings(W, H)
    RB, tB = B
    cB = -RB.T @ tB
    P = cB[:, None, None] + dB[None] * np.einsum("ji,jhw->ihw", RB, bB)
    near = np.abs(P[2] - 3.0) < 1e-6
    far = np.abs(P[2] - 6.0) < 1e-6
    from scipy.ndimage import binary_erosion
    inner_near = binary_erosion(near, np.ones((5, 5)))
    inner_far = binary_erosion(far, np.ones((5, 5)))
    got = dd > 0
    assert inner_near.sum() > 50 and inner_far.sum() > 500
    m = inner_near & got
    assert m.sum() > 0.7 * inner_near.sum()
    np.testing.assert_allclose(dd[m], dB[m], rtol=1e-9)
    m = inner_far & got
    assert m.sum() > 0.7 * inner_far.sum()
    np.testing.assert_allclose(dd[m], dB[m], rtol=1e-9)


def test_plane_seen_from_behind_yields_nothing():
    W, H = 64, 32
    plane = ([1.0, 0.0, 0.0], 1.0, None)  # x = 1
    A = _pose(np.eye(3), [0.0, -1.0, 0.0])
    B = _pose(np.eye(3), [2.0, -1.0, 0.0])  # the other side
    dA, nA = _plane_map(W, H, A, [plane])
    assert (dA > 0).mean() > 0.3
    dd, dn = oracle.warp_planes(dA, nA, A, B, PARAMS)
    assert np.all(dd == 0) and np.all(dn == 0)


def test_warped_initialisation_converges_faster():
    w = synth.scaled("hall", 192, seed=0)
    params = dict(w.params, iterations=1)
    imgs = [a.astype(np.float64) for a in w.images_f32()]
    ref, prev = w.ref, w.ref - 1
    nb = [imgs[i] for i in w.nbrs]
    nps = [w.poses[i] for i in w.nbrs]
    src_d = w.gt_depth[prev].astype(np.float64)
    src_n = w.gt_normal[prev].astype(np.float64)
    # rendered normals face the camera that saw them
    b = bearings(w.W, w.H)
    flip = (src_n * b).sum(0) > 0
    src_n[:, flip] *= -1
    wd, wn = oracle.warp_planes(src_d, src_n, w.poses[prev], w.poses[ref], params)
    assert (wd > 0).mean() > 0.5
    gt = w.gt_depth[ref].astype(np.float64)

    def acc(d):
        v = (d > 0) & (gt > 0)
        return float((np.abs(d[v] - gt[v]) <= 0.01 * gt[v]).sum() / max(v.sum(), 1))

    d0, _, _ = oracle.densify(imgs[ref], nb, w.poses[ref], nps, params)
    d1, _, _ = oracle.densify(imgs[ref], nb, w.poses[ref], nps, params, init_depth=wd, init_normal=wn)
    print(f"within 1% of ground truth after 1 iteration: random {acc(d0):.3f}, warped {acc(d1):.3f}")
    assert acc(d1) > acc(d0) + 0.1
