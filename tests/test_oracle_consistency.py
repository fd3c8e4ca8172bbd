"""More pins of the oracle's geometric-consistency step (Sec. III: once five
depth maps exist, depths that disagree with the other keyframes' maps are
removed), each fixed by geometry rather than by the oracle's own formulas:

* the relative range error is relative: a map 0.4% too far gives exactly
  that error at every pixel of a camera-centred sphere, whatever its radius;
* turning every camera half a turn about its vertical axis moves each
  image by W/2 columns and changes nothing else, so the reprojection error
  and the keep decision of every pixel move with it: the half of the image
  that crosses the seam in one frame lies away from it in the other (this
  pins the seam's handling, which would otherwise see errors of ~W pixels
  for reprojections that wrap)."""
import math

import numpy as np

import oracle
import synth


def _bearings(W, H):
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    lam = 2 * np.pi * x / W - np.pi
    phi = np.pi / 2 - np.pi * y / H
    L, P = np.meshgrid(lam, phi)
    return np.stack([np.cos(P) * np.sin(L), -np.sin(P), np.cos(P) * np.cos(L)])


def test_range_error_is_relative():
    W, H = 96, 48
    params = synth.params_for("box_room", geo_px=1.0, geo_rel_depth=0.005)
    ref_pose = synth.camera_pose([0, 0, 0], 0.0)
    nbr_pose = synth.camera_pose([0, 0, 0], 2 * math.pi * 3.0 / W)  # whole pixels: no lookup error
    for radius in (0.7, 2.5, 9.0):
        depth = np.full((H, W), radius)
        normal = -_bearings(W, H)
        cost = np.zeros((H, W))
        d, _, _, epx, ed, _ = oracle.consistency(depth, normal, cost, ref_pose, [1.004 * depth],
                                                 [nbr_pose], params, diagnostics=True)
        r = 3
        assert np.allclose(ed[0, r:H - r], 0.004, rtol=1e-9)
        assert np.allclose(epx[0, r:H - r], 0.0, atol=1e-9)
        assert np.all(d[r:H - r] == radius)  # 0.4% <= 0.5%
        d2, *_ = oracle.consistency(depth, normal, cost, ref_pose, [1.004 * depth], [nbr_pose],
                                    dict(params, geo_rel_depth=0.003))
        assert np.all(d2 == 0)  # 0.4% > 0.3%


def _half_turn(pose):
    """The camera turned by pi about its own vertical axis: camera coordinates
    (x, y, z) -> (-x, y, -z), exactly."""
    R, t = (np.asarray(a, dtype=np.float64) for a in pose)
    T = np.diag([-1.0, 1.0, -1.0])
    return T @ R, T @ t


def test_half_turn_of_every_camera_moves_errors_with_the_image(box_room):
    w = box_room
    W, H = w.W, w.H
    params = dict(w.params, geo_px=1.0, geo_rel_depth=0.01)
    rng = np.random.default_rng(3)
    gt = w.gt_depth[w.ref].astype(np.float64)
    depth = gt * (1 + 0.003 * rng.normal(size=gt.shape))
    normal = w.gt_normal[w.ref].astype(np.float64)
    cost = np.zeros_like(depth)
    maps = [w.gt_depth[i].astype(np.float64) for i in w.nbrs]
    mposes = [w.poses[i] for i in w.nbrs]
    d0, _, _, e0, ed0, _ = oracle.consistency(depth, normal, cost, w.poses[w.ref], maps, mposes,
                                              params, diagnostics=True)
    s = W // 2
    T = np.diag([-1.0, 1.0, -1.0])
    d1, _, _, e1, ed1, _ = oracle.consistency(np.roll(depth, s, axis=1),
                                              np.roll(np.einsum("ij,jhw->ihw", T, normal), s, axis=2),
                                              cost, _half_turn(w.poses[w.ref]),
                                              [np.roll(m, s, axis=1) for m in maps],
                                              [_half_turn(p) for p in mposes], params, diagnostics=True)
    e1 = np.roll(e1, -s, axis=2)
    ed1 = np.roll(ed1, -s, axis=2)
    d1 = np.roll(d1, -s, axis=1)
    fin = np.isfinite(e0) & np.isfinite(e1)
    assert np.array_equal(np.isfinite(e0), np.isfinite(e1))
    assert np.allclose(e0[fin], e1[fin], atol=1e-6)
    assert np.allclose(ed0[fin], ed1[fin], atol=1e-9)
    # decisions agree except at an error sitting on a threshold
    near = ((np.abs(e0 - 1.0) < 1e-6) | (np.abs(ed0 - 0.01) < 1e-9)).any(0)
    assert np.array_equal((d0 > 0)[~near], (d1 > 0)[~near])
    # the seam matters here: some reprojections land across it, with errors
    # up to the threshold
    cross = fin & (e0 > 0.5) & (e0 <= 1.0)
    cols = np.nonzero(cross.any(axis=(0, 1)))[0]
    assert ((cols < 2) | (cols > W - 3)).any()
