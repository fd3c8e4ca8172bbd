"""Pins of the oracle's initialisation, red-black propagation with random
refinement, and geometric consistency.

* Brute-force plane sweep (the textbook special case): inside a textured
  sphere centred on the reference camera every true plane is fronto-parallel,
  so an exhaustive fronto-parallel sweep over inverse depth bounds what
  PatchMatch must reach; PatchMatch must match or beat the sweep's cost and
  land within two sweep bins of its depth.
* Ground truth: rendered scenes give the true range per pixel.
* Order independence: a seeded random pixel order within each half-sweep,
  written in place on one thread, gives bitwise the same result as the
  threaded run.
* A neighbour identical to the reference at the same pose has cost 0 for
  every hypothesis.
* Random initialisation: inverse depth uniform, normals uniform on the
  hemisphere facing the camera.
* Consistency: ground-truth maps are kept, maps scaled by 5% are dropped, and
  a sub-pixel yaw gives a closed-form reprojection error.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth


def _sphere_scene(W, seed=0, radius=1.5, baseline=0.35):
    rng = np.random.default_rng(seed)
    centre = np.array([0.0, -1.5, 0.0])
    sph = synth._prim(synth.PRIM_SPHERE, centre, [radius])
    scene = synth._scene([sph], n_octaves=1, base_freq=1.0 / 0.3, tex_seed=seed + 17)
    poses = [synth.camera_pose(centre, rng.uniform(-math.pi, math.pi))]
    for k in range(2):
        a = rng.uniform(-math.pi, math.pi)
        c = centre + baseline * np.array([math.cos(a), rng.uniform(-0.3, 0.3), math.sin(a)])
        poses.append(synth.camera_pose(c, rng.uniform(-math.pi, math.pi)))
    imgs = [synth.render(scene, p, W, W // 2, ss=4)[0].astype(np.float64) for p in poses]
    return imgs, poses


def _bearings(W, H):
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    lam = 2 * np.pi * x / W - np.pi
    phi = np.pi / 2 - np.pi * y / H
    L, P = np.meshgrid(lam, phi)
    return np.stack([np.cos(P) * np.sin(L), -np.sin(P), np.cos(P) * np.cos(L)])


def test_patchmatch_reaches_brute_force_plane_sweep():
    W, H = 64, 32
    imgs, poses = _sphere_scene(W)
    params = synth.params_for("box_room", iterations=6, depth_min=0.5, depth_max=10.0, seed=3)
    b = _bearings(W, H)
    fronto = -b
    inv = np.linspace(1 / params["depth_max"], 1 / params["depth_min"], 128)
    best_c = np.full((H, W), np.inf)
    best_d = np.zeros((H, W))
    for rho in inv:
        d = np.full((H, W), 1.0 / rho)
        c, _ = oracle.eval_cost(imgs[0], imgs[1:], poses[0], poses[1:], params, d, fronto)
        better = c < best_c
        best_c[better] = c[better]
        best_d[better] = d[better]
    depth, normal, cost = oracle.densify(imgs[0], imgs[1:], poses[0], poses[1:], params)
    r = 3
    band = slice(r, H - r)
    sweep_ok = best_c[band] < 0.5
    reached = cost[band] <= best_c[band] + 1e-3
    assert reached[sweep_ok].mean() >= 0.95
    # within two inverse-depth bins of the sweep's depth
    bin_w = inv[1] - inv[0]
    close = np.abs(1 / depth[band] - 1 / best_d[band]) <= 2 * bin_w
    assert close[sweep_ok].mean() >= 0.95
    # and the sweep itself finds the true radius
    assert np.median(np.abs(best_d[band][sweep_ok] - 1.5)) < 0.1


def test_ground_truth_accuracy_box_room(box_room):
    w = box_room
    imgs = w.images_f32()
    depth, normal, cost = oracle.densify(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                                         [w.poses[i] for i in w.nbrs], w.params)
    gt = w.gt_depth[w.ref]
    r = (w.params["patch_size"] - 1) // 2
    band = np.zeros_like(gt, dtype=bool)
    band[r:w.H - r] = True
    assert np.all(depth[band] > 0)
    assert np.all(depth[~band] == 0) and np.all(cost[~band] == 2.0)
    rel = np.abs(depth - gt) / gt
    assert (rel[band] < 0.01).mean() >= 0.70
    assert (rel[band] < 0.05).mean() >= 0.97
    # normals are unit and face the camera
    b = _bearings(w.W, w.H)
    assert np.allclose(np.linalg.norm(normal[:, band], axis=0), 1.0, atol=1e-12)
    assert np.all((normal * b).sum(0)[band] < 0)


def test_pixel_order_does_not_change_the_result():
    w = synth.scaled("box_room", 96, seed=1)
    imgs = w.images_f32()
    args = (imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref], [w.poses[i] for i in w.nbrs])
    params = dict(w.params, iterations=2)
    a = oracle.densify(*args, params, n_threads=4)
    b = oracle.densify(*args, params, n_threads=1, order_seed=12345)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_identical_neighbour_at_same_pose_costs_zero():
    w = synth.scaled("box_room", 96, seed=2)
    img = w.images_f32()[0]
    pose = w.poses[0]
    depth, normal, cost = oracle.densify(img, [img, img], pose, [pose, pose],
                                         dict(w.params, iterations=1))
    r = (w.params["patch_size"] - 1) // 2
    assert np.all(cost[r:w.H - r] < 1e-12)


def test_random_initialisation_distribution():
    W, H = 192, 96
    w = synth.scaled("box_room", W, seed=3)
    img = w.images_f32()
    params = dict(w.params, iterations=0, depth_min=0.4, depth_max=12.0, seed=77)
    depth, normal, cost = oracle.densify(img[0], img[1:], w.poses[0], w.poses[1:], params)
    r = (params["patch_size"] - 1) // 2
    d = depth[r:H - r].ravel()
    n = normal[:, r:H - r].reshape(3, -1)
    b = _bearings(W, H)[:, r:H - r].reshape(3, -1)
    assert np.all((d >= params["depth_min"]) & (d <= params["depth_max"]))
    lo, hi = 1 / params["depth_max"], 1 / params["depth_min"]
    assert stats.kstest((1 / d - lo) / (hi - lo), "uniform").pvalue > 1e-3
    assert np.allclose(np.linalg.norm(n, axis=0), 1.0, atol=1e-12)
    cosang = (n * b).sum(0)
    assert np.all(cosang < 0)
    # uniform on the sphere => |n.b| uniform on [0, 1] (Archimedes)
    assert stats.kstest(-cosang, "uniform").pvalue > 1e-3
    # the stored cost is the cost of the stored plane
    c2, _ = oracle.eval_cost(img[0], img[1:], w.poses[0], w.poses[1:], params, depth, normal)
    assert np.array_equal(c2, cost)


def test_consistency_keeps_ground_truth_and_drops_scaled_maps(box_room):
    w = box_room
    params = dict(w.params)
    gt = w.gt_depth[w.ref].astype(np.float64)
    nrm = w.gt_normal[w.ref].astype(np.float64)
    cost = np.zeros_like(gt)
    maps = [w.gt_depth[i].astype(np.float64) for i in w.nbrs]
    mp = [w.poses[i] for i in w.nbrs]
    # The nearest-pixel lookup moves the neighbour's point by up to half a
    # pixel; at 256 px (24.5 mrad per pixel) on oblique walls that alone is a
    # few percent of range, and near the poles half a row is many pixels of
    # longitude. Ground truth must pass thresholds above that quantisation at
    # mid latitudes.
    loose = dict(params, geo_px=2.0, geo_rel_depth=0.05)
    d1, n1, c1, epx, ed, ag = oracle.consistency(gt, nrm, cost, w.poses[w.ref], maps, mp, loose,
                                                 diagnostics=True)
    lat = np.pi / 2 - np.pi * (np.arange(w.H) + 0.5) / w.H
    mid = np.abs(lat) < np.radians(60)
    assert (d1[mid] > 0).mean() >= 0.99
    assert np.median(epx[:, mid]) < 0.5
    assert np.array_equal(d1 > 0, c1 < 2.0)
    # 5% too far (beyond the lookup's quantisation): every pixel dropped at
    # the default 1% threshold
    d2, n2, c2 = oracle.consistency(gt, nrm, cost, w.poses[w.ref], [1.05 * m for m in maps], mp,
                                    params)
    assert np.all(d2 == 0) and np.all(c2 == 2.0) and np.all(n2 == 0)
    # 10% too far: every pixel dropped at the loose 5% threshold
    d3, _, _ = oracle.consistency(gt, nrm, cost, w.poses[w.ref], [1.10 * m for m in maps], mp,
                                  loose)
    assert np.all(d3 == 0)


def test_consistency_closed_form_reprojection_error():
    W, H = 128, 64
    params = synth.params_for("box_room", geo_px=1.0, geo_rel_depth=0.01)
    depth = np.full((H, W), 2.5)
    normal = -_bearings(W, H)
    cost = np.zeros((H, W))
    f = 0.3
    ref_pose = synth.camera_pose([0, 0, 0], 0.0)
    nbr_pose = synth.camera_pose([0, 0, 0], 2 * math.pi * (7 + f) / W)
    d, n, c, epx, ed, ag = oracle.consistency(depth, normal, cost, ref_pose, [depth], [nbr_pose],
                                              params, diagnostics=True)
    r = 3
    # the neighbour sees ref column x at x - 7.3; the nearest pixel is x - 7,
    # which maps back to x + 0.3
    assert np.allclose(epx[0, r:H - r], f, atol=1e-9)
    assert np.allclose(ed[0, r:H - r], 0.0, atol=1e-12)
    assert np.all(d[r:H - r] == 2.5)
    # a threshold below the error drops everything
    d, *_ = oracle.consistency(depth, normal, cost, ref_pose, [depth], [nbr_pose],
                               dict(params, geo_px=0.29))
    assert np.all(d == 0)


def test_propagation_transfers_the_plane_not_the_depth(box_room):
    """With one propagation offset and no refinement, a pixel whose neighbour
    holds the ray-cast ground-truth plane of a flat wall must take the
    ground-truth range of its OWN ray (the neighbour's plane re-intersected),
    not the neighbour's range."""
    w = box_room
    imgs = w.images_f32()
    gt = w.gt_depth[w.ref].astype(np.float64)
    gn = w.gt_normal[w.ref].astype(np.float64)
    params = dict(w.params, offsets=[(3, 0)], refine_trials=0)
    rng = np.random.default_rng(5)
    b = _bearings(w.W, w.H)
    checked = 0
    for _ in range(400):
        x, y = int(rng.integers(0, w.W)), int(rng.integers(30, w.H - 30))
        qx = (x + 3) % w.W
        if not np.allclose(gn[:, y, x], gn[:, y, qx], atol=1e-6):
            continue  # p and q on different walls
        if abs(gt[y, x] - gt[y, qx]) < 0.02 * gt[y, x]:
            continue  # want a clearly slanted wall
        depth = np.full((w.H, w.W), 2.0)
        normal = -b.copy()
        depth[y, qx] = gt[y, qx]
        normal[:, y, qx] = gn[:, y, qx]
        cost, _ = oracle.eval_cost(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                                   [w.poses[i] for i in w.nbrs], params, depth, normal)
        d, n, c = oracle.update_pixel(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                                      [w.poses[i] for i in w.nbrs], params, depth, normal, cost,
                                      1, x, y)
        if c < cost[y, x]:
            assert d == pytest.approx(gt[y, x], rel=2e-5)
            assert np.allclose(n, gn[:, y, qx], atol=1e-12)
            checked += 1
        if checked >= 20:
            break
    assert checked >= 20


def test_cost_ties_keep_the_current_plane():
    """On a textureless image every view is invalid, so every candidate ties
    with the current cost; a pixel must only move to a strictly cheaper
    plane, so sweeps leave the random initialisation untouched."""
    W, H = 64, 32
    flat = np.full((H, W), 0.5)
    poses = [synth.camera_pose([0, 0, 0], 0.0), synth.camera_pose([0.2, 0, 0], 0.1),
             synth.camera_pose([0, 0, 0.2], -0.1)]
    p0 = synth.params_for("box_room", iterations=0, seed=9)
    p2 = dict(p0, iterations=2)
    a = oracle.densify(flat, [flat, flat], poses[0], poses[1:], p0)
    b = oracle.densify(flat, [flat, flat], poses[0], poses[1:], p2)
    assert np.all(a[2][3:H - 3] == 2.0)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_row_band_halfsweeps_compose_to_a_full_iteration():
    w = synth.scaled("box_room", 96, seed=4)
    imgs = w.images_f32()
    args = (imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref], [w.poses[i] for i in w.nbrs])
    p0 = dict(w.params, iterations=0, seed=5)
    p1 = dict(w.params, iterations=1, seed=5)
    d, n, c = oracle.densify(*args, p0)
    for colour in (0, 1):
        # two bands, each updated from the same input state
        da, na, ca = oracle.halfsweep_rows(*args, p1, d, n, c, 1, colour, 0, 20)
        db, nb, cb = oracle.halfsweep_rows(*args, p1, d, n, c, 1, colour, 20, w.H)
        d = np.where(np.arange(w.H)[:, None] < 20, da, db)
        n = np.where(np.arange(w.H)[None, :, None] < 20, na, nb)
        c = np.where(np.arange(w.H)[:, None] < 20, ca, cb)
    e = oracle.densify(*args, p1)
    assert np.array_equal(d, e[0]) and np.array_equal(n, e[1]) and np.array_equal(c, e[2])
