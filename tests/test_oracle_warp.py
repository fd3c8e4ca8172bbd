"""Pins of the oracle's relative pose and plane-induced patch warp.

The warped sample positions are read back through ramp images (I(x, y) = x
and I(x, y) = y make bilinear sampling return the coordinate itself) and
compared with a route the oracle does not take: rays cast in the WORLD frame
against an analytic world plane, moved into the neighbour with its own
world->camera pose, and projected with numpy.
"""
import math

import numpy as np
import pytest

import oracle
import synth

W, H = 256, 128


def _bearing(x, y):
    lam = 2 * math.pi * (x + 0.5) / W - math.pi
    phi = math.pi / 2 - math.pi * (y + 0.5) / H
    return np.array([math.cos(phi) * math.sin(lam), -math.sin(phi), math.cos(phi) * math.cos(lam)])


def _to_pixel(Y):
    lon = math.atan2(Y[0], Y[2])
    lat = math.atan2(-Y[1], math.hypot(Y[0], Y[2]))
    return W * (lon + math.pi) / (2 * math.pi) - 0.5, H * (math.pi / 2 - lat) / math.pi - 0.5


RAMP_X = np.tile(np.arange(W, dtype=np.float64), (H, 1))
RAMP_Y = np.tile(np.arange(H, dtype=np.float64)[:, None], (1, W))


def _random_pose(rng, centre_scale=1.0):
    c = rng.uniform(-centre_scale, centre_scale, 3)
    return synth.camera_pose(c, rng.uniform(-math.pi, math.pi), rng.uniform(-0.3, 0.3),
                             rng.uniform(-0.3, 0.3))


def test_relative_pose_maps_points():
    rng = np.random.default_rng(10)
    for _ in range(50):
        A = _random_pose(rng)
        B = _random_pose(rng)
        R, t = oracle.relative_pose(A, B)
        for _ in range(5):
            X = rng.normal(size=3) * 4
            assert np.allclose(R @ (A[0] @ X + A[1]) + t, B[0] @ X + B[1], atol=1e-12)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)


def _warp_case(rng, params):
    """One random (ref pose, nbr pose, world plane, ref pixel) whose warped
    patch stays away from the seam; returns the oracle samples and the
    world-frame expectation."""
    dx, dy = oracle.patch_offsets(params)
    r = (params["patch_size"] - 1) // 2
    while True:
        ref_pose = synth.camera_pose(rng.uniform(-0.5, 0.5, 3), rng.uniform(-math.pi, math.pi),
                                     rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2))
        C_r = -ref_pose[0].T @ ref_pose[1]
        C_n = C_r + rng.uniform(-0.6, 0.6, 3)
        nbr_pose = synth.camera_pose(C_n, rng.uniform(-math.pi, math.pi), rng.uniform(-0.2, 0.2),
                                     rng.uniform(-0.2, 0.2))
        x = int(rng.integers(0, W))
        y = int(rng.integers(r + 5, H - r - 5))
        N = rng.normal(size=3)
        N /= np.linalg.norm(N)
        dir_p = ref_pose[0].T @ _bearing(x, y)
        if abs(N @ dir_p) < 0.3:
            continue
        depth = rng.uniform(1.0, 6.0)
        P0 = C_r + depth * dir_p  # the plane passes through the centre pixel at this range
        n_ref = ref_pose[0] @ N
        if n_ref @ _bearing(x, y) > 0:
            n_ref = -n_ref
        exp = []
        ok = True
        for ox, oy in zip(dx, dy):
            dq = ref_pose[0].T @ _bearing((x + ox) % W, y + oy)
            den = N @ dq
            s = (N @ (P0 - C_r)) / den
            if s <= 0:
                ok = False
                break
            Xw = C_r + s * dq
            u, v = _to_pixel(nbr_pose[0] @ Xw + nbr_pose[1])
            if not (2.0 < u < W - 3.0 and 0.0 <= v <= H - 1):
                ok = False
                break
            exp.append((u, v))
        if not ok:
            continue
        R, t = oracle.relative_pose(ref_pose, nbr_pose)
        cx, rx, sx, _, _ = oracle.view_cost(RAMP_X, RAMP_X, R, t, params, x, y, depth, n_ref)
        cy, ry, sy, _, _ = oracle.view_cost(RAMP_Y, RAMP_Y, R, t, params, x, y, depth, n_ref)
        return np.array(exp), sx, sy


@pytest.mark.parametrize("patch", [(7, 1), (11, 2), (15, 2)])
def test_plane_warp_matches_world_frame_ray_cast(patch):
    params = synth.params_for("hall", patch_size=patch[0], patch_stride=patch[1])
    rng = np.random.default_rng(11 + patch[0])
    for _ in range(25):
        exp, sx, sy = _warp_case(rng, params)
        assert np.max(np.abs(sx - exp[:, 0])) < 1e-9
        assert np.max(np.abs(sy - exp[:, 1])) < 1e-9


def test_pure_rotation_warp_is_plane_independent():
    params = synth.params_for("box_room")
    rng = np.random.default_rng(12)
    ref_pose = synth.camera_pose([0.1, -1.0, 0.2], 0.3, 0.1, -0.05)
    C = -ref_pose[0].T @ ref_pose[1]
    nbr_pose = synth.camera_pose(C, -1.1, 0.2, 0.1)  # same centre => t_rel = 0
    R, t = oracle.relative_pose(ref_pose, nbr_pose)
    assert np.allclose(t, 0, atol=1e-14)
    img = rng.uniform(0, 1, (H, W))
    for _ in range(20):
        x, y = int(rng.integers(0, W)), int(rng.integers(10, H - 10))
        b = oracle.unproject(W, H, x, y)
        n1 = -b + 0.2 * rng.normal(size=3)
        n2 = -b + 0.2 * rng.normal(size=3)
        _, _, s1, _, _ = oracle.view_cost(img, img, R, t, params, x, y, 1.3, n1)
        _, _, s2, _, _ = oracle.view_cost(img, img, R, t, params, x, y, 7.9, n2)
        assert np.max(np.abs(s1 - s2)) < 1e-12


def test_yaw_only_rotation_is_a_longitude_shift():
    params = synth.params_for("box_room")
    dxs, dys = oracle.patch_offsets(params)
    alpha = 0.37
    ref_pose = synth.camera_pose([0, 0, 0], 0.0)
    nbr_pose = synth.camera_pose([0, 0, 0], alpha)  # turned right by alpha
    R, t = oracle.relative_pose(ref_pose, nbr_pose)
    shift = alpha * W / (2 * math.pi)
    for x, y in [(100, 20), (140, 64), (200, 100)]:
        b = oracle.unproject(W, H, x, y)
        _, _, sx, _, _ = oracle.view_cost(RAMP_X, RAMP_X, R, t, params, x, y, 2.0, -b)
        _, _, sy, _, _ = oracle.view_cost(RAMP_Y, RAMP_Y, R, t, params, x, y, 2.0, -b)
        assert np.allclose(sx, (x + dxs) - shift, atol=1e-9)
        assert np.allclose(sy, y + dys, atol=1e-9)


def test_whole_pixel_yaw_reproduces_shifted_reference():
    params = synth.params_for("box_room")
    rng = np.random.default_rng(13)
    ref = rng.uniform(0, 1, (H, W))
    k = 9
    nbr = np.roll(ref, -k, axis=1)  # the neighbour sees column x + k at column x
    R, t = oracle.relative_pose(synth.camera_pose([0, 0, 0], 0.0),
                                synth.camera_pose([0, 0, 0], 2 * math.pi * k / W))
    for x, y in [(0, 10), (W - 1, 64), (77, 100)]:
        b = oracle.unproject(W, H, x, y)
        c, r_s, s_s, _, _ = oracle.view_cost(ref, nbr, R, t, params, x, y, 3.0, -b)
        assert np.max(np.abs(r_s - s_s)) < 1e-9
        assert c == pytest.approx(0.0, abs=1e-9)


def test_plane_behind_a_sample_ray_invalidates_the_view():
    params = synth.params_for("box_room")
    rng = np.random.default_rng(14)
    img = rng.uniform(0, 1, (H, W))
    R, t = np.eye(3), np.array([0.1, 0.0, 0.0])
    x, y = 50, 64
    b = oracle.unproject(W, H, x, y)
    # a plane almost containing the centre ray: some sample rays miss it
    side = np.cross(b, [0, 1, 0])
    side /= np.linalg.norm(side)
    n = -0.001 * b + side
    c, *_ = oracle.view_cost(img, img, R, t, params, x, y, 2.0, n)
    assert c == 2.0
    # a normal facing away from the camera is invalid as well
    c, *_ = oracle.view_cost(img, img, R, t, params, x, y, 2.0, b)
    assert c == 2.0
