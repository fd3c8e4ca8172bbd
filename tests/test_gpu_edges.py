"""Edge cases of the image size on the GPU, through the C ABI.

* A 12x6 image with a 7x7 patch has no row r pixels away from both poles:
  every output is invalid (depth 0, normal 0, cost 2), as in the oracle.
* An image of the largest accepted height (PMS_MAX_HEIGHT, W = 2H), whose
  re-laid-out neighbour copies fill 32-bit byte offsets up to just under
  2 GiB: one densify iteration on seeded textured images gives planes in
  range facing the camera, and at sampled pixels the stored cost is the
  oracle's cost of the stored plane.
* Degenerate inputs of the method: a constant reference (every view
  invalid: the random initial planes remain, the oracle's own), and
  neighbours seen from the reference's centre (the warp no longer depends
  on the plane: only the costs are unique).
"""
import os
import re

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


def _poses(n, seed):
    rng = np.random.default_rng(seed)
    poses = [synth.camera_pose(np.array([0.0, -1.5, 0.0]), 0.3)]
    for _ in range(n):
        a = rng.uniform(-np.pi, np.pi)
        c = np.array([0.0, -1.5, 0.0]) + rng.uniform(0.1, 0.3) * np.array([np.cos(a), 0.0, np.sin(a)])
        poses.append(synth.camera_pose(c, rng.uniform(-np.pi, np.pi)))
    return poses


def _texture(W, H, seed):
    """Seeded texture in [0.2, 0.8], float32: sinusoids along the rows and
    the columns plus noise."""
    rng = np.random.default_rng(seed)
    x = np.arange(W, dtype=np.float32)[None, :]
    y = np.arange(H, dtype=np.float32)[:, None]
    row = np.zeros((1, W), dtype=np.float32)
    col = np.zeros((H, 1), dtype=np.float32)
    for _ in range(3):
        row += np.float32(0.06) * np.sin(x * np.float32(rng.uniform(0.05, 0.6)) + np.float32(rng.uniform(0, 6.3)))
        col += np.float32(0.06) * np.sin(y * np.float32(rng.uniform(0.05, 0.6)) + np.float32(rng.uniform(0, 6.3)))
    img = rng.standard_normal(size=(H, W), dtype=np.float32)
    img *= np.float32(0.03)
    img += row
    img += col
    img += np.float32(0.5)
    return np.clip(img, 0.2, 0.8, out=img)


def test_empty_band_gives_invalid_outputs(pms):
    W, H = 12, 6
    params = dict(synth.params_for("box_room"), iterations=2)  # 7x7 patch: r = 3
    poses = _poses(2, seed=1)
    imgs = [_texture(W, H, seed=k) for k in range(3)]
    dev = [torch.from_numpy(a).cuda() for a in imgs]
    say("densify 12x6, empty band")
    d, n, c = pms.densify(dev[0], dev[1:], poses[0], poses[1:], params)
    torch.cuda.synchronize()
    assert torch.all(d == 0) and torch.all(n == 0) and torch.all(c == 2.0)
    depth = torch.full((H, W), 2.0, device="cuda")
    normal = torch.zeros((3, H, W), device="cuda")
    normal[2] = -1.0
    cost = pms.eval_cost(dev[0], dev[1:], poses[0], poses[1:], params, depth, normal)
    torch.cuda.synchronize()
    assert torch.all(cost == 2.0)
    f64 = [a.astype(np.float64) for a in imgs]
    do, no, co = oracle.densify(f64[0], f64[1:], poses[0], poses[1:], params)
    assert np.all(do == 0) and np.all(no == 0) and np.all(co == 2.0)


def test_maximum_height_densify(pms):
    hdr = open(os.path.join(ROOT, "include", "pms.h")).read()
    H = int(re.search(r"#define PMS_MAX_HEIGHT\s+(\d+)", hdr).group(1))
    W = 2 * H
    params = dict(synth.params_for("hall"), iterations=1)
    poses = _poses(4, seed=2)
    say(f"texturing 5 images of {W}x{H}")
    imgs = [_texture(W, H, seed=10 + k) for k in range(5)]
    dev = [torch.from_numpy(a).cuda() for a in imgs]
    say(f"densify {W}x{H}, 4 neighbours, 1 iteration")
    d, n, c = pms.densify(dev[0], dev[1:], poses[0], poses[1:], params)
    torch.cuda.synchronize()
    r = (params["patch_size"] - 1) // 2
    # sampled rows of the band, and the rows outside it
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([[r, H - 1 - r], rng.integers(r, H - r, 40)]))
    ri = torch.as_tensor(rows, device="cuda")
    dn = d[ri].cpu().numpy()
    nn = n[:, ri].cpu().numpy()
    cn = c[ri].cpu().numpy()
    assert np.all(dn >= params["depth_min"]) and np.all(dn <= params["depth_max"])
    assert np.all((cn >= 0.0) & (cn <= 2.0))
    # bearings of the sampled rows (the formula of helpers.bearings)
    lam = 2 * np.pi * (np.arange(W) + 0.5) / W - np.pi
    phi = np.pi / 2 - np.pi * (rows + 0.5) / H
    L, P = np.meshgrid(lam, phi)
    b = np.stack([np.cos(P) * np.sin(L), -np.sin(P), np.cos(P) * np.cos(L)])
    assert np.abs(np.linalg.norm(nn, axis=0) - 1).max() < 1e-5
    assert np.all((nn * b).sum(0) < 0)
    assert torch.all(d[:r] == 0) and torch.all(d[H - r:] == 0) and torch.all(c[:r] == 2.0)
    # the stored cost is the oracle's cost of the stored plane (sampled)
    say("oracle costs at sampled pixels")
    f64 = [a.astype(np.float64) for a in imgs]
    R = [oracle.relative_pose(poses[0], p) for p in poses[1:]]
    for _ in range(24):
        k = int(rng.integers(0, len(rows)))
        y, x = int(rows[k]), int(rng.integers(0, W))
        vc = [oracle.view_cost(f64[0], nb, Rj, tj, params, x, y, float(dn[k, x]),
                               nn[:, k, x].astype(np.float64))[0] for nb, (Rj, tj) in zip(f64[1:], R)]
        co = oracle.aggregate(vc, params["top_k"])
        assert abs(co - cn[k, x]) <= 1e-4 or min(vc) >= 2.0 and cn[k, x] == 2.0, (x, y, co, cn[k, x])


def test_textureless_reference_keeps_the_random_planes(pms):
    """A constant reference has no patch variance: every view is invalid
    (cost 2), no hypothesis is strictly better than another, and the random
    initial planes remain; the oracle draws the same ones (Philox)."""
    W, H = 64, 32
    params = dict(synth.params_for("box_room"), iterations=2, seed=5)
    poses = _poses(2, seed=4)
    imgs = [np.full((H, W), 0.5, dtype=np.float32)] + [_texture(W, H, seed=k) for k in (1, 2)]
    dev = [torch.from_numpy(a).cuda() for a in imgs]
    say("densify 64x32, constant reference")
    d, n, c = (t.cpu().numpy() for t in pms.densify(dev[0], dev[1:], poses[0], poses[1:], params))
    f64 = [a.astype(np.float64) for a in imgs]
    do, no, co = oracle.densify(f64[0], f64[1:], poses[0], poses[1:], params)
    r = (params["patch_size"] - 1) // 2
    band = slice(r, H - r)
    assert np.all(c[band] == 2.0) and np.all(co[band] == 2.0)
    assert np.all(d[band] > 0)
    np.testing.assert_allclose(d[band], do[band], rtol=1e-5)
    np.testing.assert_allclose(n[:, band], no[:, band], atol=1e-5)


def test_zero_baseline_costs(pms):
    """Neighbours seen from the reference's own centre (other yaw only): the
    warp no longer depends on the plane, so every hypothesis scores the same
    and the depths are not determined; what is unique is the cost, close to
    0 on the textured scene, and every plane must still be valid."""
    w = synth.scaled("box_room", 128, seed=3)
    c0 = -w.poses[w.ref][0].T @ w.poses[w.ref][1]
    poses = [w.poses[w.ref]] + [synth.camera_pose(c0, yaw) for yaw in (0.7, -1.9)]
    scene, _, _, _, _ = synth.scene_and_poses("box_room", 3)
    imgs = [w.images[w.ref]] + [synth.render(scene, p, w.W, w.H, ss=4)[0] for p in poses[1:]]
    dev = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in imgs]
    params = dict(w.params, iterations=2)
    say("densify 128x64, zero baseline")
    d, n, c = (t.cpu().numpy() for t in pms.densify(dev[0], dev[1:], poses[0], poses[1:], params))
    r = (params["patch_size"] - 1) // 2
    band = slice(r, w.H - r)
    assert np.all((d[band] >= params["depth_min"]) & (d[band] <= params["depth_max"]))
    valid = c[band] < 2.0
    assert valid.mean() > 0.9
    assert np.median(c[band][valid]) < 0.05
    # the oracle scores the GPU's planes the same
    f64 = [a.astype(np.float64) for a in imgs]
    co, _ = oracle.eval_cost(f64[0], f64[1:], poses[0], poses[1:], params, d.astype(np.float64),
                             n.astype(np.float64))
    both = (c < 2.0) & (co < 2.0)
    assert np.abs(c[both] - co[both]).max() <= 1e-4


def test_work_block_grows_on_another_stream_without_a_host_wait(pms):
    """A context's device block grows stream-ordered: a small call on one
    stream, then at once (no synchronisation) a larger one on another stream
    of the same context, give the results of a fresh context for each."""
    small = synth.scaled("box_room", 96, seed=4)
    large = synth.scaled("hall", 256, seed=4)
    ctx = pms.Context(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for w, st in ((small, s1), (large, s2)):
        imgs = [torch.from_numpy(a).cuda() for a in w.images]
        torch.cuda.synchronize()
        params = dict(w.params, iterations=2)
        say(f"densify {w.W}x{w.H} on its own stream, no host wait")
        with torch.cuda.stream(st):
            o = pms.densify(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                            [w.poses[i] for i in w.nbrs], params, ctx=ctx, stream=st)
        outs.append((w, imgs, params, o))
    torch.cuda.synchronize()
    for w, imgs, params, o in outs:
        fresh = pms.Context(0)
        ref = pms.densify(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                          [w.poses[i] for i in w.nbrs], params, ctx=fresh)
        torch.cuda.synchronize()
        for a, b in zip(o, ref):
            assert torch.equal(a, b)
        fresh.close()
    ctx.close()
