"""Dense point-cloud fusion and the panorama coverage measure on the GPU,
against the FP64 oracle: both lift points in FP64 and take the voxel of
floor(X / voxel), so the keep masks and counts must be equal; on rendered
depth maps of four keyframes at 384x192 for three voxel sizes and at the
full 1920x960, and the coverage of a 720x360 panorama by the kept points."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


def _maps(W):
    w = synth.scaled("hall", W, seed=2)
    ks = [0, 1, 2, 3]
    return w, [w.gt_depth[k].astype(np.float32) for k in ks], [w.poses[k] for k in ks]


@pytest.mark.parametrize("W,voxel,n_maps", [(384, 0.02, 4), (384, 0.1, 4), (384, 0.5, 4), (1920, 0.02, 4),
                                            (210, 0.03, 4), (102, 0.05, 1), (102, 0.01, 3)])
def test_keep_masks_match_oracle(pms, W, voxel, n_maps):
    """Also on sizes whose 8 x 8 insertion tiles are partial at the right and
    bottom (210 x 105, 102 x 51) and with one and three maps (the insertion
    runs one launch per map)."""
    w, depths, poses = _maps(W)
    depths, poses = depths[:n_maps], poses[:n_maps]
    say(f"fuse {n_maps} maps {W}x{W // 2} voxel {voxel}")
    keep_g, n_g = pms.fuse([torch.from_numpy(d).cuda() for d in depths], poses, voxel)
    torch.cuda.synchronize()
    keep_o, n_o = oracle.fuse([d.astype(np.float64) for d in depths], poses, voxel)
    keep_g = keep_g.cpu().numpy()
    diff = (keep_g != keep_o).mean()
    print(f"kept {n_o} of {sum((d > 0).sum() for d in depths)} points, mask differences {diff:.2e}")
    assert n_g == keep_g.sum()
    assert diff <= 1e-6 and abs(n_g - n_o) <= max(1, int(1e-6 * keep_o.size))


def test_coverage_matches_oracle(pms):
    w, depths, poses = _maps(384)
    dev = [torch.from_numpy(d).cuda() for d in depths]
    keep, _ = pms.fuse(dev, poses, 0.05)
    say("coverage 720x360")
    n_g, cover_g = pms.coverage(dev, poses, keep, poses[2])
    torch.cuda.synchronize()
    keep_o, _ = oracle.fuse([d.astype(np.float64) for d in depths], poses, 0.05)
    n_o, cover_o = oracle.coverage([d.astype(np.float64) for d in depths], poses, keep_o, poses[2])
    print(f"coverage {n_o / (720 * 360):.3f}")
    assert n_g == n_o and np.array_equal(cover_g.cpu().numpy(), cover_o)


def test_coverage_of_every_point_matches_oracle(pms):
    """Coverage without keep bytes (every point with depth > 0), three maps
    of 208 x 104: the marking waves' last span is partial. (Seen from a map's
    own camera, its pixel centres land exactly on panorama pixel borders
    unless 8 divides the map height: 720 (x + 1/2) / W, 360 (y + 1/2) / H
    is then never an integer, so no point sits on a rounding tie.)"""
    w, depths, poses = _maps(208)
    depths, poses = depths[:3], poses[:3]
    depths[1][40:60, 20:90] = 0.0  # a hole: points without depth are skipped
    dev = [torch.from_numpy(d).cuda() for d in depths]
    say("coverage 720x360 of every point, 3 maps 208x104")
    n_g, cover_g = pms.coverage(dev, poses, None, poses[1])
    torch.cuda.synchronize()
    n_o, cover_o = oracle.coverage([d.astype(np.float64) for d in depths], poses, None, poses[1])
    print(f"covered {n_o} pixels")
    assert n_o > 0 and n_g == n_o and np.array_equal(cover_g.cpu().numpy(), cover_o)


def _shifted(poses, offset):
    """The same cameras in a world frame moved by `offset` (metres)."""
    o = np.asarray(offset, dtype=np.float64)
    return [(np.asarray(R), np.asarray(t) - np.asarray(R) @ o) for R, t in poses]


def test_keep_masks_match_oracle_far_from_the_world_origin(pms):
    """Georeferenced-size world coordinates (thousands of km, far beyond 2^20
    voxels of 2 cm): voxels are taken relative to the first camera, so the
    result is still the oracle's."""
    w, depths, poses = _maps(384)
    poses = _shifted(poses, (3.2e6, -1.5e3, -2.7e6))
    say("fuse 4 maps 384x192 voxel 0.02, world offset of ~4000 km")
    keep_g, n_g = pms.fuse([torch.from_numpy(d).cuda() for d in depths], poses, 0.02)
    torch.cuda.synchronize()
    keep_o, n_o = oracle.fuse([d.astype(np.float64) for d in depths], poses, 0.02)
    keep_g = keep_g.cpu().numpy()
    diff = (keep_g != keep_o).mean()
    print(f"kept {n_o}, mask differences {diff:.2e}")
    assert n_o > 0.1 * keep_o.size / 4
    assert diff <= 1e-5


def test_points_beyond_the_key_range_are_not_kept(pms):
    """The documented limit: a point more than 2^20 voxels from the first
    map's camera centre along an axis is not kept (the oracle, with unbounded
    integer voxels, keeps it); every other decision is the oracle's."""
    w, depths, poses = _maps(192)
    voxel = 4e-6  # 2^20 voxels = 4.19 m
    dev = [torch.from_numpy(d).cuda() for d in depths]
    say("fuse 4 maps 192x96 with a 4 micrometre voxel")
    keep_g, n_g = pms.fuse(dev, poses, voxel)
    torch.cuda.synchronize()
    keep_g = keep_g.cpu().numpy().reshape(len(depths), -1)
    keep_o, _ = oracle.fuse([d.astype(np.float64) for d in depths], poses, voxel)
    keep_o = keep_o.reshape(len(depths), -1)
    # world points and their voxel offsets from the first camera's voxel
    from helpers import bearings
    b = bearings(w.W, w.H).reshape(3, -1)
    R0, t0 = poses[0]
    c0 = -np.asarray(R0).T @ np.asarray(t0)
    org = np.floor(c0 / voxel)
    for m, (d, (R, t)) in enumerate(zip(depths, poses)):
        X = np.asarray(R).T @ (d.reshape(-1).astype(np.float64) * b - np.asarray(t)[:, None])
        off = np.floor(X / voxel) - org[:, None]
        # (a margin of 2 voxels either side of the limit for FP64 rounding)
        valid = d.reshape(-1) > 0
        far = (np.abs(off) >= 2 ** 20 + 2).any(0) & valid
        near = (np.abs(off) < 2 ** 20 - 2).all(0) & valid
        assert far.sum() > 100 and near.sum() > 100
        assert not keep_g[m][far].any()
        assert keep_o[m][far].any()
        assert (keep_g[m][near] != keep_o[m][near]).mean() <= 1e-4
