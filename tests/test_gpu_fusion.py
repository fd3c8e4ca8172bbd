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


@pytest.mark.parametrize("W,voxel", [(384, 0.02), (384, 0.1), (384, 0.5), (1920, 0.02)])
def test_keep_masks_match_oracle(pms, W, voxel):
    w, depths, poses = _maps(W)
    say(f"fuse 4 maps {W}x{W // 2} voxel {voxel}")
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
