"""Plane-map warping (Sec. III-B) on the GPU, through the C ABI, against
the FP64 oracle.

* The warp itself: both sides project in FP64 and take the z-buffer decision
  on the range rounded to float, so the destination map agrees pixel for
  pixel except at decision ties (a projection on a pixel border, equal
  float ranges): validity agrees at >= 99.9% of pixels and where both carry
  the same plane the depth agrees to 1e-6 relative and the normal to 1e-6.
  At 384x192 and at the full 1920x960.
* Densification from warped initial planes (the oracle's warp of the
  previous keyframe's ground-truth planes, fed to both sides): >= 99% of
  oracle-valid pixels within 0.5% depth.
* Warped initial planes reach the ground truth faster than random ones.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import bearings, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


def _facing(w, k):
    """Ground-truth planes of keyframe k, normals turned to face its camera."""
    d = w.gt_depth[k].astype(np.float32)
    n = w.gt_normal[k].astype(np.float32).copy()
    flip = (n * bearings(w.W, w.H)).sum(0) > 0
    n[:, flip] *= -1
    return d, n


def _compare(dg, ng, do, no):
    vg, vo = dg > 0, do > 0
    agree = (vg == vo).mean()
    both = vg & vo
    rel = np.abs(dg[both] - do[both]) / do[both]
    same = rel <= 1e-6
    ndiff = np.abs(ng[:, both][:, same] - no[:, both][:, same]).max() if same.any() else 0.0
    other = (~same).mean() if both.any() else 0.0
    print(f"validity agrees at {agree:.5f}, {vg.mean():.3f} of pixels carry a plane, "
          f"{other:.2e} of them another winner, normal diff {ndiff:.2e}")
    assert agree >= 0.999
    assert other <= 1e-3
    assert ndiff <= 1e-6


@pytest.mark.parametrize("W", [384, 1920])
def test_warp_matches_oracle(pms, W):
    w = synth.scaled("hall", W, seed=1)
    prev, ref = w.ref - 1, w.ref
    d, n = _facing(w, prev)
    params = dict(w.params)
    say(f"warp {W}x{W // 2}")
    dg, ng = pms.warp_planes(torch.from_numpy(d).cuda(), torch.from_numpy(n).cuda(),
                             w.poses[prev], w.poses[ref], params)
    torch.cuda.synchronize()
    do, no = oracle.warp_planes(d.astype(np.float64), n.astype(np.float64), w.poses[prev],
                                w.poses[ref], params)
    _compare(dg.cpu().numpy(), ng.cpu().numpy(), do, no)


def test_densify_from_warped_planes_matches_oracle(pms):
    w = synth.scaled("hall", 256, seed=2)
    params = dict(w.params, iterations=2)
    prev, ref = w.ref - 1, w.ref
    d, n = _facing(w, prev)
    wd, wn = oracle.warp_planes(d, n, w.poses[prev], w.poses[ref], params)
    wd32, wn32 = wd.astype(np.float32), wn.astype(np.float32)
    imgs = [torch.from_numpy(a).cuda() for a in w.images]
    jd = pms.job(imgs[ref], [imgs[i] for i in w.nbrs], w.poses[ref], [w.poses[i] for i in w.nbrs],
                 params, init=(torch.from_numpy(wd32).cuda(), torch.from_numpy(wn32).cuda()))
    say("densify 256x128 from warped planes")
    dg = pms.densify_job(jd)[0]
    torch.cuda.synchronize()
    dg = dg.cpu().numpy()
    f64 = [a.astype(np.float64) for a in w.images_f32()]
    do, _, _ = oracle.densify(f64[ref], [f64[i] for i in w.nbrs], w.poses[ref],
                              [w.poses[i] for i in w.nbrs], params,
                              init_depth=wd32.astype(np.float64), init_normal=wn32.astype(np.float64))
    valid = do > 0
    frac = (np.abs(dg[valid] - do[valid]) <= 0.005 * do[valid]).mean()
    print(f"warm start: {frac:.4f} of oracle-valid pixels within 0.5%")
    assert frac >= 0.99


def test_warped_planes_converge_faster_on_gpu(pms):
    w = synth.scaled("hall", 384, seed=0)
    params = dict(w.params, iterations=1)
    prev, ref = w.ref - 1, w.ref
    d, n = _facing(w, prev)
    imgs = [torch.from_numpy(a).cuda() for a in w.images]
    say("GPU warp, then densify from it and from random planes")
    wd, wn = pms.warp_planes(torch.from_numpy(d).cuda(), torch.from_numpy(n).cuda(), w.poses[prev],
                             w.poses[ref], params)
    args = (imgs[ref], [imgs[i] for i in w.nbrs], w.poses[ref], [w.poses[i] for i in w.nbrs], params)
    d_rand = pms.densify(*args)[0]
    d_warm = pms.densify_job(pms.job(*args, init=(wd, wn)))[0]
    torch.cuda.synchronize()
    gt = w.gt_depth[ref]

    def acc(t):
        a = t.cpu().numpy()
        v = (a > 0) & (gt > 0)
        return float((np.abs(a[v] - gt[v]) <= 0.01 * gt[v]).sum() / max(v.sum(), 1))

    print(f"within 1% after one iteration: random {acc(d_rand):.3f}, warped {acc(d_warm):.3f}")
    assert acc(d_warm) > acc(d_rand) + 0.1
