"""pms_densify_noalloc (the entry point for callers that cannot allocate
device memory) against pms_densify, through the C ABI: two calls in a row on
one context, the second on a smaller keyframe, each equal to pms_densify's
result bit for bit (same kernels and plan; only the memory differs), and a
call larger than the fixed scratch array rejected on the host."""
import numpy as np
import pytest
import torch

import synth
from helpers import gpu_images, say, split

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


def _args(w, params):
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    maps = [torch.from_numpy(w.gt_depth[i].astype(np.float32)).cuda() for i in w.maps]
    return (ref, nbrs, w.poses[w.ref], [w.poses[i] for i in w.nbrs], params, maps,
            [w.poses[i] for i in w.maps])


def _out(w):
    return (torch.full((w.H, w.W), -1.0, device="cuda"), torch.full((3, w.H, w.W), -1.0, device="cuda"),
            torch.full((w.H, w.W), -1.0, device="cuda"))


def test_noalloc_matches_densify_on_two_calls(pms):
    ctx = pms.Context(0)
    cases = [("hall", 384, "f32", 3), ("box_room", 160, "f32", 4)]
    for family, W, _, iters in cases:
        w = synth.scaled(family, W, seed=3)
        params = dict(w.params, iterations=iters)
        args = _args(w, params)
        say(f"densify_noalloc {family} {w.W}x{w.H} ({len(w.nbrs)} views, {len(args[5])} maps)")
        got = pms.densify_noalloc(*args, out=_out(w), ctx=ctx)
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in got]
        say(f"densify {family} {w.W}x{w.H}")
        ref = [t.cpu().numpy() for t in pms.densify(*args, out=_out(w), ctx=ctx)]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert (got[0] > 0).mean() > 0.3
    ctx.close()


def test_noalloc_rejects_more_than_its_scratch(pms):
    ctx = pms.Context(0)
    w = synth.scaled("hall", 1920, seed=0, ss=1)
    params = dict(w.params, iterations=1)
    args = _args(w, params)
    out = _out(w)
    say("densify_noalloc 1920x960 with 4 neighbours: over the scratch size")
    with pytest.raises(pms.PmsError, match="PMS_NOALLOC_SCRATCH_BYTES"):
        pms.densify_noalloc(*args, out=out, ctx=ctx)
    torch.cuda.synchronize()
    # nothing was written
    assert float(out[0].min()) == -1.0 and float(out[0].max()) == -1.0
    ctx.close()
