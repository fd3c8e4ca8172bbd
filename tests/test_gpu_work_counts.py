"""The half-sweeps' executed-work counters (pms_work_count_*): counting
changes no result bit, and the counts obey the identities of the sweep
(Sec. III-C): every pixel update considers n_offsets propagation candidates
and refine_trials refinement trials, each of which is dropped unscored
(geometry or a repeat) or scored; a scored plane either fails the facing
test (no view evaluated) or evaluates views until the top-k bound prunes
the rest."""
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


@pytest.mark.parametrize("name,W,dtype", [("hall", 384, None), ("courtyard", 320, "u8"),
                                          ("hall", 256, "f16")])
def test_counting_changes_nothing_and_adds_up(pms, name, W, dtype):
    w = synth.scaled(name, W, seed=0, dtype=dtype if dtype == "u8" else None)
    if dtype == "f16":
        w.images = [a.astype(np.float16) for a in w.images]
    params = dict(w.params, iterations=3)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = w.poses[w.ref], [w.poses[i] for i in w.nbrs]
    ctx = pms.Context(0)
    say(f"densify {name} {W} {dtype}, uncounted then counted")
    a = [t.cpu().numpy() for t in pms.densify(ref, nbrs, rp, nps, params, ctx=ctx)]
    ctx.work_count_enable(True)
    b = [t.cpu().numpy() for t in pms.densify(ref, nbrs, rp, nps, params, ctx=ctx)]
    c = ctx.work_count_read(reset=True)
    ctx.work_count_enable(False)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    print(c)
    r = (params["patch_size"] - 1) // 2
    n_views = len(w.nbrs)
    assert c["pixels"] == 2 * params["iterations"] * (w.H - 2 * r) * w.W // 2
    assert c["prop_candidates"] == c["pixels"] * len(params["offsets"])
    assert c["refine_trials"] == c["pixels"] * params["refine_trials"]
    assert c["prop_candidates"] + c["refine_trials"] == (c["skipped_geometry"] + c["skipped_repeat"]
                                                          + c["scored"])
    assert c["view_evals"] + c["views_pruned"] == n_views * (c["scored"] - c["facing_rejects"])
    assert c["view_evals"] > 0 and c["views_pruned"] > 0 and c["skipped_repeat"] > 0
    # disabled again: nothing more is counted
    pms.densify(ref, nbrs, rp, nps, params, ctx=ctx)
    assert all(v == 0 for v in ctx.work_count_read().values())
    ctx.close()
