"""The view filter (Sec. III-A, Eq. 1) on the GPU against the FP64 oracle:
both count, in FP64, the sparse points whose triangulation angle lies in
[6, 60] degrees, so the counts must be equal (integers): on surface points
of the rendered hall seen from keyframe pairs at several baselines, and on
a million random points."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import centre, say, world_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


@pytest.mark.parametrize("a,b", [(1, 2), (0, 4), (2, 3)])
def test_counts_match_oracle_on_scene_points(pms, a, b):
    w = synth.scaled("hall7", 128, seed=0)
    pts = world_points(w, a, 20000, seed=a * 10 + b)
    ca, cb = centre(w.poses[a]), centre(w.poses[b])
    say(f"view filter keyframes {a},{b}")
    acc_g, k_g, c_g = pms.view_filter(ca, cb, torch.from_numpy(pts).cuda())
    acc_o, k_o, c_o = oracle.view_filter(ca, cb, pts)
    print(f"{k_o}/{c_o} points in range, accepted {acc_o}")
    assert (k_g, c_g, acc_g) == (k_o, c_o, acc_o)


def test_counts_match_oracle_on_a_million_points(pms):
    rng = np.random.default_rng(5)
    pts = rng.normal(size=(1 << 20, 3)) * [5.0, 2.0, 5.0]
    pts[:10] = [0.0, 0.0, 0.0]  # at a centre: not counted
    ca, cb = [0.0, 0.0, 0.0], [0.8, -0.1, 0.3]
    say("view filter, 2^20 points")
    acc_g, k_g, c_g = pms.view_filter(ca, cb, torch.from_numpy(pts).cuda())
    acc_o, k_o, c_o = oracle.view_filter(ca, cb, pts)
    assert (k_g, c_g, acc_g) == (k_o, c_o, acc_o)
    assert c_o == len(pts) - 10


def test_profiler_times_each_call(pms):
    """The library's per-launch events time every view-filter call as one
    entry under its own name; unknown names are refused."""
    ctx = pms.Context(0)
    pts = torch.zeros((1000, 3), dtype=torch.float64, device="cuda")
    say("profiler entries of the view filter")
    ctx.profile_enable(True)
    for _ in range(3):
        pms.view_filter([0.0, 0.0, 0.0], [1.0, 0.0, 0.0], pts, ctx=ctx)
    n, ms = ctx.profile_read("view_filter")
    assert n == 3 and ms > 0.0
    assert ctx.profile_read("view_filter") == (0, 0.0)
    ctx.profile_enable(False)
    with pytest.raises(pms.PmsError):
        ctx.profile_read("no such kernel")
