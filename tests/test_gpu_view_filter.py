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
