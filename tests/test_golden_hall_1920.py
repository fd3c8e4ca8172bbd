"""The stored FP64 oracle run of the 1920x960 hall keyframe
(tests/golden/hall_1920_seed0.npz, written by make_hall_1920.py from the
oracle and the scene renderer only) is current and sound: it was made by the
present oracle and renderer sources with the workload's present parameters,
it decodes to the ground truth's accuracy level, and splitting the
densification into PatchMatch followed by the consistency step (how it is
stored) is what the oracle's densify-with-maps computes."""
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import load_golden_hall_1920, oracle_images, split

HERE = os.path.dirname(os.path.abspath(__file__))


def _maker():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_hall_1920",
                                                  os.path.join(HERE, "golden", "make_hall_1920.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_golden_was_written_by_the_present_sources():
    _, _, _, meta = load_golden_hall_1920()
    assert meta["sources_sha256"] == _maker().source_hash(), (
        "oracle or renderer sources changed since the golden run: rerun tests/golden/make_hall_1920.py")
    p = synth.params_for("hall")
    for k, v in p.items():
        got = meta["params"][k]
        if k == "offsets":
            got = [tuple(o) for o in got]
            v = [tuple(o) for o in v]
        assert got == v, k
    assert (meta["W"], meta["H"]) == (1920, 960)


def test_golden_depth_against_ground_truth():
    depth, cost, keep, meta = load_golden_hall_1920()
    w = synth.workload("hall_1920", seed=0)
    gt = w.gt_depth[w.ref].astype(np.float64)
    r = (meta["params"]["patch_size"] - 1) // 2
    band = np.zeros_like(depth, dtype=bool)
    band[r:meta["H"] - r] = True
    assert np.all(depth[~band] == 0) and np.all(cost[~band] == 2.0)
    valid = depth > 0
    assert valid[band].mean() > 0.98
    assert np.all(keep <= valid)
    rel = np.abs(depth - gt) / np.maximum(gt, 1e-9)
    ok = (rel < 0.01) & valid & (gt > 0)
    within = ok.sum() / (valid & (gt > 0)).sum()
    within_kept = (ok & keep).sum() / (keep & (gt > 0)).sum()
    print(f"oracle hall_1920: {within:.4f} within 1% of ground truth, {within_kept:.4f} after consistency")
    assert within > 0.85 and within_kept > 0.95
    assert 0.7 < keep.mean() < 0.99


def test_densify_with_maps_is_patchmatch_then_consistency():
    w = synth.scaled("hall", 160, seed=0)
    params = dict(w.params, iterations=2)
    r64, n64 = split(w, oracle_images(w))
    rp, nps = w.poses[w.ref], [w.poses[i] for i in w.nbrs]
    maps = [w.gt_depth[i].astype(np.float64) for i in w.maps]
    mposes = [w.poses[i] for i in w.maps]
    d1, n1, c1 = oracle.densify(r64, n64, rp, nps, params, maps=maps, map_poses=mposes)
    d0, n0, c0 = oracle.densify(r64, n64, rp, nps, params)
    d2, n2, c2 = oracle.consistency(d0, n0, c0, rp, maps, mposes, params)
    assert np.array_equal(d1, d2) and np.array_equal(n1, n2) and np.array_equal(c1, c2)
    assert 0 < (d1 > 0).sum() < (d0 > 0).sum()


@pytest.mark.parametrize("vals", [[0.3, 30.0, 1.0, 5.0, 29.99]])
def test_depth_code_round_trip(vals):
    m = _maker()
    d = np.array(vals + [0.0])
    code = m.encode_depth(d, 0.3, 30.0)
    lo, hi = np.log(0.3), np.log(30.0)
    back = np.where(code > 0, np.exp(lo + (code - 1.0) / m.CODE_MAX * (hi - lo)), 0.0)
    assert back[-1] == 0.0 and code[-1] == 0
    assert np.max(np.abs(back[:-1] - d[:-1]) / d[:-1]) <= 3.6e-5
