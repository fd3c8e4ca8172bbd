"""How far the FP64 oracle moves from itself when every cost that enters an
accept decision carries an independent error of the size an FP32
implementation makes: the level of agreement GPU-vs-oracle parity bars can
ask for.

PatchMatch keeps a propagated or refined plane only if its cost is strictly
lower (Sec. III-C). Where the matching cost is flat, two candidates whose
costs differ by less than an implementation's rounding error may be taken in
either order, and a different choice then spreads by propagation. The GPU's
FP32 costs differ from the oracle's FP64 ones by up to a few 1e-7 (the cost
of its final planes: 3.6e-7 at most on the 200 px box room, 3.8e-7 on the
256 px one), by amounts that vary from candidate to candidate. The oracle's
decision-noise hook adds such an independent error, uniform in [-a, a], to
every decision cost. What is pinned here:

* the hook is inert at a = 0 (bit-identical results after it was used);
* on the single-octave box room (7x7 patch, 2 views, 4 iterations), where
  the cost surface is flattest, a = 1e-7 leaves the oracle within 0.5% depth
  of itself at only about 99.1% (200 px) and 99.6% (256 px) of valid pixels.
  The GPU's end-to-end bar of 99% therefore sits at the method's own
  sensitivity to rounding, not below it; on the hall and courtyard scenes the
  GPU agrees at >= 99.8%;
* from an identical state, one half-sweep under a = 4e-7 (the GPU's largest
  measured cost error) picks another plane at about 1% of pixels, and the
  oracle's cost of that plane exceeds the cost of its own choice by more than
  2e-4 at a few pixels in ten thousand, never by 1e-3. That is the rule the
  GPU half-sweep parity test applies (all but 0.1% within 2e-4, all within
  1e-3).

Order-preserving errors do not have this effect: image noise that moves
every view cost by up to 1.6e-5 but alike for neighbouring candidates, or
rounding the state to FP32 between half-sweeps, leave the oracle within 0.5%
at >= 99.98% of pixels; only errors that differ between the candidates of
one decision flip it.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import random_hypotheses, split

CASES = {
    "box256": dict(family="box_room", W=256, seed=0),
    "box200": dict(family="box_room", W=200, seed=1),
}


def _workload(name):
    c = CASES[name]
    return synth.scaled(c["family"], c["W"], seed=c["seed"])


def _inputs(w):
    imgs = [np.asarray(a, dtype=np.float64) for a in w.images_f32()]
    ref, nbrs = split(w, imgs)
    return ref, nbrs, w.poses[w.ref], [w.poses[i] for i in w.nbrs]


@pytest.fixture
def noise_off():
    oracle.set_decision_noise(0.0)
    yield
    oracle.set_decision_noise(0.0)


def test_decision_noise_is_inert_when_off(noise_off):
    w = synth.scaled("box_room", 96, seed=2)
    ref, nbrs, rp, nps = _inputs(w)
    params = dict(w.params, iterations=2)
    d0, n0, c0 = oracle.densify(ref, nbrs, rp, nps, params)
    oracle.set_decision_noise(1e-3)
    d1, _, c1 = oracle.densify(ref, nbrs, rp, nps, params)
    oracle.set_decision_noise(0.0)
    d2, n2, c2 = oracle.densify(ref, nbrs, rp, nps, params)
    assert np.array_equal(d0, d2) and np.array_equal(n0, n2) and np.array_equal(c0, c2)
    valid = d0 > 0
    assert not np.array_equal(c0[valid], c1[valid])  # the hook does act when on


@pytest.mark.slow
@pytest.mark.parametrize("name,lo,hi", [("box200", 0.980, 0.995), ("box256", 0.990, 0.999)])
def test_end_to_end_self_agreement_under_decision_noise(noise_off, name, lo, hi):
    w = _workload(name)
    ref, nbrs, rp, nps = _inputs(w)
    params = dict(w.params)
    assert params["iterations"] == 4
    d0, _, _ = oracle.densify(ref, nbrs, rp, nps, params)
    oracle.set_decision_noise(1e-7)
    d1, _, _ = oracle.densify(ref, nbrs, rp, nps, params)
    valid = d0 > 0
    assert np.array_equal(d1 > 0, valid)
    frac = (np.abs(d1[valid] - d0[valid]) <= 0.005 * d0[valid]).mean()
    print(f"{name}: oracle vs oracle with 1e-7 decision noise: {frac:.4f} within 0.5%")
    assert lo <= frac <= hi


@pytest.mark.slow
def test_halfsweep_tie_rule_is_the_oracles_own(noise_off):
    over_total = 0
    for name in CASES:
        w = _workload(name)
        ref, nbrs, rp, nps = _inputs(w)
        params = dict(w.params)
        r = (params["patch_size"] - 1) // 2
        yy, xx = np.mgrid[0:w.H, 0:w.W]
        for colour in (0, 1):
            d, n = random_hypotheses(w, seed=11 + colour, gt_mix=0.4)
            d, n = d.astype(np.float64), n.astype(np.float64)
            oracle.set_decision_noise(0.0)
            cost, _ = oracle.eval_cost(ref, nbrs, rp, nps, params, d, n)
            cost = cost.astype(np.float32).astype(np.float64)
            d0, n0, c0 = oracle.halfsweep_rows(ref, nbrs, rp, nps, params, d, n, cost, 3, colour, 0, w.H)
            oracle.set_decision_noise(4e-7)
            d1, n1, _ = oracle.halfsweep_rows(ref, nbrs, rp, nps, params, d, n, cost, 3, colour, 0, w.H)
            oracle.set_decision_noise(0.0)
            sel = (((xx + yy) & 1) == colour) & (yy >= r) & (yy <= w.H - 1 - r)
            same = (np.abs(d1 - d0) <= 1e-4 * d0) & (np.abs(n1 - n0).max(0) <= 1e-4)
            differ = sel & ~same
            c_other, _ = oracle.eval_cost(ref, nbrs, rp, nps, params, np.where(differ, d1, 0.0), n1)
            gaps = np.abs(c_other - c0)[differ]
            n_sel = int(sel.sum())
            over = int((gaps > 2e-4).sum())
            print(f"{name} colour {colour}: other plane at {differ.sum() / n_sel:.4f} of pixels, "
                  f"gap > 2e-4 at {over}, max gap {gaps.max() if gaps.size else 0.0:.2e}")
            assert differ.sum() <= 0.02 * n_sel
            assert over <= max(1, n_sel // 1000)
            assert gaps.size == 0 or gaps.max() <= 1e-3
            over_total += over
    # the allowance is used: an exact tie rule would fail the oracle itself
    assert over_total >= 1
