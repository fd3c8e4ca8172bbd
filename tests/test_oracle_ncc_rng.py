"""Pins of the oracle's matching cost, view aggregation and random numbers.

* NCC: exact affine identities, a constant patch is invalid, and the cost
  equals 1 - numpy.corrcoef of the exported sample vectors.
* Aggregation: with two views it is the minimum; it is invariant to the
  order of the views; top_k = N is the plain mean.
* Philox4x64-10: the oracle's block function reproduces numpy's Philox bit
  generator (an independent implementation) over 2^20 counters and several
  keys; numpy pre-increments its counter, so block c is numpy's first block
  after setting its counter to c - 1.
"""
import math

import numpy as np
import pytest

import oracle
import synth

W, H = 128, 64


def _identity_view(params, ref, nbr, x, y):
    b = oracle.unproject(W, H, x, y)
    return oracle.view_cost(ref, nbr, np.eye(3), np.zeros(3), params, x, y, 2.0, -b)


@pytest.mark.parametrize("patch", [(7, 1), (11, 2), (15, 2)])
def test_ncc_affine_identities(patch):
    params = synth.params_for("hall", patch_size=patch[0], patch_stride=patch[1])
    rng = np.random.default_rng(20)
    ref = rng.uniform(0.2, 0.8, (H, W))
    for x, y in [(3, 20), (W - 2, 30), (64, 32)]:
        c, *_ = _identity_view(params, ref, 0.3 * ref + 0.1, x, y)
        assert c == pytest.approx(0.0, abs=1e-12)
        c, *_ = _identity_view(params, ref, -2.0 * ref + 1.5, x, y)
        assert c == pytest.approx(2.0, abs=1e-12)
        c, *_ = _identity_view(params, ref, np.full_like(ref, 0.4), x, y)
        assert c == 2.0  # zero variance: invalid view


def test_ncc_matches_numpy_corrcoef(box_room):
    w = box_room
    imgs = w.images_f32()
    params = dict(w.params)
    R, t = oracle.relative_pose(w.poses[w.ref], w.poses[w.nbrs[0]])
    rng = np.random.default_rng(21)
    n_checked = 0
    for _ in range(200):
        x, y = int(rng.integers(0, w.W)), int(rng.integers(3, w.H - 3))
        b = oracle.unproject(w.W, w.H, x, y)
        n = -b + 0.5 * rng.normal(size=3)
        if n @ b >= 0:
            continue
        c, r, s, vr, vs = oracle.view_cost(imgs[w.ref], imgs[w.nbrs[0]], R, t, params, x, y,
                                           rng.uniform(0.5, 5.0), n)
        if np.isnan(s).any():
            assert c == 2.0
            continue
        assert vr == pytest.approx(np.var(r), rel=1e-12)
        assert vs == pytest.approx(np.var(s), rel=1e-12)
        if vr < params["ncc_var_floor"] or vs < params["ncc_var_floor"]:
            assert c == 2.0
            continue
        assert c == pytest.approx(1.0 - np.corrcoef(r, s)[0, 1], abs=1e-12)
        n_checked += 1
    assert n_checked > 50


def test_variance_floor_is_a_strict_threshold():
    params = synth.params_for("box_room")
    dx, dy = oracle.patch_offsets(params)
    ref = np.zeros((H, W))
    x, y = 40, 30
    # the reference patch holds +-a around 0.5 so that its variance is a^2
    signs = np.where((np.arange(len(dx)) % 2) == 0, 1.0, -1.0)
    a = math.sqrt(params["ncc_var_floor"]) * 1.5
    ref[y + dy, (x + dx) % W] = 0.5 + a * signs
    ref_lo = ref.copy()
    ref_lo[y + dy, (x + dx) % W] = 0.5 + 0.5 * a * signs
    c_hi, *_ = _identity_view(params, ref, ref, x, y)
    c_lo, *_ = _identity_view(params, ref_lo, ref_lo, x, y)
    assert c_hi < 1e-9
    assert c_lo == 2.0


def test_aggregate_rules():
    rng = np.random.default_rng(22)
    for _ in range(200):
        v = rng.uniform(0, 2, 2)
        assert oracle.aggregate(v) == min(v)
    for n in range(1, 9):
        v = rng.uniform(0, 2, n)
        k = (n + 1) // 2
        assert oracle.aggregate(v) == pytest.approx(np.sort(v)[:k].mean(), abs=1e-15)
        for _ in range(5):
            assert oracle.aggregate(rng.permutation(v)) == pytest.approx(oracle.aggregate(v), abs=1e-15)
        assert oracle.aggregate(v, top_k=n) == pytest.approx(v.mean(), abs=1e-15)
        assert oracle.aggregate(v, top_k=1) == v.min()
    # an invalid view (cost 2) is dropped when enough valid views remain
    assert oracle.aggregate([2.0, 0.1, 0.3, 2.0]) == pytest.approx(0.2)


def _numpy_blocks(key0, key1, ctr0, n):
    ctr = [(ctr0 - 1) % (1 << 64), 0, 0, 0]
    if ctr0 == 0:  # borrow through all four words
        ctr = [(1 << 64) - 1] * 4
    # uint64 arrays: a plain list would route large keys through float64
    bg = np.random.Philox(key=np.array([key0, key1], dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    return bg.random_raw(4 * n).reshape(n, 4)


@pytest.mark.parametrize("key", [(0, 0), (5, 0), (0xDEADBEEFCAFEF00D, 0), (123456789, 987654321)])
def test_philox_matches_numpy(key):
    n = 1 << 18
    for ctr0 in (0, 1 << 40):
        ours = oracle.philox4x64_10_stream(key[0], key[1], ctr0, n)
        ref = _numpy_blocks(key[0], key[1], ctr0, n)
        assert np.array_equal(ours, ref)


def test_philox_all_counter_words_matter():
    base = oracle.philox4x64_10(7, 0, [11, 22, 33, 44])
    for i in range(4):
        ctr = [11, 22, 33, 44]
        ctr[i] += 1
        other = oracle.philox4x64_10(7, 0, ctr)
        assert all(a != b for a, b in zip(base, other))
    # and numpy agrees on a block with all four words non-zero
    bg = np.random.Philox(key=[7, 0], counter=[10, 22, 33, 44])
    assert list(bg.random_raw(4)) == base


def test_uniforms_are_24_bit_and_in_range():
    seen = []
    for pix in range(2000):
        u = oracle.uniforms(3, pix, 2, 17)
        assert np.all((u >= 0) & (u < 1))
        assert np.all(u * (1 << 24) == np.floor(u * (1 << 24)))
        seen.append(u)
    seen = np.array(seen)
    assert abs(seen.mean() - 0.5) < 0.02
    assert abs(seen.var() - 1 / 12) < 0.01
    blk = oracle.philox4x64_10(3, 0, [1999, 2, 17, 0])
    assert np.array_equal(seen[-1], np.array([w >> 40 for w in blk]) / float(1 << 24))
