"""GPU (HIP, gfx950) vs the FP64 oracle, through the C ABI.

Bars:
* random numbers: bit-identical Philox4x64-10 blocks;
* matching cost on identical hypotheses: |cost_gpu - cost_oracle| <= 1e-4
  per view wherever both sides call the view valid, except views whose patch
  variance lies within a factor 10 of the floor; validity disagreements (a
  float decision at the boundary) on at most 0.1% of views;
* one half-sweep from an identical state: the GPU's chosen plane equals the
  oracle's (depth within 1e-4 relative) at >= 99% of pixels, and where it
  differs the oracle scores the GPU's plane within 2e-4 of its own choice
  (a near tie) at all but 0.1% of the sampled pixels, and within 1e-3 at all;
* end to end, at each workload's configured iteration count: >= 99% of
  oracle-valid pixels have GPU depth within 0.5%, and at >= 99.9% of them
  the oracle scores the GPU's plane within 2e-4 of its own choice. Where the
  matching cost is flat, runs whose costs differ by rounding settle on
  different but equally good planes; should a case fall below 99%, it must
  still agree with the oracle at least as well as the oracle agrees with
  itself under independent decision errors of the GPU's measured mean size
  (the oracle's decision-noise hook; see test_oracle_self_agreement.py);
* consistency on identical maps: keep/drop agrees except at <= 0.2% of pixels
  whose errors sit at a threshold.
Sizes cover several 8x8 tiles and ragged edges (W = 200 is not a multiple of
the tile), all three storage types, the full 1920x960 workload on sampled
pixels in the launch configuration the benchmark times, and the full
3840x1920 8-bit workload (6 neighbours, 15x15 sparse patch) on sampled
pixels.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import bearings, gpu_images, oracle_images, random_hypotheses, say, split

pytestmark = pytest.mark.gpu

VAR_FLOOR_MARGIN = 10.0


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


def _poses(w):
    return w.poses[w.ref], [w.poses[i] for i in w.nbrs]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    "box256": dict(family="box_room", W=256, seed=0),
    "box200": dict(family="box_room", W=200, seed=1),
    "hall384": dict(family="hall", W=384, seed=0),
    "court320_u8": dict(family="courtyard", W=320, seed=0),
    "hall384_f16": dict(family="hall", W=384, seed=2, dtype="f16"),
}


def _workload(name):
    c = CASES[name]
    dtype = c.get("dtype")
    w = synth.scaled(c["family"], c["W"], seed=c["seed"], dtype="u8" if "u8" in name else None)
    if dtype == "f16":
        # FP16 storage: both sides see the same (rounded) intensities
        w.images = [a.astype(np.float16) for a in w.images]
        w.dtype = "f16"
    return w


def _oracle_view_images(w):
    if w.dtype == "f16":
        return [a.astype(np.float64) for a in w.images]
    return oracle_images(w)


def test_philox_matches_oracle(pms):
    for key in [(0, 0), (0xDEADBEEFCAFEF00D, 0), (123456789, 987654321)]:
        say(f"philox key={key} n=2^20")
        g = pms.philox_stream(key[0], key[1], 1000, 1 << 20).cpu().numpy().view(np.uint64)
        o = oracle.philox4x64_10_stream(key[0], key[1], 1000, 1 << 20)
        assert np.array_equal(g, o)


def _compare_view_costs(w, imgs64, d, n, pv_g, pv_o, params):
    """Checks per-view costs; returns (max |diff|, p99.9 |diff|)."""
    valid_g = pv_g < 2.0
    valid_o = pv_o < 2.0
    both = valid_g & valid_o
    mismatch = (valid_g != valid_o).mean()
    assert mismatch <= 1e-3, f"validity disagrees on {mismatch:.2%} of views"
    diff = np.abs(pv_g - pv_o)
    over = np.argwhere(both & (diff > 1e-4))
    ref64, nbr64 = split(w, imgs64)
    rp, nps = _poses(w)
    floor = params["ncc_var_floor"]
    for j, y, x in over[:400]:
        R, t = oracle.relative_pose(rp, nps[j])
        _, _, _, vr, vs = oracle.view_cost(ref64, nbr64[j], R, t, params, int(x), int(y),
                                           float(d[y, x]), n[:, y, x].astype(np.float64))
        assert min(vr, vs) < VAR_FLOOR_MARGIN * floor, (
            f"view {j} pixel ({x},{y}): cost gpu {pv_g[j, y, x]:.6f} oracle {pv_o[j, y, x]:.6f}, "
            f"variances {vr:.3g} {vs:.3g}")
    assert len(over) <= 400 or len(over) <= 1e-3 * both.sum()
    d_ok = diff[both]
    return float(d_ok.max()), float(np.quantile(d_ok, 0.999))


@pytest.mark.parametrize("name", list(CASES))
def test_eval_cost_matches_oracle(pms, name):
    w = _workload(name)
    params = dict(w.params)
    d, n = random_hypotheses(w, seed=5)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say(f"eval_cost {name} {w.W}x{w.H} dtype={w.dtype}")
    cost_g, pv_g = pms.eval_cost(ref, nbrs, rp, nps, params, _t(d), _t(n), per_view=True)
    torch.cuda.synchronize()
    cost_g = cost_g.cpu().numpy().astype(np.float64)
    pv_g = pv_g.cpu().numpy().astype(np.float64)
    imgs64 = _oracle_view_images(w)
    r64, n64 = split(w, imgs64)
    cost_o, pv_o = oracle.eval_cost(r64, n64, rp, nps, params, d.astype(np.float64),
                                    n.astype(np.float64))
    mx, p999 = _compare_view_costs(w, imgs64, d, n, pv_g, pv_o, params)
    print(f"{name}: per-view |diff| max {mx:.2e} p99.9 {p999:.2e}")
    # aggregated cost follows from the per-view ones
    agg_ok = (np.abs(cost_g - cost_o) <= 1e-4) | (np.abs(cost_g - cost_o) > 1e-4) & (
        (pv_g < 2) != (pv_o < 2)).any(0)
    assert agg_ok.mean() >= 0.998
    # invalid band rows are written invalid
    r = (params["patch_size"] - 1) // 2
    assert np.all(cost_g[:r] == 2.0) and np.all(cost_g[w.H - r:] == 2.0)


def _state_from_oracle(w, seed):
    """A float32 state (depth, normal, cost) whose cost is the oracle's."""
    d, n = random_hypotheses(w, seed=seed, gt_mix=0.4)
    imgs64 = _oracle_view_images(w)
    r64, n64 = split(w, imgs64)
    rp, nps = _poses(w)
    cost, _ = oracle.eval_cost(r64, n64, rp, nps, w.params, d.astype(np.float64),
                               n.astype(np.float64))
    return d, n, cost.astype(np.float32)


def _check_halfsweep(pms, w, d, n, c, colour, iteration, pixels):
    params = dict(w.params)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    dg, ng, cg = _t(d.copy()), _t(n.copy()), _t(c.copy())
    pms.halfsweep(ref, nbrs, rp, nps, params, iteration, colour, dg, ng, cg)
    torch.cuda.synchronize()
    dg, ng, cg = dg.cpu().numpy(), ng.cpu().numpy(), cg.cpu().numpy()
    # the other colour is untouched, bit for bit
    yy, xx = np.mgrid[0:w.H, 0:w.W]
    other = ((xx + yy) & 1) != colour
    assert np.array_equal(dg[other], d[other]) and np.array_equal(cg[other], c[other])
    imgs64 = _oracle_view_images(w)
    r64, n64 = split(w, imgs64)
    d64, n64s, c64 = d.astype(np.float64), n.astype(np.float64), c.astype(np.float64)
    same = 0
    gaps = []
    for (y, x) in pixels:
        do, no, co = oracle.update_pixel(r64, n64, rp, nps, params, d64, n64s, c64, iteration, x, y)
        if abs(dg[y, x] - do) <= 1e-4 * do and np.abs(ng[:, y, x] - no).max() <= 1e-4:
            assert abs(cg[y, x] - co) <= 1e-4, (x, y, cg[y, x], co)
            same += 1
            continue
        # different choice: must be a near tie, scored by the oracle
        R = [oracle.relative_pose(rp, p) for p in nps]
        vc = [oracle.view_cost(r64, nb, Rj, tj, params, x, y, float(dg[y, x]),
                               ng[:, y, x].astype(np.float64))[0]
              for nb, (Rj, tj) in zip(n64, R)]
        gaps.append(abs(oracle.aggregate(vc, params["top_k"]) - co))
    gaps = np.array(gaps)
    if len(gaps):
        print(f"{len(gaps)} different choices, oracle cost gap max {gaps.max():.2e}")
        assert (gaps <= 2e-4).sum() >= len(gaps) - max(1, len(pixels) // 1000)
        assert gaps.max() <= 1e-3
    return same / len(pixels)


@pytest.mark.parametrize("name", ["box256", "box200", "hall384", "court320_u8"])
@pytest.mark.parametrize("colour", [0, 1])
def test_halfsweep_matches_oracle_update(pms, name, colour):
    w = _workload(name)
    d, n, c = _state_from_oracle(w, seed=11 + colour)
    r = (w.params["patch_size"] - 1) // 2
    rng = np.random.default_rng(3)
    ys = rng.integers(r, w.H - r, 1500)
    xs = rng.integers(0, w.W // 2, 1500) * 2
    xs = xs + ((ys + colour + xs) & 1)
    pix = sorted(set(zip(ys.tolist(), (xs % w.W).tolist())))
    pix = [(y, x) for y, x in pix if ((x + y) & 1) == colour]
    say(f"halfsweep {name} colour={colour} {len(pix)} sampled pixels")
    frac = _check_halfsweep(pms, w, d, n, c, colour, 3, pix)
    print(f"{name} colour {colour}: identical choice at {frac:.4f}")
    assert frac >= 0.99


@pytest.mark.parametrize("variant", ["top1", "top3", "top4", "eight_views"])
def test_aggregation_variants_match_oracle(pms, variant):
    """Other aggregations: top_k = 1, 3 and 4 of the four views (the pruning
    bound then applies after other numbers of views), and eight views (the
    four neighbours twice: two full rounds of shared view set-ups, top_k 4).
    Per-view and aggregated costs on random hypotheses, then one half-sweep
    from an oracle-scored state at sampled pixels."""
    w = _workload("hall384")
    if variant == "eight_views":
        w.nbrs = list(w.nbrs) * 2
    else:
        w.params = dict(w.params, top_k=int(variant[3:]))
    params = dict(w.params)
    d, n = random_hypotheses(w, seed=51)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say(f"eval_cost hall384 {variant}")
    cost_g, pv_g = pms.eval_cost(ref, nbrs, rp, nps, params, _t(d), _t(n), per_view=True)
    torch.cuda.synchronize()
    cost_g = cost_g.cpu().numpy().astype(np.float64)
    pv_g = pv_g.cpu().numpy().astype(np.float64)
    imgs64 = _oracle_view_images(w)
    r64, n64 = split(w, imgs64)
    cost_o, pv_o = oracle.eval_cost(r64, n64, rp, nps, params, d.astype(np.float64),
                                    n.astype(np.float64))
    _compare_view_costs(w, imgs64, d, n, pv_g, pv_o, params)
    agg_ok = (np.abs(cost_g - cost_o) <= 1e-4) | ((pv_g < 2) != (pv_o < 2)).any(0)
    assert agg_ok.mean() >= 0.998
    dd, nn, cc = _state_from_oracle(w, seed=53)
    r = (params["patch_size"] - 1) // 2
    rng = np.random.default_rng(6)
    ys = rng.integers(r, w.H - r, 600)
    xs = rng.integers(0, w.W // 2, 600) * 2 + (ys & 1)  # colour 0: x + y even
    pix = sorted({(int(y), int(x)) for y, x in zip(ys, xs)})
    say(f"halfsweep hall384 {variant} colour=0 {len(pix)} sampled pixels")
    frac = _check_halfsweep(pms, w, dd, nn, cc, 0, 2, pix)
    print(f"hall384 {variant}: identical choice at {frac:.4f}")
    assert frac >= 0.99


def _e2e(pms, w, params, maps=False):
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say(f"densify {w.name} {w.W}x{w.H} iters={params['iterations']}")
    dg, ngpu, cg = pms.densify(ref, nbrs, rp, nps, params)
    torch.cuda.synchronize()
    r64, n64 = split(w, _oracle_view_images(w))
    do, no, co = oracle.densify(r64, n64, rp, nps, params)
    return dg.cpu().numpy(), ngpu.cpu().numpy(), cg.cpu().numpy(), do, no, co


@pytest.mark.parametrize("name,iters", [("box256", None), ("box200", None), ("hall384", None),
                                        ("court320_u8", None)])
def test_densify_end_to_end_matches_oracle(pms, name, iters):
    w = _workload(name)
    params = dict(w.params)
    if iters:
        params["iterations"] = iters
    dg, ng, cg, do, no, co = _e2e(pms, w, params)
    valid = do > 0
    assert np.array_equal(dg > 0, valid) or ((dg > 0) != valid).mean() < 1e-3
    rel = np.abs(dg[valid] - do[valid]) / do[valid]
    frac = (rel <= 0.005).mean()
    # quality of the GPU's planes by the oracle's own cost: where the cost
    # landscape is flat the two runs settle on different, equally good planes
    r64, n64 = split(w, _oracle_view_images(w))
    rp, nps = _poses(w)
    c_of_gpu, _ = oracle.eval_cost(r64, n64, rp, nps, params, np.where(valid, dg, 0.0).astype(np.float64),
                                   ng.astype(np.float64))
    worse = (c_of_gpu - co)[valid]
    print(f"{name}: {frac:.4f} of oracle-valid pixels within 0.5% (median rel {np.median(rel):.2e}); "
          f"GPU planes worse than the oracle's by > 2e-4 of its cost at {(worse > 2e-4).mean():.4f}")
    assert (worse <= 2e-4).mean() >= 0.999
    if frac < 0.99:
        # Below 99% only where the oracle itself moves as far: rerun it with
        # independent decision errors, uniform on [-a, a] with the mean size
        # of the GPU's measured cost error (a = 2 x mean), and require the
        # GPU to agree at least as well as the oracle agrees with itself.
        e = np.abs(cg - c_of_gpu)[valid & (dg > 0) & (c_of_gpu < 2)]
        a = 2.0 * float(e.mean())
        oracle.set_decision_noise(a)
        try:
            d_self = oracle.densify(r64, n64, rp, nps, params)[0]
        finally:
            oracle.set_decision_noise(0.0)
        self_frac = (np.abs(d_self[valid] - do[valid]) <= 0.005 * do[valid]).mean()
        print(f"{name}: oracle vs itself under {a:.2e} decision noise: {self_frac:.4f}")
        assert frac >= self_frac
        assert frac >= 0.98
    # invalid encoding outside the band
    r = (params["patch_size"] - 1) // 2
    assert np.all(dg[:r] == 0) and np.all(cg[:r] == 2.0) and np.all(ng[:, :r] == 0)


@pytest.mark.parametrize("name,lanes", [("hall384", 2), ("court320_u8", 8)])
def test_lane_variants_match_oracle(pms, name, lanes):
    """The 2- and 8-lanes-per-pixel variants (for 36- and 64-sample patches,
    chosen by the context's schedule) against the oracle: per-view costs on
    identical hypotheses within 1e-4, end-to-end depth within 0.5% at >= 99%
    of oracle-valid pixels, and no tile shape changes their results."""
    w = _workload(name)
    params = dict(w.params, iterations=3)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    ctx = pms.Context(0)
    ctx.set_schedule(wave_rows=8, waves_x=1, lanes_per_pixel=lanes)
    assert ctx.get_schedule()["lanes_per_pixel"] == lanes
    d, n = random_hypotheses(w, seed=5)
    say(f"eval_cost {name} with {lanes} lanes per pixel")
    _, pv_g = pms.eval_cost(ref, nbrs, rp, nps, params, _t(d), _t(n), per_view=True, ctx=ctx)
    torch.cuda.synchronize()
    pv_g = pv_g.cpu().numpy().astype(np.float64)
    imgs64 = _oracle_view_images(w)
    r64, n64 = split(w, imgs64)
    _, pv_o = oracle.eval_cost(r64, n64, rp, nps, params, d.astype(np.float64), n.astype(np.float64))
    mx, p999 = _compare_view_costs(w, imgs64, d, n, pv_g, pv_o, params)
    say(f"densify {name} with {lanes} lanes per pixel, two tile shapes")
    dg = pms.densify(ref, nbrs, rp, nps, params, ctx=ctx)[0]
    ctx.set_schedule(wave_rows=2, waves_x=2, lanes_per_pixel=lanes)
    dg2 = pms.densify(ref, nbrs, rp, nps, params, ctx=ctx)[0]
    torch.cuda.synchronize()
    dg, dg2 = dg.cpu().numpy(), dg2.cpu().numpy()
    assert np.array_equal(dg, dg2)
    do = oracle.densify(r64, n64, rp, nps, params)[0]
    valid = do > 0
    frac = (np.abs(dg[valid] - do[valid]) <= 0.005 * do[valid]).mean()
    print(f"{name}, {lanes} lanes: per-view |diff| max {mx:.2e} p99.9 {p999:.2e}; "
          f"{frac:.4f} of oracle-valid pixels within 0.5%")
    assert frac >= 0.99
    ctx.close()


def test_densify_iterations_zero_is_the_random_init(pms):
    w = _workload("box256")
    params = dict(w.params, iterations=0, seed=42)
    dg, ng, cg, do, no, co = _e2e(pms, w, params)
    valid = do > 0
    # same uniforms => same plane up to float rounding
    assert np.max(np.abs(dg[valid] - do[valid]) / do[valid]) < 1e-5
    assert np.max(np.abs(ng[:, valid] - no[:, valid])) < 1e-5
    assert (np.abs(cg[valid] - co[valid]) <= 1e-4).mean() >= 0.998


def test_densify_is_deterministic(pms):
    w = _workload("box200")
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say("densify twice, bitwise")
    a = [t.cpu().numpy() for t in pms.densify(ref, nbrs, rp, nps, w.params)]
    b = [t.cpu().numpy() for t in pms.densify(ref, nbrs, rp, nps, w.params)]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("name", ["box256", "hall384"])
def test_consistency_matches_oracle(pms, name):
    w = _workload(name)
    params = dict(w.params, geo_px=1.0, geo_rel_depth=0.01)
    gt = w.gt_depth[w.ref].astype(np.float32)
    gn = w.gt_normal[w.ref].astype(np.float32)
    rng = np.random.default_rng(7)
    # ground truth with small noise, so that both sides see errors near the thresholds
    d = (gt * (1 + 0.004 * rng.normal(size=gt.shape))).astype(np.float32)
    c = np.zeros_like(d)
    idx = w.maps if w.maps else w.nbrs
    maps = [w.gt_depth[i].astype(np.float32) for i in idx]
    mposes = [w.poses[i] for i in idx]
    dg, ng, cg = _t(d.copy()), _t(gn.copy()), _t(c.copy())
    say(f"consistency {name}")
    pms.consistency(w.poses[w.ref], [_t(m) for m in maps], mposes, params, dg, ng, cg)
    torch.cuda.synchronize()
    dg = dg.cpu().numpy()
    do, no, co, epx, ed, ag = oracle.consistency(d.astype(np.float64), gn.astype(np.float64),
                                                 c.astype(np.float64), w.poses[w.ref],
                                                 [m.astype(np.float64) for m in maps], mposes,
                                                 params, diagnostics=True)
    kg, ko = dg > 0, do > 0
    mism = kg != ko
    print(f"{name}: kept gpu {kg.mean():.4f} oracle {ko.mean():.4f}, mismatch {mism.mean():.5f}")
    assert 0.05 < ko.mean() < 0.999
    assert mism.mean() <= 2e-3
    # mismatches sit at a threshold for some map
    near = ((np.abs(epx - params["geo_px"]) < 2e-2) | (np.abs(ed - params["geo_rel_depth"]) < 2e-4)
            | (ag < 0)).any(0)
    assert (mism & ~near).mean() <= 5e-4
    assert np.array_equal(dg[kg & ko], d[kg & ko])


# ---------------------------------------------------------------------------
# the full-size workloads: 1920x960 FP32 (the benchmark's, in its launch
# configuration) and 3840x1920 8-bit (6 neighbours, 15x15 sparse patch,
# 10 iterations), on pixels the oracle scores one by one
# ---------------------------------------------------------------------------

FULL = ["hall_1920", "courtyard_3840"]
# every k-th pixel is scored by the oracle in the per-view cost check
FULL_STRIDE = {"hall_1920": 7, "courtyard_3840": 61}
_full_cache = {}


def _full(name):
    if name not in _full_cache:
        _full_cache[name] = synth.workload(name, seed=0)
    return _full_cache[name]


@pytest.mark.parametrize("name", FULL)
def test_full_size_eval_cost_sampled(pms, name):
    w = _full(name)
    params = dict(w.params)
    d, n = random_hypotheses(w, seed=21)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say(f"eval_cost {name} full size")
    cost_g, pv_g = pms.eval_cost(ref, nbrs, rp, nps, params, _t(d), _t(n), per_view=True)
    torch.cuda.synchronize()
    pv_g = pv_g.cpu().numpy().astype(np.float64)
    # the oracle scores every k-th pixel (depth 0 elsewhere => skipped)
    mask = np.zeros((w.H, w.W), dtype=bool)
    mask.reshape(-1)[::FULL_STRIDE[name]] = True
    d_s = np.where(mask, d, 0.0)
    r64, n64 = split(w, oracle_images(w))
    _, pv_o = oracle.eval_cost(r64, n64, rp, nps, params, d_s, n.astype(np.float64))
    pv_gs = np.where(mask[None], pv_g, 2.0)
    assert ((pv_gs < 2) & (pv_o < 2)).sum() > 0.3 * mask.sum() * len(w.nbrs)
    mx, p999 = _compare_view_costs(w, oracle_images(w), d, n, pv_gs, pv_o, params)
    print(f"{name} full size: per-view |diff| max {mx:.2e} p99.9 {p999:.2e}")


@pytest.mark.parametrize("name", FULL)
def test_full_size_halfsweep_sampled(pms, name):
    w = _full(name)
    d, n = random_hypotheses(w, seed=31, gt_mix=0.4)
    rng = np.random.default_rng(4)
    r = (w.params["patch_size"] - 1) // 2
    ys = rng.integers(r, w.H - r, 400)
    xs = rng.integers(0, w.W // 2, 400) * 2 + ((ys + 1) & 1)  # colour 1: x + y odd
    pix = sorted({(int(y), int(x)) for y, x in zip(ys, xs)})
    assert all(((x + y) & 1) == 1 for y, x in pix)
    # the oracle's state cost is needed only where pixels are compared
    c = np.full((w.H, w.W), 2.0, dtype=np.float32)
    r64, n64 = split(w, oracle_images(w))
    rp, nps = _poses(w)
    m = np.zeros((w.H, w.W), dtype=bool)
    for y, x in pix:
        m[y, x] = True
    co, _ = oracle.eval_cost(r64, n64, rp, nps, w.params, np.where(m, d, 0.0).astype(np.float64),
                             n.astype(np.float64))
    c[m] = co[m].astype(np.float32)
    say(f"halfsweep {name} colour=1 {len(pix)} sampled pixels")
    frac = _check_halfsweep(pms, w, d, n, c, 1, 2, pix)
    print(f"{name} full size halfsweep: identical choice at {frac:.4f}")
    assert frac >= 0.99


@pytest.mark.parametrize("name", FULL)
def test_full_size_densify_properties(pms, name):
    w = _full(name)
    params = dict(w.params)
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say(f"densify {name} full size (no consistency)")
    dg, ng, cg = pms.densify(ref, nbrs, rp, nps, params)
    torch.cuda.synchronize()
    d, n, c = dg.cpu().numpy(), ng.cpu().numpy(), cg.cpu().numpy()
    r = (params["patch_size"] - 1) // 2
    band = np.zeros_like(d, dtype=bool)
    band[r:w.H - r] = True
    assert np.all(d[band] >= params["depth_min"]) and np.all(d[band] <= params["depth_max"])
    assert np.all(d[~band] == 0)
    b = bearings(w.W, w.H)
    assert np.abs(np.linalg.norm(n[:, band], axis=0) - 1).max() < 1e-5
    assert np.all((n * b).sum(0)[band] < 0)
    # the stored cost is the oracle's cost of the stored plane (sampled)
    rng = np.random.default_rng(8)
    r64, n64 = split(w, oracle_images(w))
    R = [oracle.relative_pose(rp, p) for p in nps]
    for _ in range(150):
        y, x = int(rng.integers(r, w.H - r)), int(rng.integers(0, w.W))
        vc = [oracle.view_cost(r64, nb, Rj, tj, params, x, y, float(d[y, x]),
                               n[:, y, x].astype(np.float64))[0] for nb, (Rj, tj) in zip(n64, R)]
        co = oracle.aggregate(vc, params["top_k"])
        assert abs(co - c[y, x]) <= 1e-4 or min(vc) >= 2.0 and c[y, x] == 2.0, (x, y, co, c[y, x])
    # accuracy against the rendered ground truth (the courtyard's sky has
    # no surface and is left out)
    gt = w.gt_depth[w.ref]
    rel = np.abs(d - gt) / np.maximum(gt, 1e-6)
    within = (rel[band & (gt > 0)] < 0.01).mean()
    print(f"{name} full size: {within:.3f} of pixels within 1% of ground truth")
    assert within > 0.5


def test_full_size_consistency_sampled(pms):
    """The 3840x1920 consistency step against its four depth maps, on the
    ground truth with small noise (errors near the thresholds): keep/drop
    agrees with the oracle except where an error sits at a threshold."""
    name = "courtyard_3840"
    w = _full(name)
    params = dict(w.params)
    gt = w.gt_depth[w.ref].astype(np.float32)
    gn = w.gt_normal[w.ref].astype(np.float32)
    rng = np.random.default_rng(9)
    d = (gt * (1 + 0.004 * rng.normal(size=gt.shape))).astype(np.float32)
    c = np.zeros_like(d)
    maps = [w.gt_depth[i].astype(np.float32) for i in w.maps]
    mposes = [w.poses[i] for i in w.maps]
    dg, ng, cg = _t(d.copy()), _t(gn.copy()), _t(c.copy())
    say(f"consistency {name} full size, {len(maps)} maps")
    pms.consistency(w.poses[w.ref], [_t(m) for m in maps], mposes, params, dg, ng, cg)
    torch.cuda.synchronize()
    dg = dg.cpu().numpy()
    # the oracle decides every 5th row
    rows = slice(0, w.H, 5)
    dsub = np.zeros_like(d)
    dsub[rows] = d[rows]
    do, _, _, epx, ed, ag = oracle.consistency(dsub.astype(np.float64), gn.astype(np.float64),
                                               c.astype(np.float64), w.poses[w.ref],
                                               [m.astype(np.float64) for m in maps], mposes,
                                               params, diagnostics=True)
    kg, ko = dg[rows] > 0, do[rows] > 0
    mism = kg != ko
    print(f"{name}: kept gpu {kg.mean():.4f} oracle {ko.mean():.4f}, mismatch {mism.mean():.5f}")
    assert 0.05 < ko.mean() < 0.999
    near = ((np.abs(epx[:, rows] - params["geo_px"]) < 2e-2)
            | (np.abs(ed[:, rows] - params["geo_rel_depth"]) < 2e-4) | (ag[:, rows] < 0)).any(0)
    assert (mism & ~near).mean() <= 5e-4
    assert mism.mean() <= 2e-3
    assert np.array_equal(dg[rows][kg & ko], d[rows][kg & ko])


@pytest.mark.parametrize("name", ["hall384", "box200"])
def test_cost_does_not_depend_on_wave_mates(pms, name):
    """Grazing planes at odd columns warp their patches far from the anchor
    and push their waves onto the general angle form; the costs at the even
    columns (untouched hypotheses) must come out bit for bit the same."""
    w = _workload(name)
    params = dict(w.params)
    d, n = random_hypotheses(w, seed=41, gt_mix=0.8)
    b = bearings(w.W, w.H).astype(np.float32)
    rng = np.random.default_rng(42)
    side = np.cross(b, rng.normal(size=3)[:, None, None], axis=0)
    side /= np.linalg.norm(side, axis=0)
    graze = (-0.02 * b + side).astype(np.float32)
    graze /= np.linalg.norm(graze, axis=0)
    d2, n2 = d.copy(), n.copy()
    n2[:, :, 1::2] = graze[:, :, 1::2]
    imgs = gpu_images(w)
    ref, nbrs = split(w, imgs)
    rp, nps = _poses(w)
    say(f"wave-mate independence {name}")
    c1 = pms.eval_cost(ref, nbrs, rp, nps, params, _t(d), _t(n)).cpu().numpy()
    c2 = pms.eval_cost(ref, nbrs, rp, nps, params, _t(d2), _t(n2)).cpu().numpy()
    assert np.array_equal(c1[:, 0::2], c2[:, 0::2])
    # the grazing planes did change their own costs
    assert not np.array_equal(c1[:, 1::2], c2[:, 1::2])
