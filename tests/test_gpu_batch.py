"""Batched densification on the GPU, through the C ABI.

* A batch of uneven jobs (sizes, neighbour counts, patch variants, FP32 and
  FP16 storage, with and without consistency maps) gives every job the
  outputs of pms_densify on that job alone, bit for bit.
* The tile shape of the context's schedule never changes a result.
* A prepared batch replayed as one HIP graph launch, with eager work and
  synchronisations between replays, reproduces the eager results every time.
* An FP16 job inside a batch meets the end-to-end bar against the FP64
  oracle on the same (rounded) intensities: >= 99% of oracle-valid pixels
  within 0.5% depth.
"""
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


def _hall(W, seed, f16, nbr_idx=None, **over):
    w = synth.scaled("hall", W, seed=seed, **over)
    if f16:
        w.images = [a.astype(np.float16) for a in w.images]
        w.dtype = "f16"
    if nbr_idx is not None:
        w.nbrs = list(nbr_idx)
    return w


def _tensors(w):
    dt = torch.float16 if w.dtype == "f16" else None
    out = []
    for a in w.images:
        t = torch.from_numpy(np.ascontiguousarray(a))
        out.append((t.to(dt) if dt is not None else t).cuda())
    return out


def _jobs(pms):
    """Four jobs with different sizes, views, variants and storage."""
    specs = []
    # 4 views, FP32, 192 x 96
    w = _hall(192, 0, False)
    specs.append((w, dict(w.params, iterations=3), None))
    # 3 views, FP16, 256 x 128
    w = _hall(256, 1, True, nbr_idx=[1, 3, 4])
    specs.append((w, dict(w.params, iterations=2, seed=7), None))
    # 2 views, 7x7 patch (another kernel variant), FP32, 128 x 64
    w = synth.scaled("box_room", 128, seed=2)
    specs.append((w, dict(w.params, iterations=4), None))
    # 4 views, FP16, 160 x 80, consistency against ground-truth maps
    w = _hall(160, 3, True)
    specs.append((w, dict(w.params, iterations=2), [1, 3]))
    jobs = []
    for w, params, map_idx in specs:
        imgs = _tensors(w)
        maps = [torch.from_numpy(w.gt_depth[i]).cuda() for i in (map_idx or [])]
        jobs.append(pms.job(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                            [w.poses[i] for i in w.nbrs], params, maps=maps,
                            map_poses=[w.poses[i] for i in (map_idx or [])]))
    return jobs


def _alone(pms, jd, ctx):
    return pms.densify(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params, maps=jd.maps,
                       map_poses=jd.map_poses, ctx=ctx)


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_batch_matches_each_job_alone(pms):
    ctx = pms.Context(0)
    jobs = _jobs(pms)
    say("densify 4 jobs alone")
    alone = [_alone(pms, jd, ctx) for jd in jobs]
    say("densify the same 4 jobs as one batch")
    pms.densify_batch(jobs, ctx=ctx)
    torch.cuda.synchronize()
    for k, jd in enumerate(jobs):
        assert _same(jd.out, alone[k]), f"job {k} differs from its solo run"
        kept = (jd.out[0] > 0).float().mean().item()
        print(f"job {k}: {kept:.3f} of pixels valid")
        # the last job is filtered against two ground-truth maps after only
        # two iterations, which keeps fewer pixels
        assert kept > (0.3 if not jd.maps else 0.02)
    # a permuted batch gives the same per-job results
    perm = [2, 0, 3, 1]
    for jd in jobs:
        for t in jd.out:
            t.fill_(-1.0)
    say("densify the batch in another order")
    pms.densify_batch([jobs[k] for k in perm], ctx=ctx)
    torch.cuda.synchronize()
    for k, jd in enumerate(jobs):
        assert _same(jd.out, alone[k]), f"job {k} differs after permutation"
    ctx.close()


@pytest.mark.parametrize("shape", [(1, 4), (16, 1), (2, 2), (8, 4)])
def test_tile_shape_never_changes_results(pms, shape):
    ctx = pms.Context(0)
    jobs = _jobs(pms)[:3]
    say("reference run, default tiles")
    ref = [tuple(t.clone() for t in _alone(pms, jd, ctx)) for jd in jobs]
    ctx.set_schedule(wave_rows=shape[0], waves_x=shape[1])
    assert ctx.get_schedule()["wave_rows"] == shape[0]
    say(f"batch with tiles wave_rows={shape[0]} waves_x={shape[1]}")
    pms.densify_batch(jobs, ctx=ctx)
    torch.cuda.synchronize()
    for k, jd in enumerate(jobs):
        assert _same(jd.out, ref[k]), f"job {k} changed with tile shape {shape}"
    ctx.close()


def test_graph_replays_match_eager(pms):
    ctx = pms.Context(0)
    jobs = _jobs(pms)
    say("eager reference")
    ref = [tuple(t.clone() for t in _alone(pms, jd, ctx)) for jd in jobs]
    torch.cuda.synchronize()
    batch = pms.Batch(jobs, ctx=ctx)
    assert batch.nbytes > 0
    other = jobs[2]
    for rep in range(3):
        for jd in jobs:
            for t in jd.out:
                t.fill_(float("nan"))
        say(f"graph replay {rep}")
        batch.run(graph=True)
        torch.cuda.synchronize()
        for k, jd in enumerate(jobs):
            assert _same(jd.out, ref[k]), f"replay {rep}: job {k} differs from eager"
        # eager work on the same context between replays
        _alone(pms, other, ctx)
        torch.cuda.synchronize()
    say("eager run of the prepared batch")
    batch.run(graph=False)
    torch.cuda.synchronize()
    for k, jd in enumerate(jobs):
        assert _same(jd.out, ref[k])
    batch.close()
    ctx.close()


def test_fp16_job_in_batch_matches_oracle(pms):
    ctx = pms.Context(0)
    w = _hall(192, 5, True)
    params = dict(w.params, iterations=3)
    imgs = _tensors(w)
    jd = pms.job(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                 [w.poses[i] for i in w.nbrs], params)
    filler = _jobs(pms)[2]
    say("FP16 job 192x96 in a batch of two")
    pms.densify_batch([filler, jd], ctx=ctx)
    torch.cuda.synchronize()
    dg = jd.out[0].cpu().numpy()
    f64 = [a.astype(np.float64) for a in w.images]
    do, _, _ = oracle.densify(f64[w.ref], [f64[i] for i in w.nbrs], w.poses[w.ref],
                              [w.poses[i] for i in w.nbrs], params)
    valid = do > 0
    rel = np.abs(dg[valid] - do[valid]) / do[valid]
    frac = (rel <= 0.005).mean()
    print(f"fp16 batch job: {frac:.4f} of oracle-valid pixels within 0.5%")
    assert frac >= 0.99
    ctx.close()


def test_autotune_picks_a_shape_and_keeps_results(pms):
    ctx = pms.Context(0)
    jobs = _jobs(pms)[:2]
    say("reference")
    ref = [tuple(t.clone() for t in _alone(pms, jd, ctx)) for jd in jobs]
    say("autotune over 15 tile shapes")
    best, ms = ctx.autotune(jobs, reps=1)
    assert ms > 0 and best["wave_rows"] in (1, 2, 4, 8, 16) and best["waves_x"] in (1, 2, 4)
    assert ctx.get_schedule() == best
    torch.cuda.synchronize()
    for k, jd in enumerate(jobs):
        assert _same(jd.out, ref[k])
    ctx.close()


def test_full_size_mixed_batch_sampled(pms):
    """One job of each size class of the 32-job mix (960x480, 1920x960 and
    2880x1440 hall windows, FP16 images, 3-6 neighbours), run as one batch
    replayed from a HIP graph, as the benchmark runs the mix: every job
    equals its solo run bit for bit, and at sampled pixels the stored cost
    is the oracle's cost of the stored plane on the same (FP16-rounded)
    intensities; every job finds most of the ground truth."""
    from helpers import bearings
    pool = synth.mixed_pool(seed=0, dtype="f16")
    mix = synth.mixed_jobs({960: 1, 1920: 1, 2880: 1}, seed=5)
    dev = {W: [torch.from_numpy(a).cuda() for a in w.images] for W, w in pool.items()}
    jobs = []
    for mj in mix:
        w = pool[mj.W]
        jobs.append(pms.job(dev[mj.W][mj.ref], [dev[mj.W][k] for k in mj.nbrs], w.poses[mj.ref],
                            [w.poses[k] for k in mj.nbrs], dict(w.params, seed=mj.seed)))
    ctx = pms.Context(0)
    batch = pms.Batch(jobs, ctx=ctx)
    say(f"graph batch of {len(jobs)} full-size FP16 jobs")
    batch.run(graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    for mj, jd in zip(mix, jobs):
        w = pool[mj.W]
        say(f"solo run of the {mj.W}x{mj.W // 2} job, {len(mj.nbrs)} neighbours")
        solo = _alone(pms, jd, ctx)
        torch.cuda.synchronize()
        assert _same(jd.out, solo), f"{mj.W}: batch differs from the solo run"
        d, n, c = (t.cpu().numpy() for t in jd.out)
        params = jd.params
        r = (params["patch_size"] - 1) // 2
        ref64 = w.images[mj.ref].astype(np.float64)
        nb64 = [w.images[k].astype(np.float64) for k in mj.nbrs]
        R = [oracle.relative_pose(w.poses[mj.ref], w.poses[k]) for k in mj.nbrs]
        for _ in range(60):
            y, x = int(rng.integers(r, w.H - r)), int(rng.integers(0, w.W))
            vc = [oracle.view_cost(ref64, nb, Rj, tj, params, x, y, float(d[y, x]),
                                   n[:, y, x].astype(np.float64))[0] for nb, (Rj, tj) in zip(nb64, R)]
            co = oracle.aggregate(vc, params["top_k"])
            assert abs(co - c[y, x]) <= 1e-4 or min(vc) >= 2.0 and c[y, x] == 2.0, (mj.W, x, y, co, c[y, x])
        band = np.zeros_like(d, dtype=bool)
        band[r:w.H - r] = True
        assert np.all((n * bearings(w.W, w.H)).sum(0)[band] < 0)
        gt = w.gt_depth[mj.ref]
        rel = np.abs(d - gt) / np.maximum(gt, 1e-6)
        within = (rel[band & (gt > 0)] < 0.01).mean()
        print(f"{mj.W}: {within:.3f} of pixels within 1% of ground truth")
        assert within > 0.5
    batch.close()
    ctx.close()


def test_autotune_over_lanes_keeps_solo_results(pms):
    """With try_lanes the autotuner also times 2 and 8 lanes per pixel; a
    36-sample and a 64-sample job then give, under the schedule it leaves,
    their solo results bit for bit."""
    ctx = pms.Context(0)
    hall = _hall(192, 0, False)
    court = synth.scaled("courtyard", 192, seed=1)
    jobs = []
    for w in (hall, court):
        imgs = _tensors(w)
        jobs.append(pms.job(imgs[w.ref], [imgs[i] for i in w.nbrs], w.poses[w.ref],
                            [w.poses[i] for i in w.nbrs], dict(w.params, iterations=2)))
    say("autotune over tile shapes and lanes per pixel")
    best, ms = ctx.autotune(jobs, reps=1, try_lanes=True)
    assert ms > 0 and best["lanes_per_pixel"] in (2, 4, 8)
    assert ctx.get_schedule() == best
    # (the outputs hold the last schedule tried; run the batch under the
    # schedule left on the context)
    say(f"batch and solo runs under {best}")
    pms.densify_batch(jobs, ctx=ctx)
    torch.cuda.synchronize()
    tuned = [tuple(t.clone() for t in jd.out) for jd in jobs]
    for k, jd in enumerate(jobs):
        assert _same(_alone(pms, jd, ctx), tuned[k]), f"job {k} differs from its solo run"
    ctx.close()
