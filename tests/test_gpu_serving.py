"""The continuous-batching server on the GPU, through the C ABI.

* Requests that arrive while others are on the GPU are admitted as memory
  frees up, share launches with them, and every result equals that of
  pms_densify on the same job alone, bit for bit (some of them with the
  median post-filter, which the server plans per job).
* Admission respects the arena: with room for about two jobs, no more run
  at once, all finish, and a job larger than the arena is refused at
  submission with PMS_ERR_BUDGET.
"""
import pytest
import torch

import synth
from helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pms():
    import paper_2211_16266_amd as pms
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pms.lib()
    return pms


@pytest.fixture(scope="module")
def pool():
    return synth.mixed_pool(seed=3, widths=(128, 192, 256), dtype="f16")


def _tensors(pool):
    return {W: [torch.from_numpy(a).cuda() for a in w.images] for W, w in pool.items()}


def _jobdesc(pms, pool, dev, mj, iterations, median_radius=0):
    w = pool[mj.W]
    params = dict(w.params, iterations=iterations, seed=mj.seed, median_radius=median_radius)
    imgs = dev[mj.W]
    return pms.job(imgs[mj.ref], [imgs[k] for k in mj.nbrs], w.poses[mj.ref],
                   [w.poses[k] for k in mj.nbrs], params)


def test_served_results_equal_solo_runs(pms, pool):
    from paper_2211_16266_amd import serving
    dev = _tensors(pool)
    ctx = pms.Context(0)
    reqs = synth.poisson_requests(3, 4.0, 3.0, seed=11, widths=(128, 192, 256))[:12]
    assert len(reqs) == 12
    # bursts of four, 20 ms apart: later bursts join jobs still in flight;
    # every third job with the 5x5 median post-filter
    requests = [serving.Request(0.02 * (k // 4), _jobdesc(pms, pool, dev, mj, 2 + (k % 2), 2 if k % 3 == 0 else 0),
                                tag=k)
                for k, (t, s, mj) in enumerate(reqs)]
    server = pms.Server(arena_bytes=64 << 20, max_jobs=8, ctx=ctx)
    say(f"serving {len(requests)} requests")
    done = []
    summary = serving.run(server, requests, on_done=lambda rq, res: done.append(rq.tag))
    torch.cuda.synchronize()
    assert sorted(done) == list(range(len(requests)))
    print(f"served {summary['requests']} in {summary['wall_s']:.2f}s, occupancy "
          f"{summary['mean_occupancy']:.2f}, p50 {summary['p50_ms']:.1f} ms")
    assert summary["mean_occupancy"] > 1.0
    say("solo runs of every served job")
    for rq in requests:
        jd = rq.job
        solo = pms.densify(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params, ctx=ctx)
        torch.cuda.synchronize()
        for a, b in zip(jd.out, solo):
            assert torch.equal(a, b), f"request {rq.tag} differs from its solo run"
    server.close()
    ctx.close()


def test_admission_respects_the_arena(pms, pool):
    dev = _tensors(pool)
    ctx = pms.Context(0)
    W = 256
    H = W // 2
    mjs = [synth.MixedJob(W, 3, [1, 2, 4, 5], seed=k) for k in range(5)]
    state = H * W * (16 + 4 + 8)
    assert pool[W].dtype == "f16"
    pad = (H + 1) * (2 * W + 4) * 8  # re-laid-out copies: 8-byte cells of four FP16 corners
    # the four shared neighbour copies and room for two jobs' state, not three
    arena = int(2.5 * state) + 4 * pad + (64 << 10)
    server = pms.Server(arena_bytes=max(arena, 1 << 20), max_jobs=8, ctx=ctx)
    # a job that can never fit
    big_pool = synth.mixed_pool(seed=4, widths=(512,), dtype="f16")
    big = _jobdesc(pms, big_pool, _tensors(big_pool), synth.MixedJob(512, 3, [1, 2, 4, 5], seed=0), 1)
    with pytest.raises(pms.PmsError) as exc:
        server.submit(big)
    assert exc.value.status == 5
    jds = [_jobdesc(pms, pool, dev, mj, 2) for mj in mjs]
    tickets = [server.submit(jd) for jd in jds]
    max_active = 0
    pending = set(tickets)
    say("stepping 5 jobs through an arena for about two")
    for _ in range(200):
        active, waiting = server.step()
        max_active = max(max_active, active)
        for t in list(pending):
            if server.poll(t) == pms.Server.DONE:
                pending.discard(t)
        if not pending:
            break
    torch.cuda.synchronize()
    assert not pending
    st = server.stats()
    print(f"max active {max_active}, arena peak {st['arena_peak']} of {arena}")
    assert max_active == 2
    assert st["arena_peak"] <= max(arena, 1 << 20)
    for jd in jds:
        assert (jd.out[0] > 0).float().mean() > 0.3
    server.close()
    ctx.close()


def test_served_jobs_with_initial_planes_equal_solo_runs(pms, pool):
    """Jobs that start from warped planes (Sec. III-B) inside the server."""
    from helpers import bearings
    dev = _tensors(pool)
    ctx = pms.Context(0)
    server = pms.Server(arena_bytes=64 << 20, max_jobs=4, ctx=ctx)
    jobs = []
    for W in (128, 192, 256):
        w = pool[W]
        for ref, prev in ((3, 2), (4, 3)):
            d = torch.from_numpy(w.gt_depth[prev]).cuda()
            n = w.gt_normal[prev].copy()
            flip = (n * bearings(w.W, w.H)).sum(0) > 0
            n[:, flip] *= -1
            init = pms.warp_planes(d, torch.from_numpy(n).cuda(), w.poses[prev], w.poses[ref],
                                   w.params, ctx=ctx)
            nb = [k for k in range(7) if k != ref][:4]
            jobs.append(pms.job(dev[W][ref], [dev[W][k] for k in nb], w.poses[ref],
                                [w.poses[k] for k in nb], dict(w.params, iterations=2), init=init))
    say("serving 6 warm-started jobs")
    tickets = [server.submit(jd) for jd in jobs]
    pending = set(tickets)
    for _ in range(100):
        server.step()
        pending = {t for t in pending if server.poll(t) != pms.Server.DONE}
        if not pending:
            break
    torch.cuda.synchronize()
    assert not pending
    for jd in jobs:
        solo = pms.densify_job(pms.job(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params,
                                       init=jd.init), ctx=ctx)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(jd.out, solo))
    server.close()
    ctx.close()
