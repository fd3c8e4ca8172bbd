#!/usr/bin/env python3
"""Benchmark of the densification hot path on one MI355X.

Workload (hall_1920): one 1920x960 float32 equirectangular keyframe and its
4 neighbours rendered from the seeded procedural hall (box hall, 20 random
spheres and slanted planes, 4-octave value noise), 11x11 patch sampled every
2nd pixel, 8 red-black iterations with 6 refinement trials, 0.3-30 m, then
geometric consistency (1 px, 1%) against the depth maps of the 4 neighbour
keyframes. Those maps are produced first, untimed, by densifying each
neighbour against the other four keyframes of the window.

A step is one full pms_densify call (reference statistics, random
initialisation, 16 half-sweeps, output, consistency) with every input
resident in HBM. Prints ONE JSON line on stdout; progress goes to stderr.

More sections ride on the same line (skip them with --no-next /
--lat-runs 0 / --no-quality / --no-batch / --serve-horizon 0):
* "next_rows": the calls beside densification at the headline's size, each
  timed per call with ms, items/s and achieved GB/s of its algorithmic
  bytes: plane-map warping of the result into a neighbour, the 5x5 median
  post-filter (the median kernel inside a densify call), voxel fusion and
  720x360 coverage of the window's 5 depth maps, and the view filter over
  2^20 sparse points.
* "latency_runs_ms": p50/p99 of 50 single calls of the same keyframe after
  5 untimed ones, each bracketed by HIP events: with every input resident,
  and with the five keyframe images uploaded from pinned host memory
  inside the bracket.
* "quality_3840": the 3840x1920 8-bit courtyard keyframe (6 neighbours,
  15x15 patch sampled every 2nd pixel, 10 iterations, consistency against
  4 maps of its window), timed over --quality-steps densify calls with
  accuracy against the rendered ground truth, then the window's 5 depth
  maps fused into one cloud (2 cm voxels) with its panorama coverage.
* "batch": 32 keyframe jobs (12 at 960x480, 12 at 1920x960, 8 at
  2880x1440, 3-6 neighbours each, hall generator and parameters) with
  FP16 images, as one prepared batch replayed as one HIP graph launch under
  the autotuned tile shape, against the plain FP32 path densifying the same
  32 jobs one by one; accuracy of both against the rendered ground truth per
  resolution class, and their agreement.
* "serving": 8 keyframe streams (Poisson(3/s) each, one width per stream
  from 960/1920/2880, 3-6 neighbours, FP16) through the continuous-batching
  server for --serve-horizon seconds of arrivals. Each stream's keyframes
  are densified in order, each starting from its predecessor's warped
  planes (Sec. III-B) with --serve-warm-iters iterations, and filtered
  against the stream's four previous depth maps. Keyframes/s, p50/p99
  latency from arrival to result, mean batch occupancy, accuracy against
  ground truth beside the plain FP32 path on the same keyframes; three
  served jobs re-run alone must match bit for bit.
* "serving_random_init": the same kind of request stream over
  --serve-random-horizon seconds with random initialisation and the full
  iterations for every keyframe.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "keyframes/s + p50/p99 latency @1920×960, 4 nbrs; NCC evals/s vs roofline"

# Algorithmic VALU work of the dominant kernel (the half-sweep): one NCC
# evaluation = one (pixel, hypothesis, view) patch score of P samples. The
# first-principles estimate: each sample a 3x3 warp, two atan2, a sqrt, the
# pixel map, the bilinear taps with seam wrap and the two-pass sums (76
# lane-slots, +-25%), plus ~30 slots to finish the NCC.
SLOTS_PER_SAMPLE = 76
SLOTS_PER_EVAL = 30
# The same unit re-derived from the compiled gfx950 ISA: its short-form
# sample loop issues 46 VALU instructions a sample (413 for the 9 samples of
# a lane, counted in the compiled half-sweep), 2 of them rcp at half rate:
# 48 slots; per evaluation
# the NCC finish, top-k insertion and LDS read of the view set-up (about 87
# slots) and a quarter of the FP64 view set-up and candidate handling that
# four views share (about 78): 165 slots. The roofline fraction is priced
# this way (the 76-slot estimate exceeds what this ISA needs, so a fraction
# priced by it passes 1 on a fast kernel; it is reported beside it).
ISA_SLOTS_PER_SAMPLE = 48
ISA_SLOTS_PER_EVAL = 165
# Peak: 256 CUs x 64 lanes x 2.4 GHz non-packed FP32 lane-slots.
PEAK_TSLOTS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per updated pixel of a half-sweep: own plane 16 +
# own cost 4 + patch statistics 8 + the opposite colour's plane read once 16
# + write-back of plane and cost 20
HBM_BYTES_PER_UPDATE = 64
# the half-sweep kernel of this workload (FP32 images, 4 lanes and 9 samples
# per lane, every slot filled) as profilers name it
HALFSWEEP_KERNEL = "k_tiles<1, 0, 4, 9, true>"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2211_16266_amd/csrc/pms_kernels.hpp", "paper_2211_16266_amd/csrc/pms.hip")
COUNTER_SUMMARY = "profiles/halfsweep_hall_1920_hbm_counters.md"


def _code_only(src: str) -> str:
    """C++ source without comments and blank runs (string literals kept)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c == '"':
            j = i + 1
            while j < n and src[j] != '"':
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "\n".join(line.rstrip() for line in "".join(out).splitlines() if line.strip())


def kernel_source_hash(read=None) -> str:
    """Hash of the kernel sources' code (comments and blank lines left out,
    so that a comment edit does not void the recorded counters)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(rel)
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def measured_traffic(schedule: dict):
    """HBM bytes per half-sweep launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when the summary is missing or
    was taken on other kernel sources."""
    want = [schedule["wave_rows"], schedule["waves_x"]]
    for rec in _traffic_records():
        if rec.get("kernel_sources") == kernel_source_hash() and rec.get("schedule") == want:
            return rec
    return None


def _traffic_records() -> list:
    path = os.path.join(ROOT, COUNTER_SUMMARY)
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return [json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
                for line in f if line.startswith("<!-- traffic ")]


# Host cores the oracle may use: those this process may run on, at most 16
# (a one-GPU host's share of its cores).
HOST_THREADS_MAX = 16


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, HOST_THREADS_MAX))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def valid_pixels(W: int, H: int, params: dict) -> int:
    r = (params["patch_size"] - 1) // 2
    return W * max(0, H - 2 * r)


def patch_samples(params: dict) -> int:
    r = (params["patch_size"] - 1) // 2
    side = 2 * r // params["patch_stride"] + 1
    return side * side


# Cases for the oracle agreement of the benchmark's results: each section
# registers sampled pixels of one keyframe it densified (the images as the
# oracle reads them, poses, parameters, and the GPU's plane and cost there);
# the CPU leg at the end scores those planes with the oracle.
ORACLE_CASES = []
ORACLE_SAMPLES = 4000


def register_oracle_case(name, imgs64, ref, nbrs, poses, params, depth, normal, cost, seed=0):
    """depth/normal/cost: the GPU's outputs as numpy arrays (H, W) / (3, H, W)."""
    H, W = depth.shape
    ys, xs = np.nonzero(depth > 0)
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(ys), size=min(ORACLE_SAMPLES, len(ys)), replace=False)
    ys, xs = ys[pick], xs[pick]
    ORACLE_CASES.append({"name": name, "imgs": [imgs64[ref]] + [imgs64[k] for k in nbrs],
                         "poses": [poses[ref]] + [poses[k] for k in nbrs], "params": dict(params),
                         "ys": ys, "xs": xs, "shape": (H, W), "depth": depth[ys, xs],
                         "normal": normal[:, ys, xs], "cost": cost[ys, xs]})


def oracle_agreement(threads: int) -> dict:
    """The FP64 oracle's cost of the GPU's plane at each registered case's
    sampled pixels against the cost the GPU stored with it (Sec. III-C: the
    aggregated 1 - NCC)."""
    import oracle
    out = {}
    for c in ORACLE_CASES:
        H, W = c["shape"]
        d = np.zeros((H, W))
        n = np.zeros((3, H, W))
        d[c["ys"], c["xs"]] = c["depth"]
        n[:, c["ys"], c["xs"]] = c["normal"]
        imgs = c["imgs"]
        co, _ = oracle.eval_cost(imgs[0], imgs[1:], c["poses"][0], c["poses"][1:], c["params"], d, n,
                                 n_threads=threads)
        co = co[c["ys"], c["xs"]]
        g = c["cost"].astype(np.float64)
        both = (co < 2) & (g < 2)
        err = np.abs(co - g)[both]
        out[c["name"]] = {"pixels": int(len(g)), "both_valid": int(both.sum()),
                          "validity_differs": int(((co < 2) != (g < 2)).sum()),
                          "cost_err_max": float(err.max()) if err.size else None,
                          "cost_err_p99": float(np.quantile(err, 0.99)) if err.size else None,
                          "within_1e-4": float((err <= 1e-4).mean()) if err.size else None}
    return out


def golden_depth_agreement(depth) -> dict | None:
    """The hall_1920 PatchMatch result (seed 0, no consistency step) against
    the FP64 oracle's stored run of the same inputs (tests/golden)."""
    import json as _json
    path = os.path.join(ROOT, "tests", "golden", "hall_1920_seed0.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    meta = _json.loads(str(g["meta"]))
    code = g["depth_code"].astype(np.float64)
    dc = meta["depth_code"]
    lo, hi = np.log(dc["d_min"]), np.log(dc["d_max"])
    do = np.where(code > 0, np.exp(lo + (code - 1.0) / dc["code_max"] * (hi - lo)), 0.0)
    valid = do > 0
    rel = np.abs(depth[valid] - do[valid]) / do[valid]
    return {"source": "stored FP64 oracle run, tests/golden/hall_1920_seed0.npz",
            "oracle_valid_pixels": int(valid.sum()),
            "within_0.5pct": float((rel <= 0.005).mean()), "within_0.1pct": float((rel <= 0.001).mean()),
            "median_rel_err": float(np.median(rel)), "validity_differs": int(((depth > 0) != valid).sum())}


def cpu_baseline(w, params, budget_s: float, threads: int) -> dict:
    """The oracle, as it stands, on a bounded sample of the same workload:
    red half-sweeps over successive 32-row bands of the same keyframe,
    from planes near the ground truth, until `budget_s` of wall time."""
    import oracle
    imgs = [a.astype(np.float64) for a in w.images_f32()]
    ref, nbrs = imgs[w.ref], [imgs[i] for i in w.nbrs]
    rp, nps = w.poses[w.ref], [w.poses[i] for i in w.nbrs]
    rng = np.random.default_rng(1)
    H, W = w.H, w.W
    gt_d = w.gt_depth[w.ref].astype(np.float64)
    gt_n = w.gt_normal[w.ref].astype(np.float64)
    d = np.clip(gt_d * (1 + 0.02 * rng.normal(size=gt_d.shape)), params["depth_min"],
                params["depth_max"])
    n = gt_n + 0.1 * rng.normal(size=gt_n.shape)
    n /= np.linalg.norm(n, axis=0)
    r = (params["patch_size"] - 1) // 2
    band = 32
    y = H // 2 - 4 * band
    updates = 0
    elapsed = 0.0
    rows = []
    while elapsed < budget_s and y + band <= H - r:
        # the band's stored costs (not timed)
        mask = np.zeros((H, W), dtype=bool)
        mask[y:y + band] = True
        c, _ = oracle.eval_cost(ref, nbrs, rp, nps, params, np.where(mask, d, 0.0), n,
                                n_threads=threads)
        t0 = time.perf_counter()
        oracle.halfsweep_rows(ref, nbrs, rp, nps, params, d, n, c, 1, 0, y, y + band,
                              n_threads=threads)
        elapsed += time.perf_counter() - t0
        updates += band * W // 2
        rows.append(y)
        y += band
    per_update = elapsed / updates
    kf_seconds = per_update * valid_pixels(W, H, params) * (params["iterations"] + 1.0 / 14.0)
    return {"value": 1.0 / kf_seconds, "unit": "keyframes/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "affinity_cores": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "sample": (f"red half-sweeps over rows {rows[0]}-{rows[-1] + band - 1} of the "
                       f"{W}x{H} reference ({updates} pixel updates, {elapsed:.1f} s wall on "
                       f"{threads} threads), scaled by {valid_pixels(W, H, params)} valid pixels "
                       f"x ({params['iterations']} iterations + 1/14 for the initialisation)")}


def _gt_accuracy(depth, gt, r):
    """Completeness (valid fraction of the band) and accuracy (fraction of
    valid pixels within 1% of the ground-truth range) of one depth map."""
    d = depth[r:depth.shape[0] - r]
    g = gt[r:gt.shape[0] - r]
    valid = d > 0
    ok = valid & (g > 0) & (np.abs(d - g) <= 0.01 * np.maximum(g, 1e-9))
    return float(valid.mean()), float(ok.sum() / max(valid.sum(), 1))


def latency_section(args, torch, step, host_imgs, dev_imgs) -> dict:
    """Per-call latency of the headline keyframe on a warm context: --lat-warmup
    untimed and --lat-runs timed calls, each bracketed by events on the
    stream it runs on, first with every input resident in HBM, then with
    the five keyframe images uploaded from pinned host memory inside the
    bracket (the neighbour depth maps stay resident: they are this
    pipeline's own earlier outputs)."""
    stream = torch.cuda.current_stream()

    def runs(upload):
        for _ in range(args.lat_warmup):
            if upload:
                for h, d in zip(host_imgs, dev_imgs):
                    d.copy_(h, non_blocking=True)
            step()
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.lat_runs):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            if upload:
                for h, d in zip(host_imgs, dev_imgs):
                    d.copy_(h, non_blocking=True)
            step()
            b.record(stream)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        ms = np.array(ms)
        return {"runs": len(ms), "p50": float(np.percentile(ms, 50)),
                "p99": float(np.percentile(ms, 99)), "mean": float(ms.mean())}

    log(f"latency: {args.lat_warmup} + {args.lat_runs} calls resident, then with uploads")
    upload_bytes = sum(h.numel() * h.element_size() for h in host_imgs)
    return {"resident": runs(False),
            "with_h2d_upload": dict(runs(True), bytes_uploaded=upload_bytes)}


# every kernel name the library's per-launch events are kept under
PROFILE_NAMES = ("refstats", "init", "halfsweep", "finalize", "consistency", "eval", "io", "batch",
                 "warp", "median", "fuse", "coverage", "view_filter")

# Algorithmic HBM bytes of the calls beside densification, per item: a
# pixel of the 1920x960 map (warp, median), a point of the depth maps
# (fuse, coverage) or a sparse point (view filter).
NEXT_BYTES = {
    # z-buffer clear 8, depth read 4, 64-bit atomic 8, z-buffer read 8,
    # winner's plane gathered 16, plane written 16
    "warp": 60,
    # the plane state read once (16); the window re-reads hit the caches
    "median": 16,
    # table slots of 16 cleared (2^24 for 9.2 M points: 29 per point), depth
    # 4, the slot read by the insertion 16, claimed-slot index written and
    # read 8, keep byte 1 (the claiming points' CAS and atomic min on top)
    "fuse": 58,
    # depth 4, keep byte 1, cover byte 1
    "coverage": 6,
    # one FP64 point 24
    "view_filter": 24,
}


def next_rows_section(args, torch, pms, w, params, out, maps, map_poses, ctx) -> dict:
    """The calls beside densification at the headline's size: plane-map
    warping of the keyframe's result to a neighbour (Sec. III-B), the
    median post-filter inside densify (Sec. III-C), voxel fusion and
    panorama coverage of the window's 5 depth maps, and the view filter
    (Eq. 1) over --vf-points sparse points. Each is timed with the
    library's per-launch events over --next-reps calls."""
    dev = out[0].device
    H, W = out[0].shape
    reps = max(1, args.next_reps)
    res = {}

    def timed(name, call, items, unit):
        call()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        ctx.profile_read(name)
        for _ in range(reps):
            call()
        n, ms = ctx.profile_read(name)
        ctx.profile_enable(False)
        for other in PROFILE_NAMES:
            ctx.profile_read(other)  # the rest of a densify call's launches
        per = ms / max(n, 1)
        gbs = items * NEXT_BYTES[name] / (per * 1e-3) / 1e9
        res[name] = {"ms_per_call": per, "calls": n, f"{unit}_per_s": items / (per * 1e-3),
                     "algorithmic_bytes_per_item": NEXT_BYTES[name], "achieved_GBs": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS}

    log("next rows: warp, median, fuse, coverage, view filter")
    wo = (torch.empty_like(out[0]), torch.empty_like(out[1]))
    timed("warp", lambda: pms.warp_planes(out[0], out[1], w.poses[w.ref], map_poses[0], params,
                                          out=wo, ctx=ctx), W * H, "pixels")
    res["warp"]["valid_warped_fraction"] = float((wo[0] > 0).float().mean().item())

    imgs = [torch.from_numpy(a).to(dev) for a in w.images]
    ref, nbrs = imgs[w.ref], [imgs[i] for i in w.nbrs]
    mp = dict(params, median_radius=2, median_rel=0.05)
    mo = (torch.empty_like(out[0]), torch.empty_like(out[1]), torch.empty_like(out[2]))
    timed("median", lambda: pms.densify(ref, nbrs, w.poses[w.ref], [w.poses[i] for i in w.nbrs], mp,
                                        out=mo, ctx=ctx), W * H, "pixels")

    depths = [out[0]] + list(maps)
    poses = [w.poses[w.ref]] + list(map_poses)
    kept = {}

    def fuse():
        kept["keep"], kept["n"] = pms.fuse(depths, poses, 0.02, ctx=ctx)

    timed("fuse", fuse, W * H * len(depths), "points")
    res["fuse"]["kept_points"] = kept["n"]
    cov = {}

    def coverage():
        cov["n"], _ = pms.coverage(depths, poses, kept["keep"], w.poses[w.ref], ctx=ctx)

    timed("coverage", coverage, W * H * len(depths), "points")
    res["coverage"]["covered_fraction_720x360"] = cov["n"] / (720 * 360)

    g = torch.Generator(device=dev)
    g.manual_seed(args.seed)
    centres = [-(np.asarray(R).T @ np.asarray(t)) for R, t in (w.poses[w.ref], map_poses[0])]
    pts = (torch.rand((args.vf_points, 3), generator=g, device=dev, dtype=torch.float64) - 0.5) * 30.0
    pts += torch.as_tensor(centres[0], device=dev)
    vf = {}

    def view_filter():
        vf["r"] = pms.view_filter(centres[0], centres[1], pts, ctx=ctx)

    timed("view_filter", view_filter, args.vf_points, "points")
    res["view_filter"]["accepted"], res["view_filter"]["in_range"], res["view_filter"]["counted"] = vf["r"]
    return res


def quality_section(args, torch, pms, synth, ctx) -> dict:
    """The 3840x1920 8-bit courtyard (6 neighbours, 15x15 sparse patch, 10
    iterations, consistency against 4 maps of the window), timed like the
    headline on the same context."""
    log("rendering courtyard_3840 (7 keyframes, 3840x1920, 8-bit)")
    w = synth.workload("courtyard_3840", seed=args.seed)
    params = dict(w.params)
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(a).to(dev) for a in w.images]
    log("densifying its 4 map keyframes (untimed)")
    maps, map_poses = [], []
    for i in w.maps:
        others = [k for k in range(len(w.images)) if k != i]
        d_i, _, _ = pms.densify(imgs[i], [imgs[k] for k in others], w.poses[i],
                                [w.poses[k] for k in others], params, ctx=ctx)
        maps.append(d_i)
        map_poses.append(w.poses[i])
    ref, nbrs = imgs[w.ref], [imgs[i] for i in w.nbrs]
    rp, nps = w.poses[w.ref], [w.poses[i] for i in w.nbrs]
    out = (torch.empty((w.H, w.W), device=dev), torch.empty((3, w.H, w.W), device=dev),
           torch.empty((w.H, w.W), device=dev))

    def step():
        pms.densify(ref, nbrs, rp, nps, params, maps=maps, map_poses=map_poses, out=out, ctx=ctx)

    # 4 or 8 lanes per pixel for the 64-sample patch, under the tile shape
    # already chosen: one untimed and one timed call each, the faster kept
    # (the lane count changes only the order of the patch sums)
    keep_sched = ctx.get_schedule()
    lanes_ms = {}
    for lanes in (4, 8):
        ctx.set_schedule(wave_rows=keep_sched["wave_rows"], waves_x=keep_sched["waves_x"],
                         lanes_per_pixel=lanes)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lanes_ms[lanes] = (time.perf_counter() - t0) * 1e3
    best_lanes = min(lanes_ms, key=lanes_ms.get)
    ctx.set_schedule(wave_rows=keep_sched["wave_rows"], waves_x=keep_sched["waves_x"],
                     lanes_per_pixel=best_lanes)
    log(f"courtyard lanes per pixel: {best_lanes} ({', '.join(f'{k}: {v:.0f} ms' for k, v in lanes_ms.items())})")
    step()
    torch.cuda.synchronize()
    K = max(1, args.quality_steps)
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / K
    # executed work of one more (untimed) step, by the counting half-sweep
    ctx.work_count_enable(True)
    step()
    counts = ctx.work_count_read()
    ctx.work_count_enable(False)
    hyps = len(params["offsets"]) + params["refine_trials"]
    nominal = counts["pixels"] * hyps * len(w.nbrs)
    P = patch_samples(params)
    r = (params["patch_size"] - 1) // 2
    comp, acc = _gt_accuracy(out[0].cpu().numpy(), w.gt_depth[w.ref], r)
    register_oracle_case("courtyard_3840", [np.asarray(a, dtype=np.float64) for a in w.images_f32()],
                         w.ref, w.nbrs, w.poses, params, *(t.cpu().numpy() for t in out))
    # fusion of the window's 5 depth maps (the filtered keyframe and its 4
    # map keyframes) into one de-duplicated cloud, and its panorama coverage
    depths, poses = [out[0]] + maps, [rp] + map_poses
    ctx.profile_enable(True)
    for name in ("fuse", "coverage"):
        ctx.profile_read(name)
    keep, n_kept = pms.fuse(depths, poses, 0.02, ctx=ctx)
    n_cov, _ = pms.coverage(depths, poses, keep, rp, ctx=ctx)
    (_, fuse_ms), (_, cov_ms) = ctx.profile_read("fuse"), ctx.profile_read("coverage")
    ctx.profile_enable(False)
    for name in PROFILE_NAMES:
        ctx.profile_read(name)
    n_pts = int(sum(int((d > 0).sum().item()) for d in depths))
    res = {"workload": "courtyard_3840: 3840x1920 u8, 6 neighbours, 15x15/2 (64 samples), "
                        "10 iterations, consistency vs 4 maps, fusion of the window's 5 maps",
            "keyframes_per_s": 1.0 / t, "ms_per_keyframe": t * 1e3, "steps": K,
            "schedule": ctx.get_schedule(), "lanes_per_pixel_ms": lanes_ms,
            "completeness": comp, "within_1pct_of_gt": acc,
            "executed": {"ncc_evals_per_keyframe": counts["view_evals"],
                         "executed_of_nominal": counts["view_evals"] / max(nominal, 1),
                         "samples_per_keyframe": counts["view_evals"] * P,
                         "ncc_evals_per_s": counts["view_evals"] / t,
                         # whole keyframe time, priced like the headline's roofline
                         "valu_frac_isa_pricing": counts["view_evals"] * (P * ISA_SLOTS_PER_SAMPLE + ISA_SLOTS_PER_EVAL)
                                                  / t / 1e12 / PEAK_TSLOTS,
                         "counts_per_keyframe": counts},
            "fusion": {"maps": len(depths), "valid_points": n_pts, "voxel_m": 0.02,
                       "kept_points": n_kept, "fuse_ms": fuse_ms, "coverage_ms": cov_ms,
                       "covered_fraction_720x360": n_cov / (720 * 360)}}
    ctx.set_schedule(**keep_sched)
    return res


def batch_section(args, torch, pms, synth, pool, ctx) -> dict:
    """32 uneven FP16 jobs as one graph launch vs the plain FP32 path."""
    dev = torch.device("cuda:0")
    mix = synth.mixed_jobs({960: 12, 1920: 12, 2880: 8}, seed=args.seed)
    # FP32 renders for the plain path, the same rounded to FP16 for the batch
    imgs32 = {W: [torch.from_numpy(a).to(dev) for a in w.images] for W, w in pool.items()}
    imgs16 = {W: [t.half() for t in ts] for W, ts in imgs32.items()}
    imgs16_np = {W: [t.cpu().numpy() for t in ts] for W, ts in imgs16.items()}

    def jobs_for(imgs):
        out = []
        for mj in mix:
            w = pool[mj.W]
            params = dict(w.params, seed=mj.seed)
            out.append(pms.job(imgs[mj.W][mj.ref], [imgs[mj.W][k] for k in mj.nbrs],
                               w.poses[mj.ref], [w.poses[k] for k in mj.nbrs], params))
        return out

    jobs16 = jobs_for(imgs16)
    tune_ctx = pms.Context(0)
    tune_set = [next(j for j, m in zip(jobs16, mix) if m.W == W) for W in (960, 1920, 2880)]
    log("autotuning tile shapes on one job per width")
    best, best_ms = tune_ctx.autotune(tune_set, reps=1)
    log(f"autotuned schedule {best} ({best_ms:.1f} ms of init + half-sweeps)")
    batch = pms.Batch(jobs16, ctx=tune_ctx)
    log(f"batch of {len(jobs16)} jobs, {batch.nbytes / 2**30:.2f} GiB of device memory")
    batch.run(graph=True)
    torch.cuda.synchronize()
    K = max(1, args.batch_reps)
    t0 = time.perf_counter()
    for _ in range(K):
        batch.run(graph=True)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / K

    def one_by_one(jobs):
        for jd in jobs[:2]:
            pms.densify(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params, out=jd.out, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for jd in jobs:
            pms.densify(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params, out=jd.out, ctx=ctx)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # the plain FP32 form: the same jobs, FP32 images, one pms_densify each
    jobs32 = jobs_for(imgs32)
    t_plain = one_by_one(jobs32)
    # FP16 images one job at a time (separates storage from batching)
    t_plain16 = one_by_one(jobs_for(imgs16))

    per_class = {}
    for W in (960, 1920, 2880):
        sel = [k for k, m in enumerate(mix) if m.W == W]
        r = (pool[W].params["patch_size"] - 1) // 2
        c16, a16, c32, a32, agree = [], [], [], [], []
        for k in sel:
            gt = pool[W].gt_depth[mix[k].ref]
            d16 = jobs16[k].out[0].cpu().numpy()
            d32 = jobs32[k].out[0].cpu().numpy()
            c, a = _gt_accuracy(d16, gt, r)
            c16.append(c)
            a16.append(a)
            c, a = _gt_accuracy(d32, gt, r)
            c32.append(c)
            a32.append(a)
            both = (d16 > 0) & (d32 > 0)
            agree.append(float((np.abs(d16[both] - d32[both]) <= 0.005 * d32[both]).mean()))
        k0 = sel[0]
        register_oracle_case(f"batch_fp16_{W}x{W // 2}",
                             [np.asarray(a, dtype=np.float64) for a in imgs16_np[W]], mix[k0].ref,
                             mix[k0].nbrs, pool[W].poses, jobs16[k0].params,
                             *(t.cpu().numpy() for t in jobs16[k0].out))
        per_class[f"{W}x{W // 2}"] = {
            "jobs": len(sel),
            "fp16_batch": {"completeness": float(np.mean(c16)), "within_1pct_of_gt": float(np.mean(a16))},
            "fp32_plain": {"completeness": float(np.mean(c32)), "within_1pct_of_gt": float(np.mean(a32))},
            "fp16_vs_fp32_within_0.5pct": float(np.mean(agree)),
        }
    batch.close()

    # where batching pays: keyframes too small to fill the GPU alone
    small_pool = synth.mixed_pool(seed=args.seed + 1, widths=(480,), dtype="f32")
    small_mix = synth.mixed_jobs({480: 32}, seed=args.seed + 1)
    s32 = {480: [torch.from_numpy(a).to(dev) for a in small_pool[480].images]}
    s16 = {480: [t.half() for t in s32[480]]}

    def small_jobs(imgs):
        out = []
        for mj in small_mix:
            w = small_pool[480]
            out.append(pms.job(imgs[480][mj.ref], [imgs[480][k] for k in mj.nbrs], w.poses[mj.ref],
                               [w.poses[k] for k in mj.nbrs], dict(w.params, seed=mj.seed)))
        return out

    small_batch = pms.Batch(small_jobs(s16), ctx=tune_ctx)
    small_batch.run(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        small_batch.run(graph=True)
    torch.cuda.synchronize()
    t_small_batch = (time.perf_counter() - t0) / K
    small_batch.close()
    t_small_plain = one_by_one(small_jobs(s32))
    tune_ctx.close()
    n = len(mix)
    return {"workload": "32 jobs: 12@960x480, 12@1920x960, 8@2880x1440, N~U{3..6}",
            "dtype": "f16 images, f32 accumulation",
            "launch": "one HIP graph launch per batch",
            "schedule": best,
            "keyframes_per_s": n / t_batch, "s_per_batch": t_batch,
            "plain_fp32_keyframes_per_s": n / t_plain, "plain_fp32_s": t_plain,
            "plain_fp16_keyframes_per_s": n / t_plain16,
            "speedup_vs_plain_fp32": t_plain / t_batch,
            "accuracy_per_class": per_class,
            "small_keyframes": {"workload": "32 jobs at 480x240, N~U{3..6}",
                                "batched_fp16_keyframes_per_s": 32 / t_small_batch,
                                "plain_fp32_keyframes_per_s": 32 / t_small_plain,
                                "speedup": t_small_plain / t_small_batch}}


def serving_section(args, torch, pms, synth, pool, ctx, warm: bool, horizon: float,
                    rate: float | None = None, light: bool = False) -> dict:
    """Keyframe streams through the continuous-batching server.

    warm: each stream is one camera with one resolution (drawn per stream),
    walking its window; a keyframe whose stream predecessor is already done
    starts from the predecessor's planes carried over by plane-map warping
    (Sec. III-B) and runs --serve-warm-iters iterations, and each is filtered
    against its stream's four previous depth maps.
    not warm (the serving configuration as specified): every keyframe draws
    its resolution and reference uniformly and starts from random planes
    with the full iterations.
    Accuracy against the rendered ground truth is measured on every 8th
    served keyframe (fewer past 360 requests, about 45 in all) and on the same
    keyframes densified by the plain FP32 path with the full iterations;
    `light` skips that and the solo re-runs (rate sweep points)."""
    rate = args.serve_rate if rate is None else rate
    from paper_2211_16266_amd import serving
    dev = torch.device("cuda:0")
    imgs32 = {W: [torch.from_numpy(a).to(dev) for a in w.images] for W, w in pool.items()}
    imgs16 = {W: [t.half() for t in ts] for W, ts in imgs32.items()}
    if warm:
        reqs = synth.stream_requests(args.serve_streams, rate, horizon, seed=args.seed + 7)
    else:
        # (time, stream, position in the arrival order, job): a resolution per keyframe
        reqs = [(t, st, i, mj) for i, (t, st, mj) in
                enumerate(synth.poisson_requests(args.serve_streams, rate, horizon, seed=args.seed + 7))]
    warp_ctx = pms.Context(0)
    server = pms.Server(int(args.serve_arena_gib * 2**30), max_jobs=args.serve_max_jobs,
                        ctx=pms.Context(0))
    latest = {}   # stream -> (k, width, keyframe, depth, normal) of its newest finished keyframe
    count = {"warm": 0, "cold": 0}
    # about 45 keyframes are checked whatever the horizon
    sample_every = max(8, len(reqs) // 45)
    samples = []  # (MixedJob, warm, outputs)

    def factory(i, s, k, mj):
        def make():
            w = pool[mj.W]
            prev = latest.get(s)
            init, iters = None, w.params["iterations"]
            if warm and prev is not None and prev[0] == k - 1:
                _, _, pref, pd, pn = prev
                init = pms.warp_planes(pd, pn, w.poses[pref], w.poses[mj.ref], w.params, ctx=warp_ctx)
                iters = args.serve_warm_iters
            count["warm" if init is not None else "cold"] += 1
            params = dict(w.params, seed=mj.seed, iterations=iters)
            jd = pms.job(imgs16[mj.W][mj.ref], [imgs16[mj.W][j] for j in mj.nbrs], w.poses[mj.ref],
                         [w.poses[j] for j in mj.nbrs], params, init=init)
            jd.warm = init is not None
            return jd
        return make

    requests = [serving.Request(t, factory(i, s, k, mj), tag=(i, s, k, mj))
                for i, (t, s, k, mj) in enumerate(reqs)]

    # consistency window: a finished keyframe is filtered against the depth
    # maps of its stream's four predecessors once they are all done (the
    # paper filters once five depth maps exist); on a copy, so the served
    # maps stay comparable with the plain path
    history = {}  # stream -> {k: (keyframe, depth)}
    filt = {"filtered": 0, "kept": [], "valid": []}
    geo_ctx = pms.Context(0)

    def consistency_window(s, k, mj, jd):
        h = history.setdefault(s, {})
        h[k] = (mj.ref, jd.out[0])
        for old in [j for j in h if j < k - 4]:
            del h[old]
        if not all(j in h for j in range(k - 4, k)):
            return
        w = pool[mj.W]
        d, n, c = (t.clone() for t in jd.out)
        maps = [h[j][1] for j in range(k - 4, k)]
        pms.consistency(w.poses[mj.ref], maps, [w.poses[h[j][0]] for j in range(k - 4, k)],
                        w.params, d, n, c, ctx=geo_ctx)
        filt["filtered"] += 1
        filt["kept"].append((d > 0).sum())
        filt["valid"].append((jd.out[0] > 0).sum())

    def on_done(rq, res):
        i, s, k, mj = rq.tag
        d, n, _ = rq.job.out
        if warm:
            if s not in latest or latest[s][0] < k:
                latest[s] = (k, mj.W, mj.ref, d, n)
            consistency_window(s, k, mj, rq.job)
        if i % sample_every == 0 and not light:
            samples.append((mj, rq.job.warm, rq.job))

    def ready(rq):
        # a keyframe waits for its stream predecessor, whose planes it starts from
        i, s, k, mj = rq.tag
        return k == 0 or (s in latest and latest[s][0] >= k - 1)

    log(f"serving {len(requests)} keyframes from {args.serve_streams} streams at "
        f"{rate}/s each over {horizon:.0f} s "
        f"({'warm starts from the stream predecessor' if warm else 'random initialisation, a resolution per keyframe'})")
    out = serving.run(server, requests, on_done=on_done, log=log, keep_jobs=False,
                      ready=ready if warm else None)
    torch.cuda.synchronize()
    # the same keyframes alone through the same path: bitwise equal
    solo_equal = True
    for mj, _, jd in samples[:3]:
        solo = pms.densify_job(pms.job(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params,
                                       init=jd.init), ctx=server.ctx)
        torch.cuda.synchronize()
        solo_equal &= all(torch.equal(a, b) for a, b in zip(jd.out, solo))
    server.close()

    # accuracy against the ground truth, and the plain FP32 path on the same keyframes
    def gt_acc(depth, mj):
        w = pool[mj.W]
        r = (w.params["patch_size"] - 1) // 2
        return _gt_accuracy(depth.cpu().numpy(), w.gt_depth[mj.ref], r)[1]

    served_acc = [gt_acc(jd.out[0], mj) for mj, _, jd in samples]
    plain_jobs, plain_acc, t_plain = [], [], float("nan")
    for mj, _, _ in samples:
        w = pool[mj.W]
        plain_jobs.append(pms.job(imgs32[mj.W][mj.ref], [imgs32[mj.W][j] for j in mj.nbrs],
                                  w.poses[mj.ref], [w.poses[j] for j in mj.nbrs],
                                  dict(w.params, seed=mj.seed)))
    if plain_jobs:
        for jd in plain_jobs[:2]:
            pms.densify(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params, out=jd.out, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for jd in plain_jobs:
            pms.densify(jd.ref, jd.nbrs, jd.ref_pose, jd.nbr_poses, jd.params, out=jd.out, ctx=ctx)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        plain_acc = [gt_acc(jd.out[0], mj) for (mj, _, _), jd in zip(samples, plain_jobs)]
    warp_ctx.close()
    kept = float(sum(int(t.item()) for t in filt["kept"]))
    valid = float(sum(int(t.item()) for t in filt["valid"]))
    geo_ctx.close()
    offered = args.serve_streams * rate
    widths = "one width per stream" if warm else "a width per keyframe"
    summary = {"workload": f"{args.serve_streams} keyframe streams x Poisson({rate}/s), "
                           f"{widths} from 960/1920/2880, N~U{{3..6}}, f16 images",
            "warm_start": warm, "warm_iterations": args.serve_warm_iters if warm else None,
            "warm_started": count["warm"], "cold_started": count["cold"],
            "horizon_s": horizon, "requests": out["requests"],
            "offered_keyframes_per_s": offered,
            "keyframes_per_s": out["keyframes_per_s"], "wall_s": out["wall_s"],
            "latency_ms": {"p50": out["p50_ms"], "p99": out["p99_ms"], "mean": out["mean_ms"]},
            # without the start-up transient (every stream's first keyframe
            # starts cold at about the same time, and its successors wait)
            "latency_ms_arrivals_after_2s": _late_latency(out["results"], 2.0),
            "mean_batch_occupancy": out["mean_occupancy"], "ticks": out["ticks"],
            "max_jobs": args.serve_max_jobs, "arena_peak_gib": out["arena_peak_bytes"] / 2**30,
            "within_1pct_of_gt": {"served": float(np.mean(served_acc)) if samples else None,
                                  "plain_fp32_full_iterations": float(np.mean(plain_acc)) if samples else None,
                                  "keyframes": len(samples)},
            "plain_fp32_keyframes_per_s_on_those": len(plain_jobs) / t_plain if plain_jobs else None,
            "consistency_window": {"keyframes_filtered": filt["filtered"],
                                   "kept_fraction_of_valid": kept / valid if valid else None},
            "solo_rerun_bitwise_equal": bool(solo_equal), "solo_rerun_checked": min(3, len(samples))}
    if light:
        for k in ("within_1pct_of_gt", "plain_fp32_keyframes_per_s_on_those", "consistency_window",
                  "solo_rerun_bitwise_equal", "solo_rerun_checked"):
            summary.pop(k, None)
    if not warm:
        summary.pop("consistency_window", None)
    return summary


def _late_latency(results, after_s: float) -> dict:
    lat = np.array([r.latency_s for r in results if r.arrival_s >= after_s]) * 1e3
    if lat.size == 0:
        return None
    return {"requests": int(lat.size), "p50": float(np.percentile(lat, 50)),
            "p99": float(np.percentile(lat, 99)), "mean": float(lat.mean())}


def _pmc_per_dispatch(d: str) -> dict:
    """{(file, dispatch): (kernel name, {counter: value summed over its rows})}
    of the rocprofv3 --pmc csv output under `d`."""
    import csv
    import glob
    rows = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            key = (f, r["Dispatch_Id"])
            name, vals = rows.setdefault(key, (r["Kernel_Name"], {}))
            vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return rows


def util_summary(kernel: str, dirs: list) -> str:
    """Markdown table of the per-dispatch means of every counter that
    rocprofv3 --pmc runs (csv, one directory per pass) recorded for the
    dispatches whose kernel name contains `kernel`, and the utilisation
    figures derived from them (256 CUs, 1024 SIMDs, 8 XCDs)."""
    means, n_disp = {}, {}
    for d in dirs:
        vals = [v for name, v in _pmc_per_dispatch(d).values() if kernel in name]
        for c in sorted({c for v in vals for c in v}):
            xs = [v[c] for v in vals if c in v]
            if c == "GRBM_GUI_ACTIVE" and c in means:
                continue
            means[c] = sum(xs) / len(xs)
            n_disp[c] = len(xs)
    lines = ["| counter | per dispatch | dispatches |", "|---|---|---|"]
    lines += [f"| {c} | {v:.4g} | {n_disp[c]} |" for c, v in means.items()]
    m = means
    der = []
    cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
    if cyc:
        der.append(("kernel cycles per XCD (GRBM_GUI_ACTIVE / 8)", f"{cyc:.4g} ({cyc / 2.4e6:.3f} ms at 2.4 GHz)"))

        def add(label, num, den):
            if all(k in m for k in num[1]) and den:
                der.append((label, f"{num[0] / den:.3f}"))
        if "SQ_INSTS_VALU" in m:
            add("VALU issue: SQ_INSTS_VALU x 4 / (1024 SIMDs x cycles)", (m["SQ_INSTS_VALU"] * 4, ["SQ_INSTS_VALU"]), 1024 * cyc)
        if "SQ_ACTIVE_INST_VALU" in m:
            add("VALU active: SQ_ACTIVE_INST_VALU x 4 / (1024 x cycles)", (m["SQ_ACTIVE_INST_VALU"] * 4, []), 1024 * cyc)
            if "SQ_THREAD_CYCLES_VALU" in m:
                add("VALU lane utilisation: SQ_THREAD_CYCLES_VALU / (SQ_ACTIVE_INST_VALU x 64)",
                    (m["SQ_THREAD_CYCLES_VALU"], []), 64 * m["SQ_ACTIVE_INST_VALU"])
        for c, label in (("TA_TA_BUSY_sum", "texture addresser busy"), ("TD_TD_BUSY_sum", "texture data busy"),
                         ("TCP_PENDING_STALL_CYCLES_sum", "L1 pending-miss stall")):
            if c in m:
                der.append((f"{label}: {c} / (256 CUs x cycles)", f"{m[c] / (256 * cyc):.3f}"))
        if "SQ_LDS_IDX_ACTIVE" in m:
            der.append(("LDS indexed-access busy: SQ_LDS_IDX_ACTIVE / (256 x cycles)",
                        f"{m['SQ_LDS_IDX_ACTIVE'] / (256 * cyc):.4f}"))
        if "SQ_LDS_BANK_CONFLICT" in m:
            der.append(("LDS bank-conflict stall: SQ_LDS_BANK_CONFLICT / (256 x cycles)",
                        f"{m['SQ_LDS_BANK_CONFLICT'] / (256 * cyc):.5f}"))
    if "SQ_LDS_BANK_CONFLICT" in m and "SQ_LDS_IDX_ACTIVE" in m and m["SQ_LDS_IDX_ACTIVE"] > m["SQ_LDS_BANK_CONFLICT"]:
        der.append(("LDS conflict cycles per conflict-free LDS cycle: SQ_LDS_BANK_CONFLICT / "
                    "(SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)",
                    f"{m['SQ_LDS_BANK_CONFLICT'] / (m['SQ_LDS_IDX_ACTIVE'] - m['SQ_LDS_BANK_CONFLICT']):.4f}"))
    if "TCP_TOTAL_CACHE_ACCESSES_sum" in m and "SQ_INSTS_VMEM_RD" in m:
        der.append(("L1 lookups per vector load: TCP_TOTAL_CACHE_ACCESSES_sum / SQ_INSTS_VMEM_RD",
                    f"{m['TCP_TOTAL_CACHE_ACCESSES_sum'] / m['SQ_INSTS_VMEM_RD']:.1f}"))
    if "TCP_TCC_READ_REQ_sum" in m and "TCP_TOTAL_CACHE_ACCESSES_sum" in m:
        der.append(("L1 miss fraction: TCP_TCC_READ_REQ_sum / TCP_TOTAL_CACHE_ACCESSES_sum",
                    f"{m['TCP_TCC_READ_REQ_sum'] / m['TCP_TOTAL_CACHE_ACCESSES_sum']:.3f}"))
    if "SQ_WAIT_INST_ANY" in m and "SQ_WAVE_CYCLES" in m:
        der.append(("wave cycles waiting: SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES",
                    f"{m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.3f}"))
    if "SQ_WAVES" in m:
        for c, label in (("SQ_INSTS_VALU", "VALU instructions per wave"), ("SQ_INSTS_VMEM_RD", "vector loads per wave"),
                         ("SQ_INSTS_LDS", "LDS instructions per wave")):
            if c in m:
                der.append((label, f"{m[c] / m['SQ_WAVES']:.0f}"))
    lines += ["", "| derived | value |", "|---|---|"] + [f"| {a} | {b} |" for a, b in der]
    return "\n".join(lines)


def counter_summary(fetch_dir: str, write_dir: str, probe_bytes: int, commands: list,
                    schedule: list) -> str:
    """Writes the HBM traffic summary of the half-sweep kernel from two
    rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; csv) of this benchmark with
    --copy-probe, each counter scaled by what it reads for the probe copy."""
    import csv
    import glob

    def per_dispatch(d, counter):
        rows = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                key = (f, r["Dispatch_Id"])
                name, val = r["Kernel_Name"], float(r["Counter_Value"])
                rows[key] = (name, rows.get(key, (name, 0.0))[1] + val)
        return list(rows.values())

    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = per_dispatch(d, counter)
        hs = [v for n, v in rows if HALFSWEEP_KERNEL in n]
        probe = max(v for n, v in rows if "pms::" not in n)
        out[counter] = {"halfsweep_kib": sum(hs) / len(hs), "dispatches": len(hs),
                        "probe_kib": probe, "scale": probe_bytes / 1024.0 / probe}
    fetch = out["FETCH_SIZE"]["halfsweep_kib"] * out["FETCH_SIZE"]["scale"] * 1024
    write = out["WRITE_SIZE"]["halfsweep_kib"] * out["WRITE_SIZE"]["scale"] * 1024
    rec = {"kernel_sources": kernel_source_hash(), "schedule": schedule,
           "bytes_per_launch": fetch + write,
           "fetch_bytes": fetch, "write_bytes": write,
           "fetch_kib_raw": out["FETCH_SIZE"]["halfsweep_kib"],
           "write_kib_raw": out["WRITE_SIZE"]["halfsweep_kib"],
           "fetch_scale": out["FETCH_SIZE"]["scale"], "write_scale": out["WRITE_SIZE"]["scale"],
           "dispatches": out["FETCH_SIZE"]["dispatches"]}
    block = [
        f"## Tile shape {schedule[0]},{schedule[1]}",
        "",
        *[f"    {c}" for c in commands],
        "",
        "| counter | half-sweep, KiB per dispatch (raw) | probe copy reads | scale | bytes per launch |",
        "|---|---|---|---|---|",
        f"| FETCH_SIZE | {rec['fetch_kib_raw']:.0f} | {out['FETCH_SIZE']['probe_kib']:.0f} KiB for "
        f"{probe_bytes / 1024:.0f} KiB | {rec['fetch_scale']:.3f} | {fetch / 1e6:.1f} MB |",
        f"| WRITE_SIZE | {rec['write_kib_raw']:.0f} | {out['WRITE_SIZE']['probe_kib']:.0f} KiB for "
        f"{probe_bytes / 1024:.0f} KiB | {rec['write_scale']:.3f} | {write / 1e6:.1f} MB |",
        "",
        f"Traffic per half-sweep launch: {(fetch + write) / 1e6:.1f} MB over "
        f"{rec['dispatches']} dispatches; kernel sources {rec['kernel_sources']}.",
        "",
        "<!-- traffic " + json.dumps(rec) + " -->",
        "",
    ]
    # keep the other tile shapes measured on the same kernel sources
    path = os.path.join(ROOT, COUNTER_SUMMARY)
    blocks = {tuple(schedule): block}
    if os.path.exists(path):
        text = open(path).read()
        for part in text.split("\n## Tile shape ")[1:]:
            lines = ("## Tile shape " + part).rstrip("\n").split("\n")
            recs = [json.loads(x[len("<!-- traffic "):].rsplit("-->", 1)[0])
                    for x in lines if x.startswith("<!-- traffic ")]
            if recs and recs[0].get("kernel_sources") == rec["kernel_sources"] \
                    and tuple(recs[0]["schedule"]) != tuple(schedule):
                blocks[tuple(recs[0]["schedule"])] = lines + [""]
    head = [
        "# HBM traffic of the half-sweep kernel, hall_1920 (1920x960, 4 neighbours, 36-sample patch)",
        "",
        "Per tile shape, two rocprofv3 counter runs of the benchmark with a 256 MiB",
        "device copy run once before the timed steps (the probe calibrates each",
        "counter). The benchmark reports the figure of the shape it runs, and only",
        "for the same kernel sources.",
        "",
    ]
    with open(path, "w") as f:
        f.write("\n".join(head + [x for k in sorted(blocks) for x in blocks[k]]))
    return path


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="wall seconds of oracle work for the CPU baseline (0 = skip)")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed FP16 batch section")
    ap.add_argument("--no-quality", action="store_true", help="skip the 3840x1920 8-bit section")
    ap.add_argument("--quality-steps", type=int, default=3)
    ap.add_argument("--lat-runs", type=int, default=50,
                    help="timed calls of the latency section (0 skips it)")
    ap.add_argument("--lat-warmup", type=int, default=5)
    ap.add_argument("--no-next", action="store_true",
                    help="skip the warp / median / fuse / coverage / view-filter timings")
    ap.add_argument("--next-reps", type=int, default=10)
    ap.add_argument("--vf-points", type=int, default=1 << 20)
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shape")
    ap.add_argument("--schedule", default=None, metavar="WAVE_ROWS,WAVES_X",
                    help="use this tile shape instead of autotuning (e.g. 4,2)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-sweep", default="6,12,18",
                    help="offered keyframes/s (all streams) of the random-initialisation rate sweep; "
                         "empty to skip")
    ap.add_argument("--serve-sweep-horizon", type=float, default=10.0)
    ap.add_argument("--serve-horizon", type=float, default=60.0,
                    help="seconds of request arrivals in the serving section (0 = skip)")
    ap.add_argument("--serve-random-horizon", type=float, default=15.0,
                    help="seconds of arrivals of the random-initialisation serving run (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=3.0, help="arrivals per second per stream")
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--serve-max-jobs", type=int, default=8)
    ap.add_argument("--serve-arena-gib", type=float, default=16.0)
    ap.add_argument("--serve-cold", action="store_true",
                    help="serve with random initialisation only (skip the warm-start run)")
    ap.add_argument("--serve-warm-iters", type=int, default=2,
                    help="iterations of a keyframe that starts from its predecessor's warped planes")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="bytes of a plain device-to-device copy run once before the "
                         "timed region, to calibrate HBM byte counters (0 = none)")
    ap.add_argument("--util-summary", nargs="+", metavar="KERNEL_OR_DIR",
                    help="KERNEL DIR...: print the utilisation table of the dispatches of KERNEL from "
                         "rocprofv3 --pmc csv directories (no GPU needed) and exit")
    ap.add_argument("--counter-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "SCHEDULE"),
                    help="write the traffic summary from two rocprofv3 --pmc csv directories "
                         "(no GPU needed) and exit")
    args = ap.parse_args()
    if args.util_summary:
        print(util_summary(args.util_summary[0], args.util_summary[1:]))
        return 0
    if args.counter_summary:
        fetch_dir, write_dir, sched = args.counter_summary
        cmd = ("rocprofv3 --pmc {c} --output-format csv -d gpurun_out/pmc_{c} -o pmc -- python3 "
               "bench.py --steps 2 --warmup 0 --cpu-budget 0 --no-quality --lat-runs 0 --no-next --no-batch --serve-horizon 0 "
               "--copy-probe 268435456 --schedule " + sched)
        print(counter_summary(fetch_dir, write_dir, 268435456,
                              [cmd.format(c="FETCH_SIZE"), cmd.format(c="WRITE_SIZE")],
                              [int(v) for v in sched.split(",")]))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the densifier runs one keyframe job per GPU "
              "and has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import paper_2211_16266_amd as pms
    import synth

    assert torch.cuda.is_available(), "no GPU visible"
    log("rendering hall_1920 (5 keyframes, 1920x960)")
    w = synth.workload("hall_1920", seed=args.seed)
    params = dict(w.params)
    N = len(w.nbrs)
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(a).to(dev) for a in w.images]
    ctx = pms.Context(0)

    # consistency maps: every neighbour densified against the rest of the window
    log("densifying the 4 neighbour keyframes for their depth maps (untimed)")
    maps, map_poses = [], []
    window = [w.ref] + list(w.nbrs)
    for i in w.maps:
        others = [k for k in window if k != i]
        d_i, _, _ = pms.densify(imgs[i], [imgs[k] for k in others], w.poses[i],
                                [w.poses[k] for k in others], params, ctx=ctx)
        maps.append(d_i)
        map_poses.append(w.poses[i])
    torch.cuda.synchronize()

    ref, nbrs = imgs[w.ref], [imgs[i] for i in w.nbrs]
    rp, nps = w.poses[w.ref], [w.poses[i] for i in w.nbrs]
    H, W = w.H, w.W
    out = (torch.empty((H, W), device=dev), torch.empty((3, H, W), device=dev),
           torch.empty((H, W), device=dev))

    def step():
        pms.densify(ref, nbrs, rp, nps, params, maps=maps, map_poses=map_poses, out=out, ctx=ctx)

    if args.schedule:
        wr, wx = (int(v) for v in args.schedule.split(","))
        ctx.set_schedule(wave_rows=wr, waves_x=wx)
    schedule = ctx.get_schedule()
    if not args.no_tune and not args.schedule:
        # tile shapes never change a result, only the speed
        log("autotuning the tile shape on this keyframe")
        schedule, tune_ms = ctx.autotune([pms.job(ref, nbrs, rp, nps, params)], reps=1)
        log(f"schedule {schedule}: {tune_ms:.1f} ms of init + half-sweeps")

    if args.copy_probe > 0:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 4} bytes read and {n * 4} bytes written")
        del src, dst

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ctx.profile_enable(True)
    for name in ("halfsweep", "init", "refstats", "finalize", "consistency"):
        ctx.profile_read(name)
    K = args.steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    log(f"timing {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(K):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile_enable(False)
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(K)])
    kern = {name: ctx.profile_read(name)
            for name in ("halfsweep", "init", "refstats", "finalize", "consistency")}
    # the work the half-sweeps actually execute, counted in one more step by
    # the counting variant of the same kernel (same results, not timed)
    log("counting the half-sweeps' executed work (one untimed step)")
    ctx.work_count_enable(True)
    step()
    counts = ctx.work_count_read()
    ctx.work_count_enable(False)
    # the PatchMatch result alone (no consistency step), untimed, for the
    # agreement with the FP64 oracle
    pm = [t.cpu().numpy() for t in pms.densify(ref, nbrs, rp, nps, params, ctx=ctx)]
    golden = golden_depth_agreement(pm[0]) if args.seed == 0 else None
    imgs64 = [np.asarray(a, dtype=np.float64) for a in w.images_f32()]
    register_oracle_case("hall_1920", imgs64, w.ref, w.nbrs, w.poses, params, *pm)

    wall = t1 - t0
    kfps = K / wall
    vpx = valid_pixels(W, H, params)
    P = patch_samples(params)
    hyps = len(params["offsets"]) + params["refine_trials"]
    evals_per_kf = vpx * N * (1 + hyps * params["iterations"])
    n_half, ms_half = kern["halfsweep"]
    avg_half_s = ms_half / max(n_half, 1) / 1e3
    launches_per_step = 2 * params["iterations"]
    # nominal units: every candidate of every updated pixel scored on every view
    nominal_per_launch = (vpx // 2) * hyps * N
    # executed units: the (pixel, candidate, view) evaluations the kernel ran
    evals_per_launch = counts["view_evals"] / launches_per_step
    slots_per_launch = evals_per_launch * (P * ISA_SLOTS_PER_SAMPLE + ISA_SLOTS_PER_EVAL)
    achieved = slots_per_launch / avg_half_s / 1e12
    est_slots_per_launch = evals_per_launch * (P * SLOTS_PER_SAMPLE + SLOTS_PER_EVAL)
    nominal_slots = nominal_per_launch * (P * SLOTS_PER_SAMPLE + SLOTS_PER_EVAL)
    cand = counts["prop_candidates"] + counts["refine_trials"]
    nominal_views = counts["pixels"] * hyps * N
    img_bytes = (N + 1) * W * H * w.images[0].itemsize
    hbm_bytes = (vpx // 2) * HBM_BYTES_PER_UPDATE + img_bytes
    traffic = measured_traffic(schedule)

    result = {
        "metric": METRIC,
        "value": kfps,
        "unit": "keyframes/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural hall rendered in equirectangular; stands in for "
                "the paper's DRZ-hall 360 video)",
        "config": {"workload": "hall_1920", "width": W, "height": H, "n_nbrs": N,
                   "patch": f"{params['patch_size']}x{params['patch_size']}/"
                            f"{params['patch_stride']} ({P} samples)",
                   "iterations": params["iterations"], "refine_trials": params["refine_trials"],
                   "depth_range_m": [params["depth_min"], params["depth_max"]],
                   "consistency_maps": len(maps), "seed": args.seed, "schedule": schedule},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "accuracy": dict(zip(("completeness", "within_1pct_of_gt"),
                             _gt_accuracy(out[0].cpu().numpy(), w.gt_depth[w.ref],
                                          (params["patch_size"] - 1) // 2))),
        "oracle_depth_agreement": golden,
        "ncc_evals_per_s": evals_per_kf * kfps,
        "kernels_ms_per_step": {k: v[1] / K for k, v in kern.items()},
        "roofline": {
            "kernel": "k_halfsweep",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_TSLOTS,
            "unit": "T VALU lane-slots/s",
            "frac": achieved / PEAK_TSLOTS,
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_detail": traffic,
            "avg_launch_ms": avg_half_s * 1e3,
            "launches": n_half,
            "algorithmic_per_launch": {"ncc_evals": evals_per_launch, "samples": evals_per_launch * P,
                                       "slots": slots_per_launch, "hbm_bytes": hbm_bytes,
                                       "unit": "executed (pixel, candidate, view) NCC evaluations"},
            "pricing": {"slots_per_sample": SLOTS_PER_SAMPLE, "slots_per_eval": SLOTS_PER_EVAL,
                        "isa_slots_per_sample": ISA_SLOTS_PER_SAMPLE, "isa_slots_per_eval": ISA_SLOTS_PER_EVAL},
            # the same executed units priced by the 76-slot estimate, and every
            # candidate of every pixel counted as scored on every view
            "estimate_priced_frac": est_slots_per_launch / avg_half_s / 1e12 / PEAK_TSLOTS,
            "contract_frac": nominal_slots / avg_half_s / 1e12 / PEAK_TSLOTS,
            "executed": {
                "ncc_evals_per_launch": evals_per_launch,
                "nominal_ncc_evals_per_launch": nominal_per_launch,
                "executed_of_nominal": counts["view_evals"] / nominal_views,
                "views_pruned_of_nominal": counts["views_pruned"] / nominal_views,
                "candidates_skipped_repeat": counts["skipped_repeat"] / cand,
                "candidates_skipped_geometry": counts["skipped_geometry"] / cand,
                "candidates_facing_rejected": counts["facing_rejects"] / cand,
                "counts_per_step": counts,
            },
            "isa_priced_nominal_frac": nominal_per_launch * (P * ISA_SLOTS_PER_SAMPLE + ISA_SLOTS_PER_EVAL)
                                       / avg_half_s / 1e12 / PEAK_TSLOTS,
            "hbm_achieved_GBs": hbm_bytes / avg_half_s / 1e9,
            "hbm_frac": hbm_bytes / avg_half_s / 1e9 / HBM_PEAK_GBS,
        },
    }
    if not args.no_next:
        result["next_rows"] = next_rows_section(args, torch, pms, w, params, out, maps, map_poses, ctx)
    if args.lat_runs > 0:
        host = [torch.from_numpy(w.images[i]).pin_memory() for i in window]
        result["latency_runs_ms"] = latency_section(args, torch, step, host,
                                                    [imgs[i] for i in window])
    if not args.no_quality:
        result["quality_3840"] = quality_section(args, torch, pms, synth, ctx)
    pool = None
    if not args.no_batch or args.serve_horizon > 0:
        log("rendering the mixed pool (7-keyframe hall windows at 960, 1920, 2880)")
        pool = synth.mixed_pool(seed=args.seed, dtype="f32")
    if not args.no_batch:
        result["batch"] = batch_section(args, torch, pms, synth, pool, ctx)
    if args.serve_horizon > 0:
        result["serving"] = serving_section(args, torch, pms, synth, pool, ctx, warm=not args.serve_cold,
                                            horizon=args.serve_horizon)
        if not args.serve_cold and args.serve_random_horizon > 0:
            result["serving_random_init"] = serving_section(args, torch, pms, synth, pool, ctx,
                                                            warm=False, horizon=args.serve_random_horizon)
        if args.serve_sweep:
            # the random-initialisation form at lower offered rates: where the
            # achieved rate keeps up with the offered one and latency stays flat
            sweep = []
            for total in (float(v) for v in args.serve_sweep.split(",")):
                r = serving_section(args, torch, pms, synth, pool, ctx, warm=False,
                                    horizon=args.serve_sweep_horizon, rate=total / args.serve_streams,
                                    light=True)
                sweep.append({k: r[k] for k in ("offered_keyframes_per_s", "keyframes_per_s", "requests",
                                                "horizon_s", "wall_s", "latency_ms",
                                                "latency_ms_arrivals_after_2s", "mean_batch_occupancy")})
            result["serving_rate_sweep"] = {"init": "random, full iterations, a width per keyframe",
                                            "points": sweep}
    if args.cpu_budget > 0:
        threads = host_threads()
        log(f"cpu baseline: oracle on {threads} threads ({cpu_model()}, nproc {os.cpu_count()}), "
            f"~{args.cpu_budget:.0f} s")
        result["cpu_baseline"] = cpu_baseline(w, params, args.cpu_budget, threads)
        log(f"oracle agreement: the oracle scores the GPU's planes at {ORACLE_SAMPLES} pixels "
            f"of {len(ORACLE_CASES)} keyframes")
        result["oracle_agreement"] = oracle_agreement(threads)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
