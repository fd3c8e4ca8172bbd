"""Shared helpers of the test-suite: feed one seeded workload to both the
HIP path (through the C ABI binding) and the FP64 oracle."""
from __future__ import annotations

import sys

import numpy as np


def say(msg: str) -> None:
    """Names the case before a GPU step, flushed, so a crash log shows it."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_images(w, dtype=None):
    """The workload's keyframe images as device tensors in their storage type."""
    import torch
    out = []
    for a in w.images:
        t = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.cuda())
    return out


def oracle_images(w):
    """Float64 images as the oracle sees them (8-bit scaled by 1/255)."""
    return [np.asarray(a, dtype=np.float64) for a in w.images_f32()]


def split(w, items):
    return items[w.ref], [items[i] for i in w.nbrs]


def bearings(W, H):
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    lam = 2 * np.pi * x / W - np.pi
    phi = np.pi / 2 - np.pi * y / H
    L, P = np.meshgrid(lam, phi)
    return np.stack([np.cos(P) * np.sin(L), -np.sin(P), np.cos(P) * np.cos(L)])


def random_hypotheses(w, seed, gt_mix=0.5):
    """Per-pixel (depth, normal) hypotheses in float32: a mix of perturbed
    ground truth and random planes facing the camera."""
    rng = np.random.default_rng(seed)
    H, W = w.H, w.W
    b = bearings(W, H)
    p = w.params
    gt_d = w.gt_depth[w.ref].astype(np.float64)
    gt_n = w.gt_normal[w.ref].astype(np.float64)
    rnd_d = 1.0 / rng.uniform(1 / p["depth_max"], 1 / p["depth_min"], (H, W))
    rnd_n = rng.normal(size=(3, H, W))
    rnd_n /= np.linalg.norm(rnd_n, axis=0)
    flip = (rnd_n * b).sum(0) > 0
    rnd_n[:, flip] *= -1
    use_gt = (rng.uniform(size=(H, W)) < gt_mix) & (gt_d > 0)
    pert_d = gt_d * (1 + 0.01 * rng.normal(size=(H, W)))
    pert_n = gt_n + 0.05 * rng.normal(size=(3, H, W))
    pert_n /= np.maximum(np.linalg.norm(pert_n, axis=0), 1e-12)
    d = np.where(use_gt, pert_d, rnd_d)
    n = np.where(use_gt[None], pert_n, rnd_n)
    bad = (n * b).sum(0) >= 0
    n[:, bad] = -b[:, bad]
    return d.astype(np.float32), n.astype(np.float32)


def world_points(w, k, n, seed):
    """n world points of keyframe k's rendered surfaces (random pixels with
    ground-truth depth lifted through the camera), float64 (n, 3)."""
    rng = np.random.default_rng(seed)
    d = w.gt_depth[k].astype(np.float64)
    ys, xs = np.nonzero(d > 0)
    pick = rng.choice(len(ys), size=min(n, len(ys)), replace=False)
    b = bearings(w.W, w.H)[:, ys[pick], xs[pick]]
    R, t = w.poses[k]
    R = np.asarray(R, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    X = b * d[ys[pick], xs[pick]]
    return (R.T @ (X - t[:, None])).T


def centre(pose):
    R, t = pose
    return -np.asarray(R, dtype=np.float64).T @ np.asarray(t, dtype=np.float64)


GOLDEN_HALL_1920 = "hall_1920_seed0.npz"


def load_golden_hall_1920():
    """The FP64 oracle's stored run of the 1920x960 hall keyframe (written by
    tests/golden/make_hall_1920.py): (depth before consistency (H, W) float64,
    0 = invalid; cost (H, W) float64; kept-by-consistency mask (H, W) bool;
    meta dict)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", GOLDEN_HALL_1920)
    g = np.load(path, allow_pickle=False)
    meta = json.loads(str(g["meta"]))
    code = g["depth_code"].astype(np.float64)
    dc = meta["depth_code"]
    lo, hi = np.log(dc["d_min"]), np.log(dc["d_max"])
    depth = np.where(code > 0, np.exp(lo + (code - 1.0) / dc["code_max"] * (hi - lo)), 0.0)
    cost = g["cost_code"].astype(np.float64) / 65535.0 * 2.0
    H, W = meta["H"], meta["W"]
    keep = np.unpackbits(g["keep_bits"])[:H * W].reshape(H, W).astype(bool)
    return depth, cost, keep, meta
