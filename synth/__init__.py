"""Seeded synthetic equirectangular workloads (input generator only).

The densifier's GPU path and its CPU oracle both take their inputs from
here: rendered keyframe images, ground-truth range/normal maps, world->camera
poses and the PatchMatch parameters of each named workload. Nothing in this
package performs any step of the densifier itself.

Workloads (all seeded; the scene seed and the PatchMatch seed are separate):

* ``box_room_256`` -- 4x4x3 m box room, 1-octave value noise (cell 0.2 m),
  reference near the centre, 2 neighbours 0.1-0.3 m away in a random
  horizontal direction with random yaw; 256x128 float32, 7x7 patch,
  4 iterations, 0.3-10 m, no consistency.
* ``hall_1920`` -- 24x16x8 m hall with 20 random spheres (r 0.3-2 m) and
  slanted textured planes, 4-octave noise (cell 0.4 m down to 5 cm), five
  keyframes on a smooth Catmull-Rom trajectory at 1.5+-0.5 m height; the
  middle one is the reference, the other four are neighbours (baselines
  0.2-1.0 m) and supply the consistency maps; 1920x960 float32, 11x11 patch
  sampled every 2nd pixel, 8 iterations, 0.3-30 m, 1 px consistency.
* ``courtyard_3840`` -- ground plane and 30 textured boxes under a constant
  sky, seven keyframes 0.5-3 m apart; 3840x1920 8-bit, 15x15 sparse patch,
  10 iterations, 0.3-50 m, consistency over the 5 central keyframes.

``scaled(name, W)`` gives the same scene and parameters at another width,
which the tests use for CPU-sized runs of the large workloads.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")

PRIM_ROOM, PRIM_SPHERE, PRIM_QUAD, PRIM_BOX, PRIM_PLANE = 0, 1, 2, 3, 4
_STRIDE = 16


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC",
                        "-shared", "-pthread", os.path.join(_HERE, "render.c"), "-o", tmp,
                        "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        D = C.POINTER(C.c_double)
        F = C.POINTER(C.c_float)
        L.synth_render.argtypes = [C.c_int, C.c_int, C.c_int, D, D, C.c_int,
                                   C.POINTER(C.c_int32), D, C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.c_uint64, C.c_double, F, F, F, C.c_int]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# scene description
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    types: np.ndarray          # (K,) int32
    prims: np.ndarray          # (K, 16) float64
    n_octaves: int
    base_freq: float
    lo: float = 0.2
    hi: float = 0.8
    tex_seed: int = 0
    sky: float = 0.5


def _prim(kind, *vals):
    row = np.zeros(_STRIDE)
    flat = np.concatenate([np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in vals])
    row[:len(flat)] = flat
    return kind, row


def _scene(prims, **kw) -> Scene:
    return Scene(types=np.array([k for k, _ in prims], dtype=np.int32),
                 prims=np.stack([r for _, r in prims]), **kw)


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def camera_pose(centre, yaw, pitch=0.0, roll=0.0):
    """World->camera (R, t) of a camera at ``centre`` (world frame, y down)
    turned by yaw about the vertical, then pitch and roll."""
    R_cw = rot_y(yaw) @ rot_x(pitch) @ rot_z(roll)
    R = R_cw.T
    t = -R @ np.asarray(centre, dtype=np.float64)
    return R, t


def render(scene: Scene, pose, W: int, H: int, ss: int = 2, with_gt: bool = True,
           n_threads: int = 0):
    """Returns (image float32 (H,W), depth float32 (H,W) or None,
    normal float32 (3,H,W) or None); range/normal at pixel centres, range 0
    where the ray meets no surface."""
    R, t = pose
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(9)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(3)
    img = np.zeros((H, W), dtype=np.float32)
    dep = np.zeros((H, W), dtype=np.float32) if with_gt else None
    nrm = np.zeros((3, H, W), dtype=np.float32) if with_gt else None
    types = np.ascontiguousarray(scene.types, dtype=np.int32)
    prims = np.ascontiguousarray(scene.prims, dtype=np.float64)
    D = C.POINTER(C.c_double)
    F = C.POINTER(C.c_float)
    rc = _L().synth_render(W, H, ss, R.ctypes.data_as(D), t.ctypes.data_as(D), len(types),
                           types.ctypes.data_as(C.POINTER(C.c_int32)), prims.ctypes.data_as(D),
                           scene.n_octaves, scene.base_freq, scene.lo, scene.hi,
                           scene.tex_seed, scene.sky, img.ctypes.data_as(F),
                           dep.ctypes.data_as(F) if with_gt else None,
                           nrm.ctypes.data_as(F) if with_gt else None, int(n_threads))
    if rc:
        raise ValueError("synth_render failed")
    return img, dep, nrm


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    W: int
    H: int
    dtype: str                 # "f32" | "u8" | "f16" -- storage of the images
    images: list               # per keyframe, (H, W) float32 in [0,1] or uint8
    gt_depth: list             # per keyframe, (H, W) float32 range, 0 = no surface
    gt_normal: list            # per keyframe, (3, H, W) float32, camera frame
    poses: list                # per keyframe, (R (3,3), t (3,)) world->camera
    ref: int                   # index of the reference keyframe
    nbrs: list                 # indices of the photometric neighbours
    maps: list                 # indices of the keyframes whose depth maps feed consistency
    params: dict               # PatchMatch parameters (field names of the C structs)

    def images_f32(self):
        """Images as float32 intensities in [0,1] (8-bit scaled by 1/255)."""
        if self.dtype == "u8":
            return [a.astype(np.float32) / np.float32(255.0) for a in self.images]
        return [np.asarray(a, dtype=np.float32) for a in self.images]


BASE_PARAMS = dict(
    patch_size=11, patch_stride=2, iterations=8, refine_trials=6,
    depth_min=0.3, depth_max=30.0, top_k=0, ncc_var_floor=1e-6,
    refine_sigma_logdepth0=0.0, refine_depth_shrink=0.25,
    refine_sigma_normal0=1.0, refine_normal_shrink=0.5,
    offsets=[(-3, 0), (3, 0), (0, -3), (0, 3), (-5, 0), (5, 0), (0, -5), (0, 5)],
    geo_px=1.0, geo_rel_depth=0.01, geo_min_views=0, seed=0,
    median_radius=0, median_rel=0.05,
)


def params_for(name: str, **over) -> dict:
    p = dict(BASE_PARAMS)
    if name.startswith("hall7"):
        name = "hall"
    if name.startswith("box_room"):
        p.update(patch_size=7, patch_stride=1, iterations=4, depth_min=0.3, depth_max=10.0)
    elif name.startswith("hall"):
        p.update(patch_size=11, patch_stride=2, iterations=8, depth_min=0.3, depth_max=30.0,
                 geo_px=1.0)
    elif name.startswith("courtyard"):
        p.update(patch_size=15, patch_stride=2, iterations=10, depth_min=0.3, depth_max=50.0,
                 geo_px=1.0)
    else:
        raise KeyError(name)
    p.update(over)
    return p


def _box_room(rng, W, ss):
    room = _prim(PRIM_ROOM, [-2.0, -3.0, -2.0], [2.0, 0.0, 2.0])
    scene = _scene([room], n_octaves=1, base_freq=5.0, tex_seed=int(rng.integers(1 << 62)))
    c_ref = np.array([rng.uniform(-0.3, 0.3), -1.5 + rng.uniform(-0.2, 0.2), rng.uniform(-0.3, 0.3)])
    poses = [camera_pose(c_ref, rng.uniform(-math.pi, math.pi))]
    for _ in range(2):
        a = rng.uniform(-math.pi, math.pi)
        dist = rng.uniform(0.1, 0.3)
        c = c_ref + dist * np.array([math.cos(a), 0.0, math.sin(a)])
        poses.append(camera_pose(c, rng.uniform(-math.pi, math.pi)))
    return scene, poses, 0, [1, 2], []


def _catmull_rom(pts, n_per_seg=200):
    out = []
    P = np.concatenate([pts[:1], pts, pts[-1:]])
    for i in range(1, len(P) - 2):
        p0, p1, p2, p3 = P[i - 1], P[i], P[i + 1], P[i + 2]
        for s in np.linspace(0.0, 1.0, n_per_seg, endpoint=False):
            s2, s3 = s * s, s * s * s
            out.append(0.5 * ((2 * p1) + (-p0 + p2) * s + (2 * p0 - 5 * p1 + 4 * p2 - p3) * s2
                              + (-p0 + 3 * p1 - 3 * p2 + p3) * s3))
    out.append(P[-2])
    return np.array(out)


def _trajectory_keyframes(rng, n_kf, spacing, xlim, zlim, height, dh):
    way = np.stack([np.linspace(-xlim, xlim, 5) + rng.uniform(-1.0, 1.0, 5),
                    -height + rng.uniform(-dh, dh, 5),
                    rng.uniform(-zlim, zlim, 5)], axis=1)
    path = _catmull_rom(way)
    seg = np.linalg.norm(np.diff(path, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    gaps = rng.uniform(spacing[0], spacing[1], n_kf - 1)
    start = arc[-1] * 0.5 - gaps.sum() * 0.5
    s_kf = start + np.concatenate([[0.0], np.cumsum(gaps)])
    centres, yaws = [], []
    for s in s_kf:
        k = int(np.clip(np.searchsorted(arc, s), 1, len(path) - 1))
        f = (s - arc[k - 1]) / max(arc[k] - arc[k - 1], 1e-12)
        c = path[k - 1] + f * (path[k] - path[k - 1])
        tang = path[k] - path[k - 1]
        centres.append(c)
        yaws.append(math.atan2(tang[0], tang[2]))
    return np.array(centres), np.array(yaws)


def _hall_n(rng, n_kf):
    xlim, ylo, zlim = 12.0, -8.0, 8.0
    centres, yaws = _trajectory_keyframes(rng, n_kf, (0.25, 0.5), 8.0, 4.5, 1.5, 0.5)
    prims = [_prim(PRIM_ROOM, [-xlim, ylo, -zlim], [xlim, 0.0, zlim])]

    def clear(p, radius):
        return np.min(np.linalg.norm(centres - p, axis=1)) > radius + 0.6

    n_sph = 0
    n_quad = 0
    tries = 0
    while n_sph + n_quad < 20 and tries < 10000:
        tries += 1
        if rng.uniform() < 0.5:
            r = rng.uniform(0.3, 2.0)
            c = np.array([rng.uniform(-xlim + r, xlim - r), rng.uniform(ylo + r, -0.2),
                          rng.uniform(-zlim + r, zlim - r)])
            if clear(c, r):
                prims.append(_prim(PRIM_SPHERE, c, [r]))
                n_sph += 1
        else:
            hu, hv = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
            c = np.array([rng.uniform(-xlim + 2, xlim - 2), rng.uniform(-6.0, -0.5),
                          rng.uniform(-zlim + 2, zlim - 2)])
            if clear(c, math.hypot(hu, hv)):
                a = rng.normal(size=3)
                u = a / np.linalg.norm(a)
                b = rng.normal(size=3)
                v = b - u * np.dot(u, b)
                v /= np.linalg.norm(v)
                prims.append(_prim(PRIM_QUAD, c, u, v, [hu, hv]))
                n_quad += 1
    scene = _scene(prims, n_octaves=4, base_freq=2.5, tex_seed=int(rng.integers(1 << 62)))
    poses = [camera_pose(c, y, rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05))
             for c, y in zip(centres, yaws)]
    mid = n_kf // 2
    others = [k for k in range(n_kf) if k != mid]
    return scene, poses, mid, others, others


def _hall(rng, W, ss):
    """Five keyframes; the middle one is the reference."""
    return _hall_n(rng, 5)


def _hall7(rng, W, ss):
    """The same hall generator with seven keyframes (up to six
    neighbours), for the mixed batch and serving workloads."""
    return _hall_n(rng, 7)


def _courtyard(rng, W, ss):
    centres, yaws = _trajectory_keyframes(rng, 7, (0.5, 1.5), 6.0, 3.0, 1.5, 0.0)
    prims = [_prim(PRIM_PLANE, [0.0, 0.0, 0.0], [0.0, -1.0, 0.0])]
    n = 0
    tries = 0
    while n < 30 and tries < 10000:
        tries += 1
        size = rng.uniform(1.0, 6.0, 3)
        size[1] = rng.uniform(1.0, 8.0)
        c = np.array([rng.uniform(-20, 20), 0.0, rng.uniform(-20, 20)])
        lo = np.array([c[0] - size[0] / 2, -size[1], c[2] - size[2] / 2])
        hi = np.array([c[0] + size[0] / 2, 0.0, c[2] + size[2] / 2])
        # keep 1 m between every keyframe centre and the box
        gap = np.max(np.stack([lo - centres, np.zeros_like(centres), centres - hi]), axis=0)
        if np.min(np.linalg.norm(gap, axis=1)) > 1.0:
            prims.append(_prim(PRIM_BOX, lo, hi))
            n += 1
    scene = _scene(prims, n_octaves=4, base_freq=2.0, tex_seed=int(rng.integers(1 << 62)),
                   sky=0.55)
    poses = [camera_pose(c, y, rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05))
             for c, y in zip(centres, yaws)]
    return scene, poses, 3, [0, 1, 2, 4, 5, 6], [1, 2, 4, 5]


_BUILDERS = {"box_room": (_box_room, 256, "f32"),
             "hall": (_hall, 1920, "f32"),
             "hall7": (_hall7, 1920, "f32"),
             "courtyard": (_courtyard, 3840, "u8")}

WORKLOADS = {"box_room_256": ("box_room", 256),
             "hall_1920": ("hall", 1920),
             "courtyard_3840": ("courtyard", 3840)}


def scene_and_poses(family: str, seed: int):
    builder, W0, dtype = _BUILDERS[family]
    rng = np.random.Generator(np.random.PCG64(seed))
    return builder(rng, W0, 2)


def scaled(family_or_name: str, W: int, seed: int = 0, ss: int | None = None,
           dtype: str | None = None, **param_over) -> Workload:
    """The workload family's scene and parameters rendered at width W."""
    family = family_or_name.split("_")[0] if family_or_name not in _BUILDERS else family_or_name
    if family_or_name in WORKLOADS:
        family = WORKLOADS[family_or_name][0]
    builder, _, fam_dtype = _BUILDERS[family]
    dtype = dtype or fam_dtype
    if W % 2:
        raise ValueError("W must be even")
    H = W // 2
    scene, poses, ref, nbrs, maps = scene_and_poses(family, seed)
    if ss is None:
        ss = 4 if W <= 1920 else 2
        if W >= 1920:
            ss = 2
    imgs, deps, nrms = [], [], []
    for pose in poses:
        img, dep, nrm = render(scene, pose, W, H, ss=ss)
        if dtype == "u8":
            img = np.clip(np.rint(img * 255.0), 0, 255).astype(np.uint8)
        imgs.append(img)
        deps.append(dep)
        nrms.append(nrm)
    return Workload(name=f"{family}_{W}", W=W, H=H, dtype=dtype, images=imgs, gt_depth=deps,
                    gt_normal=nrms, poses=poses, ref=ref, nbrs=list(nbrs), maps=list(maps),
                    params=params_for(family, **param_over))


def workload(name: str, seed: int = 0, **param_over) -> Workload:
    family, W = WORKLOADS[name]
    return scaled(family, W, seed=seed, **param_over)


# ----------------------------------------------------------------------------
# mixed batches and request streams (uneven keyframe jobs)
# ----------------------------------------------------------------------------

MIXED_WIDTHS = (960, 1920, 2880)


def mixed_pool(seed: int = 0, widths=MIXED_WIDTHS, dtype: str = "f16") -> dict:
    """One seven-keyframe hall window per image width, rendered with the
    hall generator and parameters; `dtype` "f16" stores the intensities in
    float16, "f32" in float32."""
    pool = {}
    for k, W in enumerate(widths):
        w = scaled("hall7", W, seed=seed + 101 * k)
        if dtype == "f16":
            w.images = [a.astype(np.float16) for a in w.images]
            w.dtype = "f16"
        pool[W] = w
    return pool


@dataclasses.dataclass
class MixedJob:
    W: int            # image width of the job's window
    ref: int          # reference keyframe index in the window
    nbrs: list        # neighbour keyframe indices (nearest along the path)
    seed: int         # PatchMatch seed of the job


def _mixed_job(rng, W, n_range, n_kf):
    N = int(rng.integers(n_range[0], n_range[1] + 1))
    ref = int(rng.integers(0, n_kf))
    others = sorted((k for k in range(n_kf) if k != ref), key=lambda k: (abs(k - ref), k))[:N]
    return MixedJob(W, ref, sorted(others), int(rng.integers(1 << 31)))


def mixed_jobs(n_by_width: dict, seed: int = 0, n_range=(3, 6), n_kf: int = 7) -> list:
    """`n_by_width[W]` jobs of width W, each with N ~ U{n_range} neighbours
    around a random reference of the window, in a seeded shuffled order."""
    rng = np.random.default_rng(seed)
    jobs = [_mixed_job(rng, W, n_range, n_kf) for W, n in n_by_width.items() for _ in range(n)]
    return [jobs[i] for i in rng.permutation(len(jobs))]


def poisson_requests(n_streams: int, rate_hz: float, horizon_s: float, seed: int = 0,
                     widths=MIXED_WIDTHS, n_range=(3, 6), n_kf: int = 7) -> list:
    """Arrivals of n_streams independent Poisson processes of rate rate_hz
    over [0, horizon_s); each request draws its width uniformly from
    `widths` and N ~ U{n_range}. Returns sorted (time, stream, MixedJob)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_streams):
        t = rng.exponential(1.0 / rate_hz)
        while t < horizon_s:
            W = int(widths[int(rng.integers(0, len(widths)))])
            out.append((float(t), s, _mixed_job(rng, W, n_range, n_kf)))
            t += rng.exponential(1.0 / rate_hz)
    return sorted(out, key=lambda r: r[0])


def stream_requests(n_streams: int, rate_hz: float, horizon_s: float, seed: int = 0,
                    widths=MIXED_WIDTHS, n_range=(3, 6), n_kf: int = 7) -> list:
    """Keyframe streams for a serving loop: each stream has one width (drawn
    uniformly from `widths`) and walks the keyframes of its window back and
    forth (0, 1, ..., n_kf-1, n_kf-2, ..., 0, 1, ...), so consecutive
    keyframes of a stream are neighbours along the trajectory; arrivals are
    Poisson with rate_hz; each keyframe takes N ~ U{n_range} neighbours
    nearest to it. Returns sorted (time, stream, k, MixedJob), k = the
    keyframe's position in its stream."""
    rng = np.random.default_rng(seed)
    out = []
    period = 2 * (n_kf - 1)
    for s in range(n_streams):
        W = int(widths[int(rng.integers(0, len(widths)))])
        t = rng.exponential(1.0 / rate_hz)
        k = 0
        while t < horizon_s:
            ph = k % period
            ref = ph if ph < n_kf else period - ph
            N = int(rng.integers(n_range[0], n_range[1] + 1))
            others = sorted((j for j in range(n_kf) if j != ref), key=lambda j: (abs(j - ref), j))[:N]
            out.append((float(t), s, k, MixedJob(W, ref, sorted(others), int(rng.integers(1 << 31)))))
            t += rng.exponential(1.0 / rate_hz)
            k += 1
    return sorted(out, key=lambda r: r[0])
