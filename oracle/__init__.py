"""ctypes view of the FP64 CPU oracle ``libpmsref.so``.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` import this package. The GPU library never
imports, links or calls it, and shares no code with it.

Every array is float64 and C-contiguous; images are (H, W) with W == 2H.
Normals are planar (3, H, W). Poses are world->camera (R 3x3, t 3).
What each call computes, and what pins it, is stated in ``pmsref.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PMSREF_LIB names another build of pmsref.c (the mutation test loads
# deliberately broken copies through it); by default the in-tree library
LIB_PATH = os.environ.get("PMSREF_LIB") or os.path.join(_HERE, "libpmsref.so")

MAX_VIEWS = 16
MAX_OFFSETS = 16


def build(force: bool = True) -> str:
    """Compile ``libpmsref.so`` with gcc (plain C11, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
               "-fPIC", "-shared", "-pthread", os.path.join(_HERE, "pmsref.c"),
               "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [
        ("patch_size", C.c_int32),
        ("patch_stride", C.c_int32),
        ("iterations", C.c_int32),
        ("refine_trials", C.c_int32),
        ("depth_min", C.c_double),
        ("depth_max", C.c_double),
        ("top_k", C.c_int32),
        ("ncc_var_floor", C.c_double),
        ("refine_sigma_logdepth0", C.c_double),
        ("refine_depth_shrink", C.c_double),
        ("refine_sigma_normal0", C.c_double),
        ("refine_normal_shrink", C.c_double),
        ("n_offsets", C.c_int32),
        ("offsets", (C.c_int32 * 2) * MAX_OFFSETS),
        ("geo_px", C.c_double),
        ("geo_rel_depth", C.c_double),
        ("geo_min_views", C.c_int32),
        ("seed", C.c_uint64),
        ("median_radius", C.c_int32),
        ("median_rel", C.c_double),
    ]


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        L.pmsref_default_params.argtypes = [C.POINTER(Params)]
        L.pmsref_check_params.argtypes = [C.POINTER(Params), C.c_int, C.c_int, C.c_int]
        L.pmsref_unproject.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _D]
        L.pmsref_project.argtypes = [C.c_int, C.c_int, _D, _D, _D]
        L.pmsref_sample.argtypes = [_D, C.c_int, C.c_int, C.c_double, C.c_double]
        L.pmsref_sample.restype = C.c_double
        L.pmsref_relative_pose.argtypes = [C.POINTER(Pose), C.POINTER(Pose), _D, _D]
        L.pmsref_philox4x64_10.argtypes = [C.c_uint64, C.c_uint64,
                                           C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.pmsref_philox4x64_10_stream.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_long,
                                                  C.POINTER(C.c_uint64)]
        L.pmsref_uniforms.argtypes = [C.c_uint64] * 4 + [_D]
        L.pmsref_patch_offsets.argtypes = [C.POINTER(Params), _I32, _I32]
        L.pmsref_view_cost.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D, C.POINTER(Params),
                                       C.c_int, C.c_int, C.c_double, _D, _D, _D, _D, _D]
        L.pmsref_view_cost.restype = C.c_double
        L.pmsref_aggregate.argtypes = [_D, C.c_int, C.c_int]
        L.pmsref_aggregate.restype = C.c_double
        L.pmsref_eval_cost.argtypes = [C.c_int, C.c_int, _D, C.c_int, C.POINTER(_D),
                                       C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Params),
                                       _D, _D, _D, _D, C.c_int]
        L.pmsref_update_pixel.argtypes = [C.c_int, C.c_int, _D, C.c_int, C.POINTER(_D),
                                          C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Params),
                                          _D, _D, _D, C.c_int, C.c_int, C.c_int, _D, _D, _D]
        L.pmsref_consistency.argtypes = [C.c_int, C.c_int, _D, _D, _D, C.POINTER(Pose), C.c_int,
                                         C.POINTER(_D), C.POINTER(Pose), C.POINTER(Params),
                                         _D, _D, _I32, C.c_int]
        L.pmsref_densify.argtypes = [C.c_int, C.c_int, _D, C.c_int, C.POINTER(_D),
                                     C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Params),
                                     _D, _D, C.c_int, C.POINTER(_D), C.POINTER(Pose),
                                     _D, _D, _D, C.c_int, C.c_uint64]
        L.pmsref_halfsweep_rows.argtypes = [C.c_int, C.c_int, _D, C.c_int, C.POINTER(_D),
                                            C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Params),
                                            _D, _D, _D, C.c_int, C.c_int, C.c_int, C.c_int,
                                            _D, _D, _D, C.c_int]
        L.pmsref_set_decision_noise.argtypes = [C.c_double]
        L.pmsref_set_decision_noise.restype = None
        L.pmsref_pixel_valid.argtypes = [C.c_int, C.c_int, C.POINTER(Params), C.c_int, C.c_int]
        _U8 = C.POINTER(C.c_uint8)
        L.pmsref_fuse.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(_D), C.POINTER(Pose), C.c_double,
                                  _U8, C.POINTER(C.c_long)]
        L.pmsref_coverage.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(_D), C.POINTER(Pose), _U8,
                                      C.POINTER(Pose), C.c_int, C.c_int, _U8]
        L.pmsref_coverage.restype = C.c_long
        L.pmsref_view_filter.argtypes = [_D, _D, _D, C.c_long, C.c_double, C.c_double, C.c_double,
                                         C.POINTER(C.c_long), C.POINTER(C.c_long)]
        L.pmsref_median_filter.argtypes = [C.c_int, C.c_int, _D, _D, _D, C.POINTER(Params)]
        L.pmsref_warp_planes.argtypes = [C.c_int, C.c_int, _D, _D, C.POINTER(Pose), C.POINTER(Pose),
                                         C.POINTER(Params), _D, _D]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------

def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_pose(R, t) -> Pose:
    p = Pose()
    R = np.asarray(R, dtype=np.float64).reshape(9)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    for i in range(9):
        p.R[i] = float(R[i])
    for i in range(3):
        p.t[i] = float(t[i])
    return p


def _poses(poses) -> "C.Array":
    arr = (Pose * max(1, len(poses)))()
    for i, (R, t) in enumerate(poses):
        arr[i] = make_pose(R, t)
    return arr


def default_params() -> dict:
    p = Params()
    lib().pmsref_default_params(C.byref(p))
    return params_to_dict(p)


def params_to_dict(p: Params) -> dict:
    d = {}
    for name, _ in Params._fields_:
        v = getattr(p, name)
        if name == "offsets":
            v = [(int(v[k][0]), int(v[k][1])) for k in range(p.n_offsets)]
        d[name] = v
    return d


def make_params(overrides: dict | None = None) -> Params:
    p = Params()
    lib().pmsref_default_params(C.byref(p))
    for k, v in (overrides or {}).items():
        if k == "offsets":
            p.n_offsets = len(v)
            for i, (ox, oy) in enumerate(v):
                p.offsets[i][0] = int(ox)
                p.offsets[i][1] = int(oy)
        elif k == "n_offsets":
            continue
        else:
            setattr(p, k, v)
    return p


class _Views:
    """Keeps float64 copies of the neighbour images alive with a pointer array."""

    def __init__(self, images):
        self.arrs = [_f64(a) for a in images]
        self.ptrs = (_D * max(1, len(self.arrs)))(*[_dptr(a) for a in self.arrs])


# ----------------------------------------------------------------------------
# public calls
# ----------------------------------------------------------------------------

def check_params(params: dict, W: int, H: int, n_views: int) -> int:
    return lib().pmsref_check_params(C.byref(make_params(params)), W, H, n_views)


def unproject(W: int, H: int, x: float, y: float) -> np.ndarray:
    b = np.zeros(3)
    lib().pmsref_unproject(W, H, float(x), float(y), _dptr(b))
    return b


def project(W: int, H: int, Y) -> tuple[float, float]:
    Y = _f64(Y)
    x = C.c_double()
    y = C.c_double()
    lib().pmsref_project(W, H, _dptr(Y), C.byref(x), C.byref(y))
    return x.value, y.value


def sample(img, x: float, y: float) -> float:
    img = _f64(img)
    H, W = img.shape
    return lib().pmsref_sample(_dptr(img), W, H, float(x), float(y))


def relative_pose(ref_pose, nbr_pose):
    R = np.zeros(9)
    t = np.zeros(3)
    a = make_pose(*ref_pose)
    b = make_pose(*nbr_pose)
    lib().pmsref_relative_pose(C.byref(a), C.byref(b), _dptr(R), _dptr(t))
    return R.reshape(3, 3), t


def philox4x64_10(key0: int, key1: int, ctr) -> list[int]:
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    out = (C.c_uint64 * 4)()
    lib().pmsref_philox4x64_10(int(key0), int(key1), c, out)
    return [int(v) for v in out]


def philox4x64_10_stream(key0: int, key1: int, ctr0: int, n: int) -> np.ndarray:
    """Blocks for counters (ctr0 + i, 0, 0, 0), i < n, as an (n, 4) uint64 array."""
    out = np.zeros((n, 4), dtype=np.uint64)
    lib().pmsref_philox4x64_10_stream(int(key0), int(key1), int(ctr0), int(n),
                                      out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return out


def uniforms(seed: int, pixel: int, iteration: int, stage: int) -> np.ndarray:
    u = np.zeros(4)
    lib().pmsref_uniforms(int(seed), int(pixel), int(iteration), int(stage), _dptr(u))
    return u


def patch_offsets(params: dict | None = None):
    p = make_params(params)
    n = lib().pmsref_patch_offsets(C.byref(p), None, None)
    dx = np.zeros(n, dtype=np.int32)
    dy = np.zeros(n, dtype=np.int32)
    lib().pmsref_patch_offsets(C.byref(p), dx.ctypes.data_as(_I32), dy.ctypes.data_as(_I32))
    return dx, dy


def view_cost(ref, nbr, R, t, params: dict, x: int, y: int, d: float, n):
    """Returns (cost, r_samples, s_samples, var_r, var_s)."""
    ref = _f64(ref)
    nbr = _f64(nbr)
    H, W = ref.shape
    p = make_params(params)
    P = lib().pmsref_patch_offsets(C.byref(p), None, None)
    r = np.full(P, np.nan)
    s = np.full(P, np.nan)
    vr = C.c_double(np.nan)
    vs = C.c_double(np.nan)
    Rf = _f64(R).reshape(9)
    tf = _f64(t).reshape(3)
    nf = _f64(n).reshape(3)
    c = lib().pmsref_view_cost(W, H, _dptr(ref), _dptr(nbr), _dptr(Rf), _dptr(tf), C.byref(p),
                               int(x), int(y), float(d), _dptr(nf), _dptr(r), _dptr(s),
                               C.byref(vr), C.byref(vs))
    return c, r, s, vr.value, vs.value


def aggregate(view_costs, top_k: int = 0) -> float:
    v = _f64(view_costs)
    return lib().pmsref_aggregate(_dptr(v), len(v), int(top_k))


def eval_cost(ref, nbrs, ref_pose, nbr_poses, params: dict, depth, normal, n_threads: int = 0):
    """Aggregated and per-view cost of given hypotheses. Returns (cost, per_view)."""
    ref = _f64(ref)
    H, W = ref.shape
    V = _Views(nbrs)
    N = len(V.arrs)
    depth = _f64(depth)
    normal = _f64(normal)
    cost = np.zeros((H, W))
    pv = np.zeros((N, H, W))
    rp = _poses([ref_pose])
    npz = _poses(nbr_poses)
    rc = lib().pmsref_eval_cost(W, H, _dptr(ref), N, V.ptrs, rp, npz,
                                C.byref(make_params(params)), _dptr(depth), _dptr(normal),
                                _dptr(cost), _dptr(pv), int(n_threads))
    if rc:
        raise ValueError(f"pmsref_eval_cost failed: {rc}")
    return cost, pv


def update_pixel(ref, nbrs, ref_pose, nbr_poses, params: dict, depth, normal, cost,
                 iteration: int, x: int, y: int):
    ref = _f64(ref)
    H, W = ref.shape
    V = _Views(nbrs)
    depth = _f64(depth)
    normal = _f64(normal)
    cost = _f64(cost)
    d = C.c_double()
    n = np.zeros(3)
    c = C.c_double()
    rc = lib().pmsref_update_pixel(W, H, _dptr(ref), len(V.arrs), V.ptrs, _poses([ref_pose]),
                                   _poses(nbr_poses), C.byref(make_params(params)),
                                   _dptr(depth), _dptr(normal), _dptr(cost), int(iteration),
                                   int(x), int(y), C.byref(d), _dptr(n), C.byref(c))
    if rc:
        raise ValueError(f"pmsref_update_pixel failed: {rc}")
    return d.value, n, c.value


def halfsweep_rows(ref, nbrs, ref_pose, nbr_poses, params: dict, depth, normal, cost,
                   iteration: int, colour: int, y0: int, y1: int, n_threads: int = 0):
    """One half-sweep over rows [y0, y1); returns the new (depth, normal, cost)."""
    ref = _f64(ref)
    H, W = ref.shape
    V = _Views(nbrs)
    depth = _f64(depth)
    normal = _f64(normal)
    cost = _f64(cost)
    d1 = np.empty_like(depth)
    n1 = np.empty_like(normal)
    c1 = np.empty_like(cost)
    rc = lib().pmsref_halfsweep_rows(W, H, _dptr(ref), len(V.arrs), V.ptrs, _poses([ref_pose]),
                                     _poses(nbr_poses), C.byref(make_params(params)),
                                     _dptr(depth), _dptr(normal), _dptr(cost), int(iteration),
                                     int(colour), int(y0), int(y1), _dptr(d1), _dptr(n1),
                                     _dptr(c1), int(n_threads))
    if rc:
        raise ValueError(f"pmsref_halfsweep_rows failed: {rc}")
    return d1, n1, c1


def consistency(depth, normal, cost, ref_pose, maps, map_poses, params: dict,
                n_threads: int = 0, diagnostics: bool = False):
    """Filters copies of (depth, normal, cost). Returns them, plus (err_px,
    err_depth, agree) per map when ``diagnostics``."""
    depth = _f64(depth).copy()
    normal = _f64(normal).copy()
    cost = _f64(cost).copy()
    H, W = depth.shape
    M = _Views(maps)
    nm = len(M.arrs)
    epx = np.zeros((nm, H, W)) if diagnostics else None
    ed = np.zeros((nm, H, W)) if diagnostics else None
    ag = np.zeros((nm, H, W), dtype=np.int32) if diagnostics else None
    rc = lib().pmsref_consistency(W, H, _dptr(depth), _dptr(normal), _dptr(cost),
                                  _poses([ref_pose]), nm, M.ptrs, _poses(map_poses),
                                  C.byref(make_params(params)),
                                  _dptr(epx) if diagnostics else None,
                                  _dptr(ed) if diagnostics else None,
                                  ag.ctypes.data_as(_I32) if diagnostics else None,
                                  int(n_threads))
    if rc:
        raise ValueError(f"pmsref_consistency failed: {rc}")
    if diagnostics:
        return depth, normal, cost, epx, ed, ag
    return depth, normal, cost


def densify(ref, nbrs, ref_pose, nbr_poses, params: dict, init_depth=None, init_normal=None,
            maps=None, map_poses=None, n_threads: int = 0, order_seed: int = 0):
    """Full densification. Returns (depth (H,W), normal (3,H,W), cost (H,W))."""
    ref = _f64(ref)
    H, W = ref.shape
    V = _Views(nbrs)
    depth = np.zeros((H, W))
    normal = np.zeros((3, H, W))
    cost = np.zeros((H, W))
    idp = _f64(init_depth) if init_depth is not None else None
    inn = _f64(init_normal) if init_normal is not None else None
    M = _Views(maps or [])
    nm = len(M.arrs)
    rc = lib().pmsref_densify(W, H, _dptr(ref), len(V.arrs), V.ptrs, _poses([ref_pose]),
                              _poses(nbr_poses), C.byref(make_params(params)),
                              _dptr(idp) if idp is not None else None,
                              _dptr(inn) if inn is not None else None,
                              nm, M.ptrs if nm else None,
                              _poses(map_poses) if nm else None,
                              _dptr(depth), _dptr(normal), _dptr(cost), int(n_threads),
                              int(order_seed))
    if rc:
        raise ValueError(f"pmsref_densify failed: {rc}")
    return depth, normal, cost


def set_decision_noise(amplitude: float) -> None:
    """Study hook, off (0) by default: adds a deterministic offset uniform in
    [-amplitude, amplitude] to every cost that enters an accept decision
    (initial costs, propagation and refinement candidates). Used only to
    measure how far the oracle moves under independent per-evaluation
    errors; see ``pmsref.h``."""
    lib().pmsref_set_decision_noise(float(amplitude))


def warp_planes(src_depth, src_normal, src_pose, dst_pose, params: dict):
    """Plane map of the keyframe at src_pose carried into the keyframe at
    dst_pose (Sec. III-B). Returns (depth (H,W), normal (3,H,W)); depth 0
    where no plane arrives."""
    sd = _f64(src_depth)
    sn = _f64(src_normal)
    H, W = sd.shape
    dd = np.zeros((H, W))
    dn = np.zeros((3, H, W))
    rc = lib().pmsref_warp_planes(W, H, _dptr(sd), _dptr(sn), _poses([src_pose]), _poses([dst_pose]),
                                  C.byref(make_params(params)), _dptr(dd), _dptr(dn))
    if rc:
        raise ValueError(f"pmsref_warp_planes failed: {rc}")
    return dd, dn


def median_filter(depth, normal, cost, params: dict):
    """Median post-filter (Sec. III-C item 2) of copies of the maps."""
    depth = _f64(depth).copy()
    normal = _f64(normal).copy()
    cost = _f64(cost).copy()
    H, W = depth.shape
    rc = lib().pmsref_median_filter(W, H, _dptr(depth), _dptr(normal), _dptr(cost),
                                    C.byref(make_params(params)))
    if rc:
        raise ValueError(f"pmsref_median_filter failed: {rc}")
    return depth, normal, cost


def view_filter(centre_a, centre_b, points, min_deg=6.0, max_deg=60.0, min_frac=0.2):
    """Eq. (1): (accepted, points in the angle range, points counted)."""
    ca, cb = _f64(centre_a).reshape(3), _f64(centre_b).reshape(3)
    pts = _f64(points).reshape(-1, 3)
    k, c = C.c_long(), C.c_long()
    rc = lib().pmsref_view_filter(_dptr(ca), _dptr(cb), _dptr(pts) if len(pts) else None, len(pts),
                                  float(min_deg), float(max_deg), float(min_frac), C.byref(k), C.byref(c))
    if rc < 0:
        raise ValueError(f"pmsref_view_filter failed: {rc}")
    return bool(rc), k.value, c.value


def fuse(depths, poses, voxel: float):
    """Keep masks (n_maps, H, W) uint8 of the de-duplicated points and their count."""
    M = _Views(depths)
    H, W = M.arrs[0].shape
    keep = np.zeros((len(M.arrs), H, W), dtype=np.uint8)
    n = C.c_long()
    rc = lib().pmsref_fuse(W, H, len(M.arrs), M.ptrs, _poses(poses), float(voxel),
                           keep.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(n))
    if rc:
        raise ValueError(f"pmsref_fuse failed: {rc}")
    return keep, n.value


def coverage(depths, poses, keep, view_pose, Wc: int = 720, Hc: int = 360):
    """(number of covered pixels, cover mask (Hc, Wc))."""
    M = _Views(depths)
    H, W = M.arrs[0].shape
    cover = np.zeros((Hc, Wc), dtype=np.uint8)
    kp = None
    if keep is not None:
        keep = np.ascontiguousarray(keep, dtype=np.uint8)
        kp = keep.ctypes.data_as(C.POINTER(C.c_uint8))
    c = lib().pmsref_coverage(W, H, len(M.arrs), M.ptrs, _poses(poses), kp, _poses([view_pose]),
                              Wc, Hc, cover.ctypes.data_as(C.POINTER(C.c_uint8)))
    if c < 0:
        raise ValueError(f"pmsref_coverage failed: {c}")
    return c, cover
