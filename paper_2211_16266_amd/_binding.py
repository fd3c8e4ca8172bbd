"""Thin ctypes binding of libpms (include/pms.h) over PyTorch device tensors.

Argument marshalling only: every step of the densifier runs in the HIP
kernels of libpms. Tensors supply device memory, torch's current stream
supplies the hipStream_t. There is no CPU fallback: without the built
library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
# PMS_LIB names another build of the same sources (the host-sanitizer
# test loads one); by default the in-tree library
LIB_PATH = os.environ.get("PMS_LIB") or os.path.join(PKG, "libpms.so")

NOALLOC_SCRATCH_BYTES = 128 << 20  # PMS_NOALLOC_SCRATCH_BYTES of pms.h
MAX_VIEWS = 8
MAX_MAPS = 8
MAX_OFFSETS = 16

PMS_F32, PMS_F16, PMS_U8 = 0, 1, 2
_DTYPES = {torch.float32: (PMS_F32, 4), torch.float16: (PMS_F16, 2), torch.uint8: (PMS_U8, 1)}

STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "device error",
          4: "unsupported", 5: "scratch budget exceeded"}


class PmsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_bytes", C.c_int64), ("dtype", C.c_int32)]


class Plane(C.Structure):
    _fields_ = [("data", C.c_void_p), ("pitch_elems", C.c_int64)]


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


MAX_BATCH = 256


class Params(C.Structure):
    _fields_ = [
        ("patch_size", C.c_int32), ("patch_stride", C.c_int32), ("iterations", C.c_int32),
        ("refine_trials", C.c_int32), ("depth_min", C.c_double), ("depth_max", C.c_double),
        ("top_k", C.c_int32), ("ncc_var_floor", C.c_double),
        ("refine_sigma_logdepth0", C.c_double), ("refine_depth_shrink", C.c_double),
        ("refine_sigma_normal0", C.c_double), ("refine_normal_shrink", C.c_double),
        ("n_offsets", C.c_int32), ("offsets", (C.c_int32 * 2) * MAX_OFFSETS),
        ("geo_px", C.c_double), ("geo_rel_depth", C.c_double), ("geo_min_views", C.c_int32),
        ("seed", C.c_uint64), ("median_radius", C.c_int32), ("median_rel", C.c_double),
    ]


class Job(C.Structure):
    _fields_ = [("ref", Image), ("ref_pose", Pose), ("nbrs", C.POINTER(Image)),
                ("nbr_poses", C.POINTER(Pose)), ("n_nbrs", C.c_int32),
                ("maps", C.POINTER(Plane)), ("map_poses", C.POINTER(Pose)), ("n_maps", C.c_int32),
                ("params", C.POINTER(Params)), ("depth_out", Plane), ("normal_out", Plane * 3),
                ("cost_out", Plane), ("init_depth", Plane), ("init_normal", Plane * 3)]


WORK_FIELDS = ("pixels", "prop_candidates", "refine_trials", "skipped_geometry", "skipped_repeat",
               "scored", "facing_rejects", "view_evals", "views_pruned")


class WorkCounts(C.Structure):
    _fields_ = [(n, C.c_int64) for n in WORK_FIELDS]


class Schedule(C.Structure):
    _fields_ = [("wave_rows", C.c_int32), ("waves_x", C.c_int32), ("lanes_per_pixel", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """The loaded libpms; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(the densifier has no CPU path)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.pms_default_params.argtypes = [P(Params)]
        L.pms_context_create.argtypes = [C.c_int32, C.c_size_t, P(C.c_void_p)]
        L.pms_context_destroy.argtypes = [C.c_void_p]
        L.pms_densify.argtypes = [C.c_void_p, P(Image), P(Pose), P(Image), P(Pose), C.c_int32,
                                  P(Plane), P(Pose), C.c_int32, P(Params), Plane, P(Plane), Plane,
                                  C.c_void_p]
        L.pms_densify_noalloc.argtypes = L.pms_densify.argtypes
        L.pms_eval_cost.argtypes = [C.c_void_p, P(Image), P(Pose), P(Image), P(Pose), C.c_int32,
                                    P(Params), Plane, P(Plane), Plane, P(Plane), C.c_void_p]
        L.pms_halfsweep.argtypes = [C.c_void_p, P(Image), P(Pose), P(Image), P(Pose), C.c_int32,
                                    P(Params), C.c_int32, C.c_int32, Plane, P(Plane), Plane,
                                    C.c_void_p]
        L.pms_consistency.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(Pose), P(Plane), P(Pose),
                                      C.c_int32, P(Params), Plane, P(Plane), Plane, C.c_void_p]
        L.pms_warp_planes.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(Pose), Plane, P(Plane),
                                      P(Pose), P(Params), Plane, P(Plane), C.c_void_p]
        L.pms_fuse.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, P(Plane), P(Pose), C.c_double,
                               C.c_void_p, C.c_void_p, C.c_void_p]
        L.pms_coverage.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, P(Plane), P(Pose),
                                   C.c_void_p, P(Pose), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
        L.pms_view_filter.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), C.c_void_p, C.c_int64,
                                      C.c_double, C.c_double, C.c_void_p, C.c_void_p]
        L.pms_philox_stream.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int64,
                                        C.c_void_p, C.c_void_p]
        L.pms_profile_enable.argtypes = [C.c_void_p, C.c_int32]
        L.pms_work_count_enable.argtypes = [C.c_void_p, C.c_int32]
        L.pms_work_count_read.argtypes = [C.c_void_p, P(WorkCounts), C.c_int32]
        L.pms_profile_read.argtypes = [C.c_void_p, C.c_char_p, P(C.c_int64), P(C.c_double)]
        L.pms_densify_batch.argtypes = [C.c_void_p, P(Job), C.c_int32, C.c_void_p]
        L.pms_batch_create.argtypes = [C.c_void_p, P(Job), C.c_int32, P(C.c_void_p)]
        L.pms_batch_run.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
        L.pms_batch_bytes.argtypes = [C.c_void_p, P(C.c_size_t)]
        L.pms_batch_destroy.argtypes = [C.c_void_p]
        L.pms_get_schedule.argtypes = [C.c_void_p, P(Schedule)]
        L.pms_set_schedule.argtypes = [C.c_void_p, P(Schedule)]
        L.pms_autotune.argtypes = [C.c_void_p, P(Job), C.c_int32, C.c_int32, C.c_int32,
                                   P(Schedule), P(C.c_double), C.c_void_p]
        L.pms_server_create.argtypes = [C.c_void_p, C.c_size_t, C.c_int32, P(C.c_void_p)]
        L.pms_server_submit.argtypes = [C.c_void_p, P(Job), P(C.c_int64)]
        L.pms_server_step.argtypes = [C.c_void_p, C.c_void_p, P(C.c_int32), P(C.c_int32)]
        L.pms_server_poll.argtypes = [C.c_void_p, C.c_int64, P(C.c_int32)]
        L.pms_server_stats.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int64), P(C.c_size_t),
                                       P(C.c_size_t)]
        L.pms_server_destroy.argtypes = [C.c_void_p]
        L.pms_status_string.argtypes = [C.c_int]
        L.pms_status_string.restype = C.c_char_p
        L.pms_last_error.argtypes = [C.c_void_p]
        L.pms_last_error.restype = C.c_char_p
        for name in ("pms_default_params", "pms_context_create", "pms_context_destroy",
                     "pms_densify", "pms_densify_noalloc", "pms_eval_cost", "pms_halfsweep", "pms_consistency",
                     "pms_philox_stream", "pms_profile_enable", "pms_profile_read",
                     "pms_work_count_enable", "pms_work_count_read",
                     "pms_densify_batch", "pms_batch_create", "pms_batch_run", "pms_batch_bytes",
                     "pms_batch_destroy", "pms_get_schedule", "pms_set_schedule", "pms_autotune",
                     "pms_server_create", "pms_server_submit", "pms_server_step",
                     "pms_server_poll", "pms_server_stats", "pms_server_destroy",
                     "pms_warp_planes", "pms_view_filter", "pms_fuse", "pms_coverage"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# marshalling
# ----------------------------------------------------------------------------

def default_params() -> dict:
    p = Params()
    lib().pms_default_params(C.byref(p))
    d = {}
    for name, _ in Params._fields_:
        v = getattr(p, name)
        if name == "offsets":
            v = [(int(v[k][0]), int(v[k][1])) for k in range(p.n_offsets)]
        d[name] = v
    return d


def make_params(overrides: dict | None = None) -> Params:
    p = Params()
    lib().pms_default_params(C.byref(p))
    for k, v in (overrides or {}).items():
        if k == "offsets":
            if len(v) > MAX_OFFSETS:
                raise ValueError("too many propagation offsets")
            p.n_offsets = len(v)
            for i, (ox, oy) in enumerate(v):
                p.offsets[i][0] = int(ox)
                p.offsets[i][1] = int(oy)
        elif k != "n_offsets":
            setattr(p, k, v)
    return p


def make_pose(pose) -> Pose:
    R, t = pose
    R = torch.as_tensor(R, dtype=torch.float64).reshape(9).tolist()
    t = torch.as_tensor(t, dtype=torch.float64).reshape(3).tolist()
    p = Pose()
    for i in range(9):
        p.R[i] = R[i]
    for i in range(3):
        p.t[i] = t[i]
    return p


def _poses(poses):
    arr = (Pose * max(1, len(poses)))()
    for i, pz in enumerate(poses):
        arr[i] = make_pose(pz)
    return arr


def _device_2d(t: torch.Tensor, what: str) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{what} must be 2-D with unit column stride")


def make_image(t: torch.Tensor, what: str = "image") -> Image:
    _device_2d(t, what)
    if t.dtype not in _DTYPES:
        raise ValueError(f"{what}: dtype must be float32, float16 or uint8")
    code, size = _DTYPES[t.dtype]
    H, W = t.shape
    return Image(t.data_ptr(), W, H, t.stride(0) * size, code)


def make_plane(t: torch.Tensor, what: str = "plane") -> Plane:
    _device_2d(t, what)
    if t.dtype != torch.float32:
        raise ValueError(f"{what} must be float32")
    return Plane(t.data_ptr(), t.stride(0))


def _planes3(normal: torch.Tensor, what: str):
    if normal.dim() != 3 or normal.shape[0] != 3:
        raise ValueError(f"{what} must be (3, H, W)")
    return (Plane * 3)(*[make_plane(normal[i], what) for i in range(3)])


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Context:
    """A libpms context: the scratch memory of one stream's work."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.device = device
        h = C.c_void_p()
        st = lib().pms_context_create(int(device), int(budget_bytes), C.byref(h))
        if st:
            raise PmsError(st, "pms_context_create")
        self.handle = h

    def check(self, st: int, what: str) -> None:
        if st:
            msg = lib().pms_last_error(self.handle).decode() if self.handle else ""
            raise PmsError(st, f"{what}: {msg}")

    def close(self) -> None:
        if self.handle:
            lib().pms_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, on: bool = True) -> None:
        self.check(lib().pms_profile_enable(self.handle, int(bool(on))), "pms_profile_enable")

    def work_count_enable(self, on: bool = True) -> None:
        """Half-sweeps of this context count their executed work while on."""
        self.check(lib().pms_work_count_enable(self.handle, int(on)), "pms_work_count_enable")

    def work_count_read(self, reset: bool = True) -> dict:
        """Totals of the half-sweep work counters (synchronises the device)."""
        w = WorkCounts()
        self.check(lib().pms_work_count_read(self.handle, C.byref(w), int(reset)), "pms_work_count_read")
        return {n: int(getattr(w, n)) for n in WORK_FIELDS}

    def get_schedule(self) -> dict:
        sc = Schedule()
        self.check(lib().pms_get_schedule(self.handle, C.byref(sc)), "pms_get_schedule")
        return {"wave_rows": sc.wave_rows, "waves_x": sc.waves_x,
                "lanes_per_pixel": sc.lanes_per_pixel}

    def set_schedule(self, wave_rows: int = 4, waves_x: int = 2, lanes_per_pixel: int = 4) -> None:
        sc = Schedule(int(wave_rows), int(waves_x), int(lanes_per_pixel))
        self.check(lib().pms_set_schedule(self.handle, C.byref(sc)), "pms_set_schedule")

    def autotune(self, jobs, reps: int = 2, try_lanes: bool = False, stream=None) -> tuple[dict, float]:
        """Times every tile shape on ``jobs`` (see ``job``) and keeps the
        fastest; returns (schedule, milliseconds of init + half-sweeps)."""
        arr, keep = _job_array(jobs)
        sc = Schedule()
        ms = C.c_double()
        self.check(lib().pms_autotune(self.handle, arr, len(jobs), int(reps), int(bool(try_lanes)),
                                      C.byref(sc), C.byref(ms), C.c_void_p(_stream_handle(stream))),
                   "pms_autotune")
        del keep
        return ({"wave_rows": sc.wave_rows, "waves_x": sc.waves_x,
                 "lanes_per_pixel": sc.lanes_per_pixel}, ms.value)

    def profile_read(self, name: str) -> tuple[int, float]:
        n = C.c_int64()
        ms = C.c_double()
        self.check(lib().pms_profile_read(self.handle, name.encode(), C.byref(n), C.byref(ms)),
                   "pms_profile_read")
        return n.value, ms.value


_default_ctx: dict = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _views(nbrs):
    if len(nbrs) > MAX_VIEWS:
        raise ValueError("too many neighbours")
    return (Image * max(1, len(nbrs)))(*[make_image(t, "neighbour") for t in nbrs])


def densify(ref: torch.Tensor, nbrs, ref_pose, nbr_poses, params: dict | None = None, maps=None,
            map_poses=None, out=None, ctx: Context | None = None, stream=None):
    """Depth (H, W), normal (3, H, W) and cost (H, W) float32 device tensors
    of the reference keyframe. ``maps``/``map_poses`` enable the consistency
    filter. ``out`` may supply the three output tensors."""
    return _densify_call("pms_densify", ref, nbrs, ref_pose, nbr_poses, params, maps, map_poses,
                         out, ctx, stream)


def densify_noalloc(ref: torch.Tensor, nbrs, ref_pose, nbr_poses, params: dict | None = None,
                    maps=None, map_poses=None, out=None, ctx: Context | None = None, stream=None):
    """``densify`` through ``pms_densify_noalloc``: the library's working
    memory comes from its fixed per-device scratch array. Pass ``out`` to
    make the call itself allocate nothing (otherwise the three output
    tensors are allocated here, by torch, before the call)."""
    return _densify_call("pms_densify_noalloc", ref, nbrs, ref_pose, nbr_poses, params, maps,
                         map_poses, out, ctx, stream)


def _densify_call(fn: str, ref, nbrs, ref_pose, nbr_poses, params, maps, map_poses, out, ctx,
                  stream):
    ctx = ctx or default_context(ref.device.index or 0)
    H, W = ref.shape
    if out is None:
        depth = torch.empty((H, W), dtype=torch.float32, device=ref.device)
        normal = torch.empty((3, H, W), dtype=torch.float32, device=ref.device)
        cost = torch.empty((H, W), dtype=torch.float32, device=ref.device)
    else:
        depth, normal, cost = out
    maps = list(maps or [])
    map_poses = list(map_poses or [])
    if len(maps) != len(map_poses):
        raise ValueError("maps and map_poses differ in length")
    mp = (Plane * max(1, len(maps)))(*[make_plane(m, "map") for m in maps])
    st = getattr(lib(), fn)(ctx.handle, C.byref(make_image(ref, "ref")), C.byref(make_pose(ref_pose)),
                            _views(nbrs), _poses(nbr_poses), len(nbrs),
                            mp if maps else None, _poses(map_poses) if maps else None, len(maps),
                            C.byref(make_params(params)), make_plane(depth, "depth"),
                            _planes3(normal, "normal"), make_plane(cost, "cost"),
                            C.c_void_p(_stream_handle(stream)))
    ctx.check(st, fn)
    return depth, normal, cost


def eval_cost(ref: torch.Tensor, nbrs, ref_pose, nbr_poses, params: dict | None, depth: torch.Tensor,
              normal: torch.Tensor, per_view: bool = False, ctx: Context | None = None, stream=None):
    """Aggregated cost (H, W) of given hypotheses, and the per-view costs
    (N, H, W) when ``per_view``."""
    ctx = ctx or default_context(ref.device.index or 0)
    H, W = ref.shape
    cost = torch.empty((H, W), dtype=torch.float32, device=ref.device)
    pv = torch.empty((len(nbrs), H, W), dtype=torch.float32, device=ref.device) if per_view else None
    pvp = (Plane * len(nbrs))(*[make_plane(pv[j]) for j in range(len(nbrs))]) if per_view else None
    st = lib().pms_eval_cost(ctx.handle, C.byref(make_image(ref, "ref")), C.byref(make_pose(ref_pose)),
                             _views(nbrs), _poses(nbr_poses), len(nbrs),
                             C.byref(make_params(params)), make_plane(depth, "depth"),
                             _planes3(normal, "normal"), make_plane(cost, "cost"), pvp,
                             C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_eval_cost")
    return (cost, pv) if per_view else cost


def halfsweep(ref: torch.Tensor, nbrs, ref_pose, nbr_poses, params: dict | None, iteration: int,
              colour: int, depth: torch.Tensor, normal: torch.Tensor, cost: torch.Tensor,
              ctx: Context | None = None, stream=None) -> None:
    """One red (colour 0) or black (colour 1) half-sweep on the given state,
    in place."""
    ctx = ctx or default_context(ref.device.index or 0)
    st = lib().pms_halfsweep(ctx.handle, C.byref(make_image(ref, "ref")), C.byref(make_pose(ref_pose)),
                             _views(nbrs), _poses(nbr_poses), len(nbrs),
                             C.byref(make_params(params)), int(iteration), int(colour),
                             make_plane(depth, "depth"), _planes3(normal, "normal"),
                             make_plane(cost, "cost"), C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_halfsweep")


def consistency(ref_pose, maps, map_poses, params: dict | None, depth: torch.Tensor,
                normal: torch.Tensor, cost: torch.Tensor, ctx: Context | None = None,
                stream=None) -> None:
    """Geometric-consistency filter of (depth, normal, cost), in place."""
    ctx = ctx or default_context(depth.device.index or 0)
    H, W = depth.shape
    mp = (Plane * max(1, len(maps)))(*[make_plane(m, "map") for m in maps])
    st = lib().pms_consistency(ctx.handle, W, H, C.byref(make_pose(ref_pose)), mp,
                               _poses(map_poses), len(maps), C.byref(make_params(params)),
                               make_plane(depth, "depth"), _planes3(normal, "normal"),
                               make_plane(cost, "cost"), C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_consistency")


def warp_planes(src_depth: torch.Tensor, src_normal: torch.Tensor, src_pose, dst_pose,
                params: dict | None = None, out=None, ctx: Context | None = None, stream=None):
    """The plane map (depth (H, W), normal (3, H, W)) of the keyframe at
    src_pose carried into the keyframe at dst_pose (Sec. III-B)."""
    ctx = ctx or default_context(src_depth.device.index or 0)
    H, W = src_depth.shape
    if out is None:
        out = (torch.empty((H, W), dtype=torch.float32, device=src_depth.device),
               torch.empty((3, H, W), dtype=torch.float32, device=src_depth.device))
    dd, dn = out
    st = lib().pms_warp_planes(ctx.handle, W, H, C.byref(make_pose(src_pose)),
                               make_plane(src_depth, "src depth"), _planes3(src_normal, "src normal"),
                               C.byref(make_pose(dst_pose)), C.byref(make_params(params)),
                               make_plane(dd, "dst depth"), _planes3(dn, "dst normal"),
                               C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_warp_planes")
    return dd, dn


def view_filter(centre_a, centre_b, points: torch.Tensor, min_deg: float = 6.0,
                max_deg: float = 60.0, min_frac: float = 0.2, ctx: Context | None = None,
                stream=None):
    """Eq. (1) on device points (n, 3) float64: (accepted, in range,
    counted). Synchronises the stream to read the two counts."""
    ctx = ctx or default_context(points.device.index or 0)
    if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3 or not points.is_cuda:
        raise ValueError("points must be a (n, 3) float64 device tensor")
    pts = points.contiguous()
    counts = torch.empty(2, dtype=torch.int64, device=points.device)
    ca = (C.c_double * 3)(*[float(v) for v in centre_a])
    cb = (C.c_double * 3)(*[float(v) for v in centre_b])
    st = lib().pms_view_filter(ctx.handle, ca, cb, C.c_void_p(pts.data_ptr()), pts.shape[0],
                               float(min_deg), float(max_deg), C.c_void_p(counts.data_ptr()),
                               C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_view_filter")
    k, c = [int(v) for v in counts.cpu().tolist()]
    return (c > 0 and k >= min_frac * c), k, c


def fuse(depths, poses, voxel: float, ctx: Context | None = None, stream=None):
    """Voxel de-duplication of the points of the depth maps (Sec. III):
    (keep (n_maps, H, W) uint8 device tensor, number of kept points)."""
    ctx = ctx or default_context(depths[0].device.index or 0)
    H, W = depths[0].shape
    dp = (Plane * len(depths))(*[make_plane(d, "depth map") for d in depths])
    keep = torch.empty((len(depths), H, W), dtype=torch.uint8, device=depths[0].device)
    n = torch.empty(1, dtype=torch.int64, device=depths[0].device)
    st = lib().pms_fuse(ctx.handle, W, H, len(depths), dp, _poses(poses), float(voxel),
                        C.c_void_p(keep.data_ptr()), C.c_void_p(n.data_ptr()),
                        C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_fuse")
    return keep, int(n.item())


def coverage(depths, poses, keep, view_pose, out_width: int = 720, out_height: int = 360,
             ctx: Context | None = None, stream=None):
    """Pixels of an out_width x out_height panorama at view_pose marked by
    the kept points: (count, cover (out_height, out_width) uint8 tensor)."""
    ctx = ctx or default_context(depths[0].device.index or 0)
    H, W = depths[0].shape
    dp = (Plane * len(depths))(*[make_plane(d, "depth map") for d in depths])
    cover = torch.empty((out_height, out_width), dtype=torch.uint8, device=depths[0].device)
    n = torch.empty(1, dtype=torch.int64, device=depths[0].device)
    st = lib().pms_coverage(ctx.handle, W, H, len(depths), dp, _poses(poses),
                            C.c_void_p(keep.data_ptr()) if keep is not None else None,
                            C.byref(make_pose(view_pose)), out_width, out_height,
                            C.c_void_p(cover.data_ptr()), C.c_void_p(n.data_ptr()),
                            C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_coverage")
    return int(n.item()), cover


def densify_job(jd: "JobDesc", ctx: Context | None = None, stream=None):
    """One job (with its optional initial planes) through the batch path."""
    return densify_batch([jd], ctx=ctx, stream=stream)[0]


def philox_stream(key0: int, key1: int, ctr0: int, n: int, device: int = 0,
                  ctx: Context | None = None, stream=None) -> torch.Tensor:
    """(n, 4) int64 tensor holding the uint64 Philox4x64-10 blocks."""
    ctx = ctx or default_context(device)
    out = torch.empty((n, 4), dtype=torch.int64, device=f"cuda:{device}")
    st = lib().pms_philox_stream(ctx.handle, int(key0), int(key1), int(ctr0), int(n),
                                 C.c_void_p(out.data_ptr()), C.c_void_p(_stream_handle(stream)))
    ctx.check(st, "pms_philox_stream")
    return out


# ----------------------------------------------------------------------------
# batches
# ----------------------------------------------------------------------------

class JobDesc:
    """One keyframe job for the batch calls: the arguments of ``densify``.
    ``out`` = (depth, normal, cost) tensors; allocated when omitted."""

    def __init__(self, ref, nbrs, ref_pose, nbr_poses, params=None, maps=None, map_poses=None,
                 out=None, init=None):
        self.init = init  # optional (depth (H, W), normal (3, H, W)) initial planes
        self.ref, self.nbrs = ref, list(nbrs)
        self.ref_pose, self.nbr_poses = ref_pose, list(nbr_poses)
        self.params = params
        self.maps, self.map_poses = list(maps or []), list(map_poses or [])
        if len(self.maps) != len(self.map_poses):
            raise ValueError("maps and map_poses differ in length")
        if len(self.nbrs) != len(self.nbr_poses):
            raise ValueError("nbrs and nbr_poses differ in length")
        if out is None:
            H, W = ref.shape
            out = (torch.empty((H, W), dtype=torch.float32, device=ref.device),
                   torch.empty((3, H, W), dtype=torch.float32, device=ref.device),
                   torch.empty((H, W), dtype=torch.float32, device=ref.device))
        self.out = out


def job(ref, nbrs, ref_pose, nbr_poses, params=None, maps=None, map_poses=None, out=None,
        init=None) -> JobDesc:
    return JobDesc(ref, nbrs, ref_pose, nbr_poses, params, maps, map_poses, out, init)


def _job_array(jobs):
    if not 1 <= len(jobs) <= MAX_BATCH:
        raise ValueError(f"a batch holds 1 to {MAX_BATCH} jobs")
    arr = (Job * len(jobs))()
    keep = []
    for i, jd in enumerate(jobs):
        nb = _views(jd.nbrs)
        npz = _poses(jd.nbr_poses)
        mp = (Plane * max(1, len(jd.maps)))(*[make_plane(m, "map") for m in jd.maps])
        mpz = _poses(jd.map_poses)
        prm = make_params(jd.params)
        depth, normal, cost = jd.out
        arr[i].ref = make_image(jd.ref, "ref")
        arr[i].ref_pose = make_pose(jd.ref_pose)
        arr[i].nbrs = C.cast(nb, C.POINTER(Image))
        arr[i].nbr_poses = C.cast(npz, C.POINTER(Pose))
        arr[i].n_nbrs = len(jd.nbrs)
        arr[i].maps = C.cast(mp, C.POINTER(Plane)) if jd.maps else None
        arr[i].map_poses = C.cast(mpz, C.POINTER(Pose)) if jd.maps else None
        arr[i].n_maps = len(jd.maps)
        arr[i].params = C.pointer(prm)
        arr[i].depth_out = make_plane(depth, "depth")
        for k in range(3):
            arr[i].normal_out[k] = make_plane(normal[k], "normal")
        arr[i].cost_out = make_plane(cost, "cost")
        if jd.init is not None:
            idp, inn = jd.init
            arr[i].init_depth = make_plane(idp, "init depth")
            for k in range(3):
                arr[i].init_normal[k] = make_plane(inn[k], "init normal")
        keep += [nb, npz, mp, mpz, prm]
    return arr, keep


def densify_batch(jobs, ctx: Context | None = None, stream=None):
    """Densifies every ``JobDesc`` in one batch; returns their ``out``."""
    ctx = ctx or default_context(jobs[0].ref.device.index or 0)
    arr, keep = _job_array(jobs)
    ctx.check(lib().pms_densify_batch(ctx.handle, arr, len(jobs),
                                      C.c_void_p(_stream_handle(stream))), "pms_densify_batch")
    del keep
    return [jd.out for jd in jobs]


class Batch:
    """A prepared batch (pms_batch_*): device memory and argument tables are
    set up once; ``run`` enqueues the whole batch, as one HIP graph launch
    when ``graph`` is set. The jobs' tensors must outlive the batch."""

    def __init__(self, jobs, ctx: Context | None = None):
        self.ctx = ctx or default_context(jobs[0].ref.device.index or 0)
        self.jobs = list(jobs)
        arr, keep = _job_array(self.jobs)
        h = C.c_void_p()
        self.ctx.check(lib().pms_batch_create(self.ctx.handle, arr, len(jobs), C.byref(h)),
                       "pms_batch_create")
        del keep
        self.handle = h

    def run(self, graph: bool = True, stream=None) -> None:
        self.ctx.check(lib().pms_batch_run(self.handle, int(bool(graph)),
                                           C.c_void_p(_stream_handle(stream))), "pms_batch_run")

    @property
    def nbytes(self) -> int:
        n = C.c_size_t()
        self.ctx.check(lib().pms_batch_bytes(self.handle, C.byref(n)), "pms_batch_bytes")
        return n.value

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().pms_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (pms_server_*): jobs are submitted as they
    arrive and advance one half-sweep per ``step`` together with every other
    admitted job. ``poll`` reports a ticket's state once it is done; the
    job's tensors must stay alive until then."""

    WAITING, RUNNING, DONE = 0, 1, 2

    def __init__(self, arena_bytes: int, max_jobs: int = 64, ctx: Context | None = None):
        self.ctx = ctx or default_context(0)
        h = C.c_void_p()
        self.ctx.check(lib().pms_server_create(self.ctx.handle, int(arena_bytes), int(max_jobs),
                                               C.byref(h)), "pms_server_create")
        self.handle = h
        self._jobs = {}

    def submit(self, jd: JobDesc) -> int:
        arr, keep = _job_array([jd])
        t = C.c_int64()
        self.ctx.check(lib().pms_server_submit(self.handle, arr, C.byref(t)), "pms_server_submit")
        del keep
        self._jobs[t.value] = jd  # keeps the tensors alive
        return t.value

    def step(self, stream=None) -> tuple[int, int]:
        a = C.c_int32()
        w = C.c_int32()
        self.ctx.check(lib().pms_server_step(self.handle, C.c_void_p(_stream_handle(stream)),
                                             C.byref(a), C.byref(w)), "pms_server_step")
        return a.value, w.value

    def poll(self, ticket: int) -> int:
        st = C.c_int32()
        self.ctx.check(lib().pms_server_poll(self.handle, int(ticket), C.byref(st)), "pms_server_poll")
        if st.value == self.DONE:
            self._jobs.pop(ticket, None)
        return st.value

    def stats(self) -> dict:
        t, jt = C.c_int64(), C.c_int64()
        used, peak = C.c_size_t(), C.c_size_t()
        self.ctx.check(lib().pms_server_stats(self.handle, C.byref(t), C.byref(jt), C.byref(used),
                                              C.byref(peak)), "pms_server_stats")
        return {"ticks": t.value, "job_ticks": jt.value, "arena_used": used.value,
                "arena_peak": peak.value,
                "mean_occupancy": jt.value / t.value if t.value else 0.0}

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().pms_server_destroy(self.handle)
            self.handle = None
            self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
