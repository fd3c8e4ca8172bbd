"""The C ABI of libpms, without a GPU: every symbol declared in
include/pms.h is exported, the binding's structs match the header's layout,
and a validation-only context (device -1) rejects every malformed call with
PMS_ERR_INVALID_ARG before anything could be enqueued, while a well-formed
call passes validation and stops at PMS_ERR_DEVICE."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pms.h")

OK, INVALID, OOM, DEVICE, UNSUPPORTED, BUDGET = 0, 1, 2, 3, 4, 5


@pytest.fixture(scope="module")
def B():
    from paper_2211_16266_amd import _binding
    return _binding


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pms_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(B):
    names = _declared_functions()
    assert "pms_densify" in names and "pms_eval_cost" in names and len(names) >= 12
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n


def test_struct_sizes_match_c_layout(B):
    # sizes implied by the header's field order and C alignment rules
    assert C.sizeof(B.Image) == 32
    assert C.sizeof(B.Plane) == 16
    assert C.sizeof(B.Pose) == 96
    assert C.sizeof(B.Params) == 16 + 16 + 8 + 8 + 32 + 4 + 128 + 4 + 16 + 8 + 8 + 8 + 8


def test_default_params(B):
    p = B.default_params()
    assert p["refine_trials"] == 6  # Sec. III-C: six random hypothesis tests
    assert p["n_offsets"] == 8      # Sec. III-C: 8-neighbourhood
    for ox, oy in p["offsets"]:
        assert (abs(ox) + abs(oy)) % 2 == 1


class _Call:
    """A well-formed pms_densify call on fake device pointers."""

    def __init__(self, B, W=64, n=2, dtype=0):
        self.B = B
        H = W // 2
        fake = 0x10000
        esz = {0: 4, 1: 2, 2: 1}[dtype]
        self.ref = B.Image(fake, W, H, W * esz, dtype)
        self.nbrs = (B.Image * n)(*[B.Image(fake + 0x1000 * (j + 1), W, H, W * esz, dtype)
                                    for j in range(n)])
        self.pose = B.make_pose((np.eye(3), np.zeros(3)))
        self.nposes = (B.Pose * n)(*[B.make_pose((np.eye(3), [0.1 * (j + 1), 0, 0])) for j in range(n)])
        self.n = n
        self.params = B.make_params({"patch_size": 7, "patch_stride": 1, "iterations": 2})
        self.depth = B.Plane(fake + 0x9000, W)
        self.normal = (B.Plane * 3)(B.Plane(fake + 0xA000, W), B.Plane(fake + 0xB000, W),
                                    B.Plane(fake + 0xC000, W))
        self.cost = B.Plane(fake + 0xD000, W)
        self.maps = None
        self.map_poses = None
        self.n_maps = 0

    def densify(self, ctx, fn="pms_densify"):
        return getattr(self.B.lib(), fn)(ctx, C.byref(self.ref), C.byref(self.pose), self.nbrs,
                                         self.nposes, self.n, self.maps, self.map_poses,
                                         self.n_maps, C.byref(self.params), self.depth,
                                         self.normal, self.cost, None)


DENSIFY_FNS = ["pms_densify", "pms_densify_noalloc"]


@pytest.fixture()
def vctx(B):
    h = C.c_void_p()
    assert B.lib().pms_context_create(-1, 0, C.byref(h)) == OK
    yield h
    B.lib().pms_context_destroy(h)


@pytest.mark.parametrize("fn", DENSIFY_FNS)
def test_well_formed_call_reaches_the_device_step(B, vctx, fn):
    for dtype in (0, 1, 2):
        assert _Call(B, dtype=dtype).densify(vctx, fn) == DEVICE
    assert b"validation-only" in B.lib().pms_last_error(vctx)


@pytest.mark.parametrize("mutate,expect", [
    (lambda c: setattr(c.ref, "width", 66), INVALID),                 # W != 2H
    (lambda c: setattr(c.ref, "data", None), INVALID),                # null image
    (lambda c: setattr(c.nbrs[1], "height", 16), INVALID),            # size mismatch
    (lambda c: setattr(c.nbrs[0], "dtype", 1), INVALID),              # dtype mismatch
    (lambda c: setattr(c.ref, "dtype", 7), INVALID),                  # unknown dtype
    (lambda c: setattr(c.ref, "pitch_bytes", 10), INVALID),           # pitch too small
    (lambda c: setattr(c, "n", 0), INVALID),                          # no neighbours
    (lambda c: setattr(c, "n", 9), INVALID),                          # too many
    (lambda c: c.nposes[0].t.__setitem__(1, float("nan")), INVALID),  # NaN pose
    (lambda c: c.pose.R.__setitem__(4, float("inf")), INVALID),
    (lambda c: setattr(c.params, "depth_min", 0.0), INVALID),
    (lambda c: setattr(c.params, "depth_max", 0.2), INVALID),         # depth_min >= depth_max
    (lambda c: setattr(c.params, "patch_size", 8), INVALID),          # even patch
    (lambda c: setattr(c.params, "patch_stride", 4), INVALID),        # stride does not divide 2r
    (lambda c: setattr(c.params, "patch_size", 17), UNSUPPORTED),     # 289 samples
    (lambda c: setattr(c.params, "iterations", -1), INVALID),
    (lambda c: setattr(c.params, "refine_trials", 17), INVALID),
    (lambda c: setattr(c.params, "top_k", 3), INVALID),               # > n_nbrs
    (lambda c: c.params.offsets[2].__setitem__(0, 1), INVALID),       # (1,-3): same colour
    (lambda c: setattr(c.params, "n_offsets", 17), INVALID),
    (lambda c: setattr(c.params, "ncc_var_floor", float("nan")), INVALID),
    (lambda c: setattr(c.params, "geo_px", -1.0), INVALID),
    (lambda c: setattr(c.params, "median_radius", 9), INVALID),
    (lambda c: setattr(c.params, "median_rel", -0.1), INVALID),
    (lambda c: setattr(c.depth, "data", None), INVALID),              # null output
    (lambda c: setattr(c.cost, "pitch_elems", 10), INVALID),
    (lambda c: setattr(c, "n_maps", 2), INVALID),                     # maps missing
    (lambda c: setattr(c, "n_maps", 9), INVALID),
])
@pytest.mark.parametrize("fn", DENSIFY_FNS)
def test_malformed_calls_are_rejected_before_launch(B, vctx, mutate, expect, fn):
    c = _Call(B)
    mutate(c)
    assert c.densify(vctx, fn) == expect
    assert B.lib().pms_last_error(vctx) != b""


def test_image_height_limit(B, vctx):
    """A re-laid-out neighbour copy must stay under 2 GiB of 32-bit byte
    offsets: the largest accepted height is PMS_MAX_HEIGHT."""
    hdr = open(HEADER).read()
    hmax = int(re.search(r"#define PMS_MAX_HEIGHT\s+(\d+)", hdr).group(1))
    # (H + 1) rows of 2W + 4 cells of 16 bytes, W = 2H
    assert (hmax + 1) * (4 * hmax + 4) * 16 < 2 ** 31 <= (hmax + 2) * (4 * hmax + 8) * 16
    assert _Call(B, W=2 * hmax).densify(vctx) == DEVICE
    assert _Call(B, W=2 * (hmax + 1)).densify(vctx) == INVALID
    assert b"PMS_MAX_HEIGHT" in B.lib().pms_last_error(vctx)


def test_other_entry_points_validate(B, vctx):
    L = B.lib()
    c = _Call(B)
    assert L.pms_eval_cost(vctx, C.byref(c.ref), C.byref(c.pose), c.nbrs, c.nposes, c.n,
                           C.byref(c.params), c.depth, c.normal, c.cost, None, None) == DEVICE
    bad = B.Plane(0x1234, 8)  # pitch < W
    assert L.pms_eval_cost(vctx, C.byref(c.ref), C.byref(c.pose), c.nbrs, c.nposes, c.n,
                           C.byref(c.params), bad, c.normal, c.cost, None, None) == INVALID
    assert L.pms_halfsweep(vctx, C.byref(c.ref), C.byref(c.pose), c.nbrs, c.nposes, c.n,
                           C.byref(c.params), 1, 0, c.depth, c.normal, c.cost, None) == DEVICE
    assert L.pms_halfsweep(vctx, C.byref(c.ref), C.byref(c.pose), c.nbrs, c.nposes, c.n,
                           C.byref(c.params), 0, 0, c.depth, c.normal, c.cost, None) == INVALID
    assert L.pms_halfsweep(vctx, C.byref(c.ref), C.byref(c.pose), c.nbrs, c.nposes, c.n,
                           C.byref(c.params), 1, 2, c.depth, c.normal, c.cost, None) == INVALID
    maps = (B.Plane * 1)(B.Plane(0x5000, 64))
    mposes = (B.Pose * 1)(c.nposes[0])
    assert L.pms_consistency(vctx, 64, 32, C.byref(c.pose), maps, mposes, 1, C.byref(c.params),
                             c.depth, c.normal, c.cost, None) == DEVICE
    assert L.pms_consistency(vctx, 64, 31, C.byref(c.pose), maps, mposes, 1, C.byref(c.params),
                             c.depth, c.normal, c.cost, None) == INVALID
    assert L.pms_consistency(vctx, 64, 32, C.byref(c.pose), maps, mposes, 0, C.byref(c.params),
                             c.depth, c.normal, c.cost, None) == INVALID
    assert L.pms_philox_stream(vctx, 1, 2, 3, -1, None, None) == INVALID
    assert L.pms_densify(None, None, None, None, None, 0, None, None, 0, None, c.depth, c.normal,
                         c.cost, None) == INVALID


def test_status_strings(B):
    L = B.lib()
    for s in range(6):
        assert L.pms_status_string(s)
    assert L.pms_status_string(99) == b"unknown status"


def test_struct_sizes_of_batch_types(B):
    # pms_job: image 32 + pose 96 + 2 pointers + int (padded to 8) + 2 pointers
    # + int (padded) + params pointer + 5 output planes + 4 initial planes
    assert C.sizeof(B.Job) == 32 + 96 + 16 + 8 + 16 + 8 + 8 + 5 * 16 + 4 * 16
    assert C.sizeof(B.Schedule) == 12


def _job(B, c, depth_at=0x9000):
    """A pms_job over the fake buffers of a _Call; outputs at `depth_at`."""
    j = B.Job()
    j.ref = c.ref
    j.ref_pose = c.pose
    j.nbrs = C.cast(c.nbrs, C.POINTER(B.Image))
    j.nbr_poses = C.cast(c.nposes, C.POINTER(B.Pose))
    j.n_nbrs = c.n
    j.n_maps = 0
    j.params = C.pointer(c.params)
    W = c.ref.width
    j.depth_out = B.Plane(0x100000 + depth_at, W)
    for k in range(3):
        j.normal_out[k] = B.Plane(0x100000 + depth_at + 0x100 * (k + 1), W)
    j.cost_out = B.Plane(0x100000 + depth_at + 0x400, W)
    return j


def test_batch_entry_points_validate(B, vctx):
    L = B.lib()
    calls = [_Call(B, W=64), _Call(B, W=128, n=3, dtype=1)]
    jobs = (B.Job * 2)(_job(B, calls[0], 0x1000), _job(B, calls[1], 0x2000))
    assert L.pms_densify_batch(vctx, jobs, 2, None) == DEVICE
    assert L.pms_densify_batch(vctx, jobs, 0, None) == INVALID
    assert L.pms_densify_batch(vctx, None, 2, None) == INVALID
    h = C.c_void_p()
    assert L.pms_batch_create(vctx, jobs, 2, C.byref(h)) == DEVICE
    assert not h.value
    sc = B.Schedule()
    best = C.c_double()
    assert L.pms_autotune(vctx, jobs, 2, 1, 0, C.byref(sc), C.byref(best), None) == DEVICE
    assert L.pms_autotune(vctx, jobs, 2, 0, 0, C.byref(sc), C.byref(best), None) == INVALID
    # a malformed job names itself
    calls[1].params.patch_size = 8
    assert L.pms_densify_batch(vctx, jobs, 2, None) == INVALID
    assert L.pms_last_error(vctx).startswith(b"job 1:")
    calls[1].params.patch_size = 7
    # two jobs writing one plane
    jobs[1].cost_out = jobs[0].cost_out
    assert L.pms_densify_batch(vctx, jobs, 2, None) == INVALID
    jobs[1].cost_out = B.Plane(0x100000 + 0x2400, 128)
    # a consistency map that another job writes
    maps = (B.Plane * 1)(jobs[0].depth_out)
    mposes = (B.Pose * 1)(calls[1].nposes[0])
    maps[0].pitch_elems = 128
    jobs[1].maps = C.cast(maps, C.POINTER(B.Plane))
    jobs[1].map_poses = C.cast(mposes, C.POINTER(B.Pose))
    jobs[1].n_maps = 1
    assert L.pms_densify_batch(vctx, jobs, 2, None) == INVALID
    jobs[1].n_maps = 0
    assert L.pms_densify_batch(vctx, jobs, 2, None) == DEVICE


def test_schedule_round_trip_and_rejection(B, vctx):
    L = B.lib()
    sc = B.Schedule()
    assert L.pms_get_schedule(vctx, C.byref(sc)) == OK
    assert (sc.wave_rows, sc.waves_x, sc.lanes_per_pixel) == (4, 2, 4)
    for bad in [(3, 2, 4), (32, 2, 4), (4, 8, 4), (4, 3, 4), (4, 2, 1), (0, 2, 4), (4, 2, 3), (4, 2, 16)]:
        assert L.pms_set_schedule(vctx, C.byref(B.Schedule(*bad))) == INVALID
    for good in [(16, 1, 2), (8, 1, 8), (4, 2, 4)]:
        assert L.pms_set_schedule(vctx, C.byref(B.Schedule(*good))) == OK
        assert L.pms_get_schedule(vctx, C.byref(sc)) == OK
        assert (sc.wave_rows, sc.waves_x, sc.lanes_per_pixel) == good


def test_server_entry_points_validate(B, vctx):
    L = B.lib()
    h = C.c_void_p()
    assert L.pms_server_create(vctx, 1 << 26, 0, C.byref(h)) == INVALID
    assert L.pms_server_create(vctx, 1 << 10, 4, C.byref(h)) == INVALID
    assert L.pms_server_create(vctx, 1 << 26, 4, C.byref(h)) == DEVICE
    assert not h.value
    assert L.pms_server_submit(None, None, None) == INVALID
    assert L.pms_server_step(None, None, None, None) == INVALID
    st = C.c_int32()
    assert L.pms_server_poll(None, 1, C.byref(st)) == INVALID


def test_warp_and_init_planes_validate(B, vctx):
    L = B.lib()
    c = _Call(B)
    W, H = 64, 32
    src = (B.Plane * 3)(B.Plane(0x20000, W), B.Plane(0x21000, W), B.Plane(0x22000, W))
    dst = (B.Plane * 3)(B.Plane(0x30000, W), B.Plane(0x31000, W), B.Plane(0x32000, W))
    sd, dd = B.Plane(0x23000, W), B.Plane(0x33000, W)
    args = lambda w, h, s_d, d_d: (vctx, w, h, C.byref(c.pose), s_d, src, C.byref(c.nposes[0]),
                                   C.byref(c.params), d_d, dst, None)
    assert L.pms_warp_planes(*args(W, H, sd, dd)) == DEVICE
    assert L.pms_warp_planes(*args(W, 31, sd, dd)) == INVALID
    assert L.pms_warp_planes(*args(W, H, sd, B.Plane(0x21000, W))) == INVALID  # overlap
    assert L.pms_warp_planes(*args(W, H, B.Plane(0x23000, 8), dd)) == INVALID  # pitch < W
    # a job's initial planes: one pitch for all four, not an output of the batch
    j = _job(B, c, 0x1000)
    j.init_depth = B.Plane(0x40000, W)
    for k in range(3):
        j.init_normal[k] = B.Plane(0x41000 + 0x1000 * k, W)
    jobs = (B.Job * 1)(j)
    assert L.pms_densify_batch(vctx, jobs, 1, None) == DEVICE
    jobs[0].init_normal[1] = B.Plane(0x42000, W + 8)
    assert L.pms_densify_batch(vctx, jobs, 1, None) == INVALID
    jobs[0].init_normal[1] = B.Plane(0x42000, W)
    jobs[0].init_depth = jobs[0].depth_out
    assert L.pms_densify_batch(vctx, jobs, 1, None) == INVALID


def test_fusion_entry_points_validate(B, vctx):
    L = B.lib()
    c = _Call(B)
    W, H = 64, 32
    maps = (B.Plane * 2)(B.Plane(0x50000, W), B.Plane(0x51000, W))
    poses = (B.Pose * 2)(c.pose, c.nposes[0])
    keep, cnt = C.c_void_p(0x60000), C.c_void_p(0x61000)
    assert L.pms_fuse(vctx, W, H, 2, maps, poses, 0.02, keep, cnt, None) == DEVICE
    assert L.pms_fuse(vctx, W, H, 2, maps, poses, 0.0, keep, cnt, None) == INVALID
    assert L.pms_fuse(vctx, W, H, 9, maps, poses, 0.02, keep, cnt, None) == INVALID
    assert L.pms_fuse(vctx, W, 30, 2, maps, poses, 0.02, keep, cnt, None) == INVALID
    assert L.pms_fuse(vctx, W, H, 2, maps, poses, 0.02, None, cnt, None) == INVALID
    cov = C.c_void_p(0x70000)
    assert L.pms_coverage(vctx, W, H, 2, maps, poses, keep, C.byref(c.pose), 720, 360, cov, cnt,
                          None) == DEVICE
    assert L.pms_coverage(vctx, W, H, 2, maps, poses, None, C.byref(c.pose), 720, 300, cov, cnt,
                          None) == INVALID


def test_struct_offsets_match_the_compiled_header(B, tmp_path):
    """Every field offset and struct size of the binding's ctypes structs
    equals what a C compiler makes of include/pms.h (gcc, host ABI)."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    structs = {"pms_image": B.Image, "pms_plane": B.Plane, "pms_pose": B.Pose,
               "pms_params": B.Params, "pms_job": B.Job, "pms_schedule": B.Schedule}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pms.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            cname, field, val = ln.split()
            got[(cname, field)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
