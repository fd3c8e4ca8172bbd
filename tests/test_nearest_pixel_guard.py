"""The coverage kernel's guarded FP32 pixel decision (nearest_pixel in
pms_kernels.hpp), emulated in numpy float32 with the kernel's constants and
its atan2 (octant reduction, degree-2 core): wherever the guard admits the
FP32 result it must equal the FP64 formulas' pixel (nearest_pixel64, the
oracle's projection), and the FP32 position error must stay inside the
bound the guard is built on (3e-7 W + 1e-4). Directions are random over
scales of e^-5..e^5, with a tenth near the poles and a tenth next to the
seam behind the camera."""
import numpy as np
import pytest

f32 = np.float32
TAN_PI_8 = f32(0.41421356)


def atan_core(t):
    s = t * t
    p = (s * f32(-1.122516319e-01) + f32(1.971414387e-01)).astype(f32)
    p = (p * s + f32(-3.332550824e-01)).astype(f32)
    return (t * s * p + t).astype(f32)


def atan2_full(y, x):
    ax, ay = np.abs(x), np.abs(y)
    mx = np.maximum(np.maximum(ax, ay), f32(1e-30))
    t = (np.minimum(ax, ay) * (f32(1) / mx)).astype(f32)
    big = t > TAN_PI_8
    u = np.where(big, ((t - f32(1)) * (f32(1) / (t + f32(1)))).astype(f32), t)
    r = (atan_core(u) + np.where(big, f32(0.78539816339744831), f32(0))).astype(f32)
    r = np.where(ay > ax, (f32(1.57079632679489662) - r).astype(f32), r)
    r = np.where(x < 0, (f32(3.14159265358979324) - r).astype(f32), r)
    return np.copysign(r, y).astype(f32)


def pixel64(Y, W, H):
    lam = np.arctan2(Y[:, 0], Y[:, 2])
    phi = np.arctan2(-Y[:, 1], np.hypot(Y[:, 0], Y[:, 2]))
    u = W * (lam + np.pi) / (2 * np.pi) - 0.5
    v = H * (np.pi / 2 - phi) / np.pi - 0.5
    fx = np.floor(u + 0.5)
    fx -= W * np.floor(fx / W)
    xi = fx.astype(np.int64) % W
    yi = np.clip(np.floor(v + 0.5), 0, H - 1).astype(np.int64)
    return xi, yi, u + 0.5, v + 0.5


def pixel32(Y, W, H):
    y0, y1, y2 = (Y[:, k].astype(f32) for k in range(3))
    hz = np.sqrt((y0 * y0 + y2 * y2).astype(f32)).astype(f32)
    lam, phi = atan2_full(y0, y2), atan2_full(-y1, hz)
    fu = (f32(W * 0.15915494) * lam + f32(0.5 * W)).astype(f32)
    fv = (f32(-H * 0.31830989) * phi + f32(0.5 * H)).astype(f32)
    gu, gv = f32(4e-6 * W + 1e-3), f32(4e-6 * H + 1e-3)
    ru, rv = fu - np.floor(fu), fv - np.floor(fv)
    ok = (hz > f32(1e-18) * np.abs(y1)) & (ru > gu) & (ru < 1 - gu) & (rv > gv) & (rv < 1 - gv)
    x = np.floor(fu).astype(np.int64) % W
    y = np.clip(np.floor(fv).astype(np.int64), 0, H - 1)
    return x, y, ok, fu, fv


@pytest.mark.parametrize("W", [720, 1920, 3840, 11582, 6])
def test_guarded_fp32_pixel_equals_fp64(W):
    H = W // 2
    rng = np.random.default_rng(W)
    n = 400_000
    Y = rng.normal(size=(n, 3)) * np.exp(rng.uniform(-5, 5, (n, 1)))
    Y[: n // 10, 0] *= 1e-6
    Y[: n // 10, 2] *= 1e-6
    s = slice(n // 10, n // 5)
    Y[s, 0] = np.abs(Y[s, 0]) * 1e-9 * np.sign(rng.normal(size=n // 10))
    Y[s, 2] = -np.abs(Y[s, 2])
    a, b, u64, v64 = pixel64(Y, W, H)
    c, d, ok, fu, fv = pixel32(Y, W, H)
    assert ((a != c) | (b != d))[ok].sum() == 0
    # the error bound behind the guard, on the general directions
    g = slice(n // 5, n)
    assert np.abs(fu[g] - u64[g]).max() < 3e-7 * W + 1e-4
    assert np.abs(fv[g] - v64[g]).max() < 3e-7 * H + 1e-4
    # the guard bands (both sides of every border, on both axes) are all
    # that falls back there
    gu, gv = 4e-6 * W + 1e-3, 4e-6 * H + 1e-3
    assert ok[g].mean() > 1.0 - 1.5 * (2 * gu + 2 * gv)
