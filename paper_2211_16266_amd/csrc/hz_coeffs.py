"""Derives the polynomial the kernels use for the horizontal length of a
warped sample ray (pms_kernels.hpp, the short longitude form).

For a ray (y0, y1, y2) with y2 > 0 and tau = y0 / y2, the horizontal length
is hz = y2 sqrt(1 + tau^2) = y2 + y2 tau^2 G(tau^2), G(u) = 1 / (1 + sqrt(1
+ u)). In the short longitude form |tau| <= tan(pi/8), so u lies in
[0, tan^2(pi/8)]; there G is approximated by a polynomial of degree 3 that
minimises the maximum RELATIVE error (a linear program on 4001 points;
scipy's HiGHS): 2.8e-7, so hz itself is off by at most u G(u) 2.8e-7 of
y2, i.e. 2.7e-8 of hz, below its float32 rounding. hz enters the kernels only through hz - hz_c, the increment
from the anchor, formed as e2 + y2 u G(u) - K_c without cancellation.
Run this file to print the coefficients (as float32) and the error of the
float32 evaluation; the kernels hold the printed values.
"""
import numpy as np
from scipy.optimize import linprog

DEGREE = 3
U_MAX = float(np.tan(np.pi / 8)) ** 2


def g_exact(u):
    return 1.0 / (1.0 + np.sqrt(1.0 + u))


def fit(deg: int = DEGREE, n: int = 4000):
    u = np.linspace(0.0, U_MAX, n + 1)
    g = g_exact(u)
    # rows divided by G(u): |A c - G| <= e G becomes |A' c - 1| <= e
    A = np.stack([u ** k for k in range(deg + 1)], axis=1) / g[:, None]
    f = np.ones_like(u)
    cs = np.abs(A).max(axis=0)
    scale = 1e6
    cobj = np.zeros(deg + 2)
    cobj[-1] = 1.0
    ones = np.ones((len(u), 1))
    A_ub = np.vstack([np.hstack([scale * A / cs, -ones]), np.hstack([-scale * A / cs, -ones])])
    b_ub = np.concatenate([scale * f, -scale * f])
    res = linprog(cobj, A_ub=A_ub, b_ub=b_ub,
                  bounds=[(None, None)] * (deg + 1) + [(0, None)], method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return np.float32(res.x[:-1] / cs), float(res.x[-1]) / scale


def eval_f32(c, u):
    u = np.asarray(u, dtype=np.float32)
    p = np.float32(c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = np.float32(p * u + c[k])
    return p


if __name__ == "__main__":
    c, e = fit()
    u = np.linspace(0.0, U_MAX, 2_000_001).astype(np.float32)
    ref = g_exact(u.astype(np.float64))
    rel = np.abs(eval_f32(c, u).astype(np.float64) - ref) / ref
    print(f"coefficients (c0..c{DEGREE}):", ", ".join(f"{float(x):.9e}f" for x in c))
    print(f"exact-arithmetic relative error {e:.3e}, float32 evaluation {rel.max():.3e}")
