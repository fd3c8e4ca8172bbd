"""Derives the atan polynomial used by the kernels' atan2 (pms_kernels.hpp).

atan(t) on [0, tan(pi/8)] is approximated as t + t*s*P(s), s = t^2, with P
of degree 2 chosen to minimise the maximum RELATIVE error (a linear program
on 4001 points; scipy's HiGHS): 6.5e-7 in exact arithmetic, 7.1e-7 in the
float32 evaluation. Larger arguments are reduced to this range by the
kernels (octant symmetry and atan t = pi/4 + atan((t-1)/(t+1))). The
kernels mostly call it on local angles (measured from an anchor pixel),
where relative accuracy keeps a sample within 7.1e-7 of its offset from the
anchor: 4e-6 px at 5 px. (Degree 3 reaches 8e-8 for one more FMA per
angle, two per sample.)
A second, cheaper polynomial (fit_anchor) serves the choice of the anchor
pixel, which needs the angle only to a fraction of a pixel. Run this file
to print the coefficients (as float32) and the errors of the float32
evaluation; the kernels hold the printed values.
"""
import numpy as np
from scipy.optimize import linprog

DEGREE = 2
T_MAX = float(np.tan(np.pi / 8))


def fit(deg: int = DEGREE, n: int = 4000):
    t = np.concatenate([np.linspace(1e-5, T_MAX, n), [T_MAX]])
    s = t * t
    w = np.arctan(t)
    # rows divided by atan(t): |A c - f| <= e atan(t) becomes |A' c - f'| <= e
    A = np.stack([t * s * s ** k for k in range(deg + 1)], axis=1) / w[:, None]
    f = (np.arctan(t) - t) / w
    # the errors (~1e-8) sit below the solver's tolerances: scale columns to
    # unit size and the residuals up
    cs = np.abs(A).max(axis=0)
    scale = 1e6
    cobj = np.zeros(deg + 2)
    cobj[-1] = 1.0
    ones = np.ones((len(t), 1))
    A_ub = np.vstack([np.hstack([scale * A / cs, -ones]), np.hstack([-scale * A / cs, -ones])])
    b_ub = np.concatenate([scale * f, -scale * f])
    res = linprog(cobj, A_ub=A_ub, b_ub=b_ub,
                  bounds=[(None, None)] * (deg + 1) + [(0, None)], method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return np.float32(res.x[:-1] / cs), float(res.x[-1]) / scale


def eval_f32(c, t):
    t = np.asarray(t, dtype=np.float32)
    s = t * t
    p = np.float32(c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = np.float32(p * s + c[k])
    return np.float32(t + np.float32(t * s) * p)


def fit_anchor(deg: int = 3, n: int = 8000):
    """atan(t) on [0, 1] as t * P(t^2) with P of degree `deg`, minimising the
    maximum ABSOLUTE error: the anchor pixel of a warped patch needs its
    angle only to a small fraction of a pixel, and without the reduction to
    [0, tan(pi/8)] the polynomial costs fewer instructions."""
    t = np.linspace(0.0, 1.0, n + 1)
    s = t * t
    A = np.stack([t * s ** k for k in range(deg + 1)], axis=1)
    f = np.arctan(t)
    cs = np.abs(A).max(axis=0)
    scale = 1e4
    cobj = np.zeros(deg + 2)
    cobj[-1] = 1.0
    ones = np.ones((len(t), 1))
    A_ub = np.vstack([np.hstack([scale * A / cs, -ones]), np.hstack([-scale * A / cs, -ones])])
    b_ub = np.concatenate([scale * f, -scale * f])
    res = linprog(cobj, A_ub=A_ub, b_ub=b_ub,
                  bounds=[(None, None)] * (deg + 1) + [(0, None)], method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return np.float32(res.x[:-1] / cs), float(res.x[-1]) / scale


def eval_anchor_f32(c, t):
    t = np.asarray(t, dtype=np.float32)
    s = t * t
    p = np.float32(c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = np.float32(p * s + c[k])
    return np.float32(t * p)


if __name__ == "__main__":
    c, e = fit()
    t = np.linspace(1e-6, T_MAX, 2_000_001).astype(np.float32)
    ref = np.arctan(t.astype(np.float64))
    rel = np.abs(eval_f32(c, t).astype(np.float64) - ref) / ref
    print(f"coefficients (c0..c{DEGREE}):", ", ".join(f"{float(x):.9e}f" for x in c))
    print(f"exact-arithmetic relative error {e:.3e}, float32 evaluation {rel.max():.3e}")
    ca, ea = fit_anchor()
    t = np.linspace(0.0, 1.0, 2_000_001).astype(np.float32)
    err = np.abs(eval_anchor_f32(ca, t).astype(np.float64) - np.arctan(t.astype(np.float64)))
    print("anchor coefficients (a0..a3):", ", ".join(f"{float(x):.9e}f" for x in ca))
    print(f"anchor: exact-arithmetic absolute error {ea:.3e} rad, float32 evaluation {err.max():.3e} rad")
