"""Derives the atan polynomial used by the kernels' atan2 (pms_kernels.hpp).

atan(t) on [0, 1] is approximated as t + t*s*P(s), s = t^2, with P of
degree 6 chosen to minimise the maximum RELATIVE error (a linear program on
4001 points; scipy's HiGHS). The kernels only call it on local angles
(measured from an anchor pixel), where relative accuracy is what keeps the
sample coordinates exact to a few 1e-6 px. Run this file to print the
coefficients (as float32) and the error of the float32 evaluation; the
kernels hold the printed values.
"""
import numpy as np
from scipy.optimize import linprog

DEGREE = 6


def fit(deg: int = DEGREE, n: int = 4000):
    t = np.concatenate([np.linspace(1e-4, 1.0, n), [1.0]])
    s = t * t
    A = np.stack([t * s * s ** k for k in range(deg + 1)], axis=1)
    f = np.arctan(t) - t
    w = np.arctan(t)
    cobj = np.zeros(deg + 2)
    cobj[-1] = 1.0
    A_ub = np.vstack([np.hstack([A, -w[:, None]]), np.hstack([-A, -w[:, None]])])
    b_ub = np.concatenate([f, -f])
    res = linprog(cobj, A_ub=A_ub, b_ub=b_ub,
                  bounds=[(None, None)] * (deg + 1) + [(0, None)], method="highs")
    return np.float32(res.x[:-1]), float(res.x[-1])


def eval_f32(c, t):
    t = np.asarray(t, dtype=np.float32)
    s = t * t
    p = np.float32(c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = np.float32(p * s + c[k])
    return np.float32(t + np.float32(t * s) * p)


if __name__ == "__main__":
    c, e = fit()
    t = np.linspace(1e-6, 1.0, 2_000_001).astype(np.float32)
    ref = np.arctan(t.astype(np.float64))
    rel = np.abs(eval_f32(c, t).astype(np.float64) - ref) / ref
    print("coefficients (c0..c6):", ", ".join(f"{float(x):.9e}f" for x in c))
    print(f"exact-arithmetic relative error {e:.3e}, float32 evaluation {rel.max():.3e}")
