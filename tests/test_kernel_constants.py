"""The polynomial constants in the kernels are the ones the committed
fitting scripts print (paper_2211_16266_amd/csrc/atan_coeffs.py and
hz_coeffs.py): each fit is re-run and its float32 coefficients must appear
in pms_kernels.hpp as written, and the float32 evaluation must meet the
error the kernels' comments state."""
import os
import re
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_16266_amd", "csrc")
sys.path.insert(0, CSRC)

import atan_coeffs  # noqa: E402
import hz_coeffs  # noqa: E402


def _kernel_floats():
    src = open(os.path.join(CSRC, "pms_kernels.hpp"), encoding="utf-8").read()
    return {np.float32(float(m)) for m in re.findall(r"([-+]?\d\.\d{9}e[-+]\d\d)f", src)}


def test_atan_core_constants():
    c, e = atan_coeffs.fit()
    assert all(np.float32(x) in _kernel_floats() for x in c)
    t = np.linspace(1e-6, atan_coeffs.T_MAX, 200001).astype(np.float32)
    rel = np.abs(atan_coeffs.eval_f32(c, t).astype(np.float64) - np.arctan(t.astype(np.float64)))
    assert (rel / np.arctan(t.astype(np.float64))).max() < 7.5e-7


def test_anchor_atan_constants():
    c, e = atan_coeffs.fit_anchor()
    assert all(np.float32(x) in _kernel_floats() for x in c)
    assert e < 1e-4


def test_horizontal_length_constants():
    c, e = hz_coeffs.fit()
    assert all(np.float32(x) in _kernel_floats() for x in c)
    assert e < 3e-7
    # the error reaches the horizontal length only through y2 u G(u): below
    # the float32 rounding of the length over the whole range
    u = np.linspace(0.0, hz_coeffs.U_MAX, 200001)
    g = hz_coeffs.g_exact(u)
    gf = hz_coeffs.eval_f32(c, u.astype(np.float32)).astype(np.float64)
    hz_rel = np.abs(u * (gf - g)) / np.sqrt(1.0 + u)
    assert hz_rel.max() < 2 ** -24
