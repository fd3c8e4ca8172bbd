"""The oracle's pins catch plausible mistakes: each case below plants one
error in a copy of oracle/pmsref.c (a flipped sign, a transposed rotation, a
dropped term, a wrong index, an accepted tie, a copied instead of
re-intersected depth, ...), builds it, and runs the oracle's pin tests
against that build (PMSREF_LIB). Every mutant must make at least one pin
fail. The copy lives in a temporary directory; the oracle itself is never
changed.

UNCAUGHT would list any mutant the pins do not catch, with the reason; it
is empty (the refinement schedule, a reading, is caught through the
brute-force plane sweep it must reach). The two consistency mutants were
caught only once test_oracle_consistency.py existed."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pmsref.c")

# fast files first; pytest -x stops at the first failing pin
PIN_FILES = ["test_oracle_ncc_rng.py", "test_oracle_camera.py", "test_oracle_consistency.py", "test_oracle_warp.py",
             "test_oracle_warp_init.py", "test_oracle_median.py", "test_oracle_view_filter.py",
             "test_oracle_fusion.py", "test_oracle_densify.py"]

MUTANTS = {
    "bearing_y_sign": ("    b[1] = -sin(phi);", "    b[1] = sin(phi);"),
    "project_half_pixel_dropped": ("    *y = H * (PI / 2.0 - phi) / PI - 0.5;", "    *y = H * (PI / 2.0 - phi) / PI;"),
    "relative_rotation_transposed": ("s += nbr->R[3 * i + k] * ref->R[3 * j + k];",
                                     "s += nbr->R[3 * k + i] * ref->R[3 * k + j];"),
    "bilinear_lower_row_tap": ("int y0 = clamp_index(fy, H), y1 = clamp_index(fy + 1.0, H);",
                               "int y0 = clamp_index(fy, H), y1 = clamp_index(fy, H);"),
    "warp_ray_scale_inverted": ("double lambda = c / den;", "double lambda = den / c;"),
    "ncc_variance_mean_dropped": ("vs += (ss[q] - ms) * (ss[q] - ms);", "vs += ss[q] * ss[q];"),
    "aggregate_all_views": ("int k = top_k > 0 ? top_k : (n_views + 1) / 2;", "int k = n_views;"),
    "rng_counter_words_swapped": ("uint64_t ctr[4] = {pixel, iteration, stage, 0}, w[4];",
                                  "uint64_t ctr[4] = {iteration, pixel, stage, 0}, w[4];"),
    "init_uniform_in_depth": ("double rho = 1.0 / p->depth_max + u[0] * (1.0 / p->depth_min - 1.0 / p->depth_max);",
                              "double rho = 1.0 / (p->depth_min + u[0] * (p->depth_max - p->depth_min));"),
    "propagation_copies_depth": ("double dd = cq / den;", "double dd = dq;"),
    "propagation_accepts_ties": ("        if (c < best_c) {\n            best_c = c;\n            best_d = dd;\n            best_n[0] = nq[0];",
                                 "        if (c <= best_c) {\n            best_c = c;\n            best_d = dd;\n            best_n[0] = nq[0];"),
    "consistency_seam_not_folded": ("ddx -= W * floor((ddx + 0.5 * W) / W);", "(void)W;"),
    "consistency_depth_error_absolute": ("ed = fabs(sqrt(dot3(Xb, Xb)) - d) / d;", "ed = fabs(sqrt(dot3(Xb, Xb)) - d);"),
    "refine_range_does_not_shrink": ("double sd = sd0 * pow(p->refine_depth_shrink, k);", "double sd = sd0;"),
}

# planted errors the pins are not expected to catch, and why
UNCAUGHT: dict = {}


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_error_is_caught(name, workdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found exactly once"
    d = workdir / name
    d.mkdir()
    shutil.copy(os.path.join(ROOT, "oracle", "pmsref.h"), d / "pmsref.h")
    (d / "pmsref.c").write_text(src.replace(old, new))
    lib = d / "libpmsref.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                    str(d / "pmsref.c"), "-o", str(lib), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, PMSREF_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *[os.path.join(ROOT, "tests", f) for f in PIN_FILES]],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    caught = res.returncode != 0
    failed = [ln for ln in res.stdout.splitlines() if ln.startswith("FAILED")]
    print(f"{name}: {'caught by ' + failed[0] if caught and failed else 'not caught'}")
    if name in UNCAUGHT:
        pytest.skip(f"not pinned: {UNCAUGHT[name]}" + (" (caught anyway)" if caught else ""))
    assert caught, f"no pin fails with the planted error {name}"
    assert "errors" not in res.stdout.splitlines()[-1] or failed, res.stdout[-2000:]
