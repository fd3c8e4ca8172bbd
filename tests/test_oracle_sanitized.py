"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a copy
of oracle/pmsref.c built with -fsanitize=address,undefined (host code only,
gcc) runs the oracle's pin tests (all but the slow end-to-end densify
ones) through PMSREF_LIB, with the sanitizer runtime preloaded into the
test process. Any out-of-bounds access, use after free, signed overflow,
misaligned load or invalid shift in the oracle fails the run; leak
checking is off (the Python process itself keeps allocations alive)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["test_oracle_ncc_rng.py", "test_oracle_camera.py", "test_oracle_consistency.py",
             "test_oracle_warp.py", "test_oracle_warp_init.py", "test_oracle_median.py",
             "test_oracle_view_filter.py", "test_oracle_fusion.py"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    shutil.copy(os.path.join(ROOT, "oracle", "pmsref.h"), tmp_path / "pmsref.h")
    shutil.copy(os.path.join(ROOT, "oracle", "pmsref.c"), tmp_path / "pmsref.c")
    lib = tmp_path / "libpmsref_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", str(tmp_path / "pmsref.c"), "-o", str(lib), "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, PMSREF_LIB=str(lib), LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *[os.path.join(ROOT, "tests", f) for f in PIN_FILES]],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    print(out[-1500:])
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
