"""The library's host code under AddressSanitizer: libpms is rebuilt with
the sanitizer on its host code only (the device code is compiled as
usual, at -O1 to save time) and the C-ABI tests run against it
(PMS_LIB) with clang's ASan runtime preloaded. They exercise every entry
point's host-side validation on a validation-only context (device -1), so
no kernel runs; any out-of-bounds access or use after free in that host
code aborts the run. Leak checking is off (the Python process keeps its
allocations)."""
import glob
import os
import shlex
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_checks_pass_with_host_asan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    hipcc = "/opt/rocm/bin/hipcc"
    if not rt or not os.path.exists(hipcc):
        pytest.skip("hipcc or clang's ASan runtime is not installed")
    lib = tmp_path / "libpms_asan.so"
    cmd = (f"{hipcc} --offload-arch=gfx950 -O1 -std=c++17 -fPIC -shared "
           "-Xclang -target-feature -Xclang -packed-fp32-ops "
           "-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -Xarch_host -g "
           f"-I {os.path.join(ROOT, 'include')} -o {lib} "
           f"{os.path.join(ROOT, 'paper_2211_16266_amd', 'csrc', 'pms.hip')}")
    subprocess.run(shlex.split(cmd), check=True, capture_output=True)
    env = dict(os.environ, PMS_LIB=str(lib), LD_PRELOAD=rt[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    print(out[-800:])
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
