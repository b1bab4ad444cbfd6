"""The controller's exact-stage logarithm, sine and cosine (csrc/ctl_math.h),
on the CPU: built from the same header as the kernels (host and device give
the same bits: explicit fused operations, no contraction) and measured against
the C library's long double functions over dense samples of the arguments
that reach them.  Within one unit in the last place they round as a libm
does, so the exact stage's decision equals the reference's (which uses the C
library's double functions) unless a measured TTC lies within about 1e-15 of
a threshold."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not installed")
def test_ctl_math_within_one_ulp(tmp_path):
    exe = str(tmp_path / "ctl_math_check")
    r = subprocess.run([CLANG, "-x", "c++", "-std=c++17", "-O2", "-ffp-contract=off",
                        "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2604_27193_amd", "csrc"),
                        os.path.join(ROOT, "tests", "ctl_math_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    worst = {m.group(1): float(m.group(2))
             for m in re.finditer(r"(\w+) max ulp ([0-9.]+)", out.stdout)}
    assert set(worst) == {"log", "sin", "cos"}, out.stdout
    for name, e in worst.items():
        assert e < 1.0, (name, out.stdout)
