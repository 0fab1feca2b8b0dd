"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the plan builder (lpb_plan.cpp: trees, V/U/W/X lists, work items, point
operators) driven through a host stand-in of the point builder on uniform,
clustered and interface-clustered inputs, uniform and adaptive trees, with
every index it hands to the kernels checked; and the oracle's entry points on
small inputs, uniform and adaptive trees.  Any out-of-bounds access, use
after free or undefined behaviour aborts the driver (leak checks are off)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, exe, tmp):
    subprocess.run(cmd, check=True, cwd=ROOT, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], cwd=tmp, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"), reason="needs g++ and HIP headers")
def test_plan_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_driver")
    cmd = ["g++", "-std=c++17", *SAN, "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-o", exe,
           "tests/sanitize/plan_driver.cpp", "paper_2002_01334_amd/csrc/lpb_plan.cpp"]
    out = _run(cmd, exe, tmp_path)
    assert "failures: 0" in out, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", *SAN, "-fopenmp", "-o", exe, "oracle/lpb_oracle.c", "tests/sanitize/oracle_driver.c", "-lm"]
    out = _run(cmd, exe, tmp_path)
    assert "0 failures" in out, out
