"""Host-only checks of the block planners (CPU, no GPU): tests/host/*.cpp are
compiled with the host C++ compiler against the library's headers and run.

check_plans.cpp: the Z2 block layout against dense arithmetic (per-sector
products equal the dense contraction over the shared leg, block permutations
equal the dense transposition, for total parities 0 and 1 and every leg
order and row split), and a contraction written straight into a permuted
layout (the enlarged corners and the edge renormalisation) stores every
element where forming the product and permuting it would, bit for bit, each
element once; sectors with an empty contraction are left to the separate
copy; packing between a plain array and the blocks keeps exactly the
entries of the tensor's total parity, for plain arrays stored row-major and
with their legs reversed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INCLUDE = "/opt/rocm/include"


def _compiler():
    for c in ("g++", "c++", "clang++"):
        p = shutil.which(c)
        if p:
            return p
    return None


@pytest.mark.parametrize("src", ["check_plans.cpp"])
def test_host_planner(tmp_path, src):
    cxx = _compiler()
    if cxx is None or not os.path.isdir(os.path.join(ROCM_INCLUDE, "hip")):
        pytest.skip("no host C++ compiler or HIP headers")
    exe = str(tmp_path / "check")
    cmd = [cxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INCLUDE}",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(ROOT, 'paper_2410_11596_amd', 'csrc')}",
           os.path.join(ROOT, "tests", "host", src), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout
