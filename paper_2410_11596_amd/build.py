"""Build libhctm.so in place (hipcc, gfx950).

Usage: python -m paper_2410_11596_amd.build   (or call build())
The library is written next to this file so that it travels with the tree.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhctm.so")

SOURCES = ["gemm.hip", "perm.hip", "linalg.hip", "tensor.hip", "peak.hip", "ctm.cpp", "ctm_complex.cpp", "api.cpp",
           "serve.cpp", "hotrg.cpp"]
ARCH = os.environ.get("HCTM_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=None):
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="hctm_build_")
    objs = []
    procs = []
    try:
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc, *FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj]
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
            if p.returncode != 0:
                failed.append((src, out))
            elif verbose and out.strip():
                print(out)
        if failed:
            msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
            raise RuntimeError("HIP build failed:\n" + msg)
        tmp_lib = os.path.join(tmp, "libhctm.so")
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib]
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if p.returncode != 0:
            raise RuntimeError("link failed:\n" + p.stdout)
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
