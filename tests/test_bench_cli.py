"""The benchmark's command line and its bookkeeping (no GPU): more than one
GPU is refused with a message, and the committed GEMM traffic record carries
what the roofline object needs."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout == ""


def test_traffic_record_is_tied_to_the_gemm_source():
    sys.path.insert(0, ROOT)
    import bench

    rec = json.load(open(os.path.join(ROOT, "profiles", "gemm_f64_kernel_traffic_D6_chi144.json")))
    for key in ("gemm_source_sha256", "bytes_per_launch", "fetch_bytes_per_launch", "write_bytes_per_launch",
                "counter_scale", "commands"):
        assert key in rec
    assert rec["bytes_per_launch"] > 0
    t = bench.gemm_traffic()
    if rec["gemm_source_sha256"] == bench.gemm_source_hash():
        assert t == rec["bytes_per_launch"]
    else:
        assert t is None  # a changed kernel has no traffic figure until it is profiled again


def test_serving_stream_recipe():
    """The mixed-solve stream the serving figures are quoted on: its sizes
    follow the stated recipe, it is the same on every call, and the 512
    requests hold 37 complex tensors, all at D <= 5."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench

    reqs = bench.serving_requests(512)
    again = bench.serving_requests(512)
    assert [(D, chi, c) for D, chi, c, _ in reqs] == [(D, chi, c) for D, chi, c, _ in again]
    for (D, chi, cplx, A), (_, _, _, B) in zip(reqs, again):
        assert 2 <= D <= 7 and chi in bench.SERVE_CHI and chi >= D * D
        assert A.shape == (2, D, D, D, D) and np.array_equal(A, B)
        assert np.iscomplexobj(A) == cplx
        assert not cplx or D <= 5
    assert sum(c for _, _, c, _ in reqs) == 37
    assert len({D for D, _, _, _ in reqs}) == 6
