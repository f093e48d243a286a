#!/usr/bin/env python3
"""CTMRG iterations per second on one MI355X: Z2 (Hermitian) form vs plain form.

Workload: directional CTMRG on a 1x1 unit cell, real iPEPS with d = 2, D = 6
(joined bra-ket leg 36 = 21 even + 15 odd), chi = 144, FP64, i.i.d. N(0,1)
tensor (seed 0, max-abs normalised).  One step = one CTMRG iteration = four
directional moves.  Both forms start from the same traced-boundary
environment; W untimed iterations bring every bond to chi, then K iterations
are timed between two device synchronisations.

Printed: one JSON line with the Z2 throughput as `value`, the plain-form
throughput and their ratio, the live MFMA roofline of the FP64 GEMM kernel
(algorithmic block-product flops over the summed HIP-event durations of its
launches in the timed Z2 region) and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PHASES = ["corners", "halves", "svd", "renormalise", "convergence"]
METRIC = "CTMRG steps/s Z2 vs dense (FP64 vs mixed) at D=6 χ=144; p50/p99 solve latency"
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak (datasheet)
GEMM_SOURCE = os.path.join(ROOT, "paper_2410_11596_amd", "csrc", "gemm.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f64_kernel_traffic_D6_chi144.json")


def gemm_source_hash():
    with open(GEMM_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def gemm_traffic():
    """HBM bytes per GEMM launch measured with the FETCH_SIZE / WRITE_SIZE
    counters for the current kernel source, or None when there is no
    measurement of this source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("gemm_source_sha256") != gemm_source_hash():
        return None
    return t.get("bytes_per_launch")


def copy_check(nbytes):
    """A plain device copy of nbytes (read nbytes, write nbytes), three times:
    the reference the HBM counters are scaled by."""
    import torch

    from paper_2410_11596_amd import binding

    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        binding.dev_copy(src, dst, [n], [1], [1])
    torch.cuda.synchronize()
    assert bool((dst == 1.0).all())


def measured_peaks():
    """The chip's own ceilings, measured with the library's probes on the
    same stream as everything else: the FP64 matrix-core rate of back-to-back
    independent MFMAs with no memory traffic (2048 workgroups, eight per CU),
    the HBM bandwidth of a 1 GiB contiguous copy (read + write), and the GEMM
    kernel's own rate on one 8192^3 FP64 product.  Medians of five timed
    launches after two untimed ones."""
    import torch

    from paper_2410_11596_amd import binding

    def timed(fn, reps=5, warm=2):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts))

    blocks, iters = 2048, 32
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    flops = binding.dev_mfma_probe(sink, blocks, 1)  # builds the kernel; flops of one round
    flops = flops * iters
    t_mfma = timed(lambda: binding.dev_mfma_probe(sink, blocks, iters))
    assert bool(torch.isfinite(sink).all())
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    t_copy = timed(lambda: binding.dev_stream_probe(src, dst, n))
    assert bool((dst == 1.0).all())
    del src, dst
    m = 8192
    a = torch.rand(m, m, dtype=torch.float64, device="cuda")
    b = torch.rand(m, m, dtype=torch.float64, device="cuda")
    c = torch.empty(m, m, dtype=torch.float64, device="cuda")
    t_gemm = timed(lambda: binding.dev_gemm(a, b, c, m, m, m, m, m, m), reps=3, warm=1)
    del a, b, c
    return {"fp64_mfma_tflops": flops / t_mfma / 1e12, "hbm_copy_gbps": 2 * 8 * n / t_copy / 1e9,
            "gemm_f64_8192_tflops": 2.0 * m ** 3 / t_gemm / 1e12,
            "probes": "hctm_dev_mfma_probe (2048 workgroups x 4 waves, 1024 rounds of 8 independent "
                      "16x16x4 FP64 MFMAs each), hctm_dev_stream_probe (1 GiB copy, one 16-byte non-temporal load "
                      "and store per thread), "
                      "hctm_dev_gemm 8192^3; medians of 5 (GEMM: 3) timed launches"}


def event_pair_overhead(n=200):
    """Mean duration of an empty HIP event pair on the current stream, right
    after a small kernel (the fixed cost inside every timed launch)."""
    import torch

    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for _ in range(n):
        x.add_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        e1.record()
        e1.synchronize()
        t += e0.elapsed_time(e1) * 1e-3
    return t / n


def time_form(A, chi, form, steps, warmup, profile):
    import torch

    from paper_2410_11596_amd import CTMRG

    g = CTMRG(A, chi, form=form, profile=profile)
    g.step(warmup)
    torch.cuda.synchronize()
    g.gemm_stats(reset=True)
    h0 = g.svd_health()
    nrec0 = g.num_records()
    # one iteration per call, an event on the library's stream between them:
    # the window's total and each iteration's own time
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    phases = np.zeros(len(PHASES))
    for i in range(steps):
        g.step(1)
        ev[i + 1].record()
        phases += g.timing()  # GPU seconds per phase of this iteration
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    stats = g.gemm_stats()
    split = g.sector_dims(3)
    h1 = g.svd_health()
    recs = [g.record(m) for m in range(nrec0, g.num_records())]
    g.close()
    stats["svd_unconverged_in_window"] = h1[0] - h0[0]
    stats["multiplet_splits_in_window"] = h1[1] - h0[1]
    stats["truncations_in_window"] = len(recs)
    # per truncation, the larger of the two sectors' counts
    stats["svd_in_window"] = {
        "truncations": len(recs),
        "with_subspace_iteration": int(sum(max(r["iters"]) > 0 for r in recs)),
        "subspace_iterations_mean": float(np.mean([max(r["iters"]) for r in recs])) if recs else 0.0,
        "jacobi_sweeps_mean": float(np.mean([max(r["sweeps"]) for r in recs])) if recs else 0.0,
        "matrix_applied_through_corners": int(sum(r["implicit"] for r in recs)),
    }
    stats["iteration_ms"] = {"p10": float(np.percentile(per, 10)), "p50": float(np.percentile(per, 50)),
                             "p90": float(np.percentile(per, 90))}
    return (t1 - t0), stats, phases, split


def late_iterations(A, chi, skip, steps):
    """Time per iteration later in the same solve (iterations skip+1 ..
    skip+steps): the cost of an iteration falls as the cuts converge (the
    decomposed matrix is applied through the corners, fewer subspace
    iterations)."""
    import torch

    from paper_2410_11596_amd import CTMRG

    g = CTMRG(A, chi)
    g.step(skip)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.close()
    return {"iterations": [skip + 1, skip + steps], "ms_per_step": 1e3 * (t1 - t0) / steps,
            "value": steps / (t1 - t0), "unit": "CTMRG iterations/s"}


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    """Stored FP64 oracle outputs for D = 6, chi = 144 (written by
    tests/golden/make_ctmrg_d6_chi144.py from the oracle alone)."""
    with open(os.path.join(GOLDEN_DIR, f"ctmrg_d6_chi144_{name}.json")) as f:
        return json.load(f)


def _obs_err(g, ob, h):
    o = np.concatenate([g.rdm1().ravel(), g.rdm2("h").ravel(), g.rdm2("v").ravel()])
    r = np.concatenate([np.ravel(ob["rho1"]), np.ravel(ob["rho2_h"]), np.ravel(ob["rho2_v"])])
    return float(np.abs(o - r).max()), float(abs(g.energy(h) - ob["energy"]))


def mixed_precision(A, chi, steps, warmup, golden, refine_max=40, tol=1e-10, precision="fp32"):
    """Block products of the moves in FP32 or BF16x3: timed like the FP64
    form; the error of the RDMs and the energy against the FP64 oracle
    (stored outputs of the same tensor) after 12 iterations in low precision,
    and after 3 more FP64 iterations (the refinement) against the oracle after
    15; the FP64 form's own error at the same points beside it; then the FP64
    iterations until the corner spectra change by less than tol."""
    import torch

    from paper_2410_11596_amd import CTMRG, inputs

    h = inputs.heisenberg_bond_matrix()
    g32 = CTMRG(A, chi, precision=precision)
    g32.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g32.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g32.close()
    res = {"value": steps / (t1 - t0), "unit": "CTMRG iterations/s", "ms_per_step": 1e3 * (t1 - t0) / steps,
           "precision": {"fp32": "FP32 block products of the moves (FP32 MFMA, FP32 accumulation)",
                         "bf16x3": "BF16x3 block products of the moves (hi*hi + hi*lo + lo*hi on BF16 MFMA, "
                                   "FP32 accumulation)"}[precision] + "; FP64 SVD, normalisation and observables",
           "reference": "FP64 oracle: " + golden["input"]}
    n_lo = 12
    g = CTMRG(A, chi, precision=precision).step(n_lo)
    e_rdm, e_e = _obs_err(g, golden["observables"][str(n_lo)], h)
    g.set_precision("fp64").step(3)
    a_rdm, a_e = _obs_err(g, golden["observables"][str(n_lo + 3)], h)
    n = 3
    while not g.converged(tol)[0] and n < refine_max:
        g.step(1)
        n += 1
    g.close()
    f = CTMRG(A, chi).step(n_lo)
    f_rdm, f_e = _obs_err(f, golden["observables"][str(n_lo)], h)
    f.step(3)
    f3_rdm, f3_e = _obs_err(f, golden["observables"][str(n_lo + 3)], h)
    f.close()
    res["error_vs_oracle"] = {
        "after_12_low_precision": {"max_abs_rdm": e_rdm, "abs_energy": e_e},
        "after_3_fp64_refinement": {"max_abs_rdm": a_rdm, "abs_energy": a_e},
        "fp64_form_after_12": {"max_abs_rdm": f_rdm, "abs_energy": f_e},
        "fp64_form_after_15": {"max_abs_rdm": f3_rdm, "abs_energy": f3_e},
        "targets": {"before_refinement": 1e-6, "after_refinement": 1e-10},
    }
    res["refinement_iterations_to_delta_1e-10"] = n
    return res


def large_shape(D=8, chi=256, warmup=2, steps=2):
    """The largest workload: D = 8 (joined leg 64 = 36 even + 28 odd),
    chi = 256, 1x1 cell, i.i.d. tensor seed 0, Z2 form with BF16x3 block
    products and in FP64: time per iteration after the bonds have reached chi,
    the device memory the solve holds (its workspace, the peak of torch's
    allocator over the run) and the block products' throughput in the timed
    iterations (algorithmic 2 M N K flops over the summed launch times; BF16x3
    issues three BF16 matrix products per product)."""
    import torch

    from paper_2410_11596_amd import CTMRG, inputs, workspace_size

    A = inputs.iid_tensor(2, D, 0)
    res = {"workload": f"Z2 directional CTMRG, 1x1 cell, real iPEPS d=2 D={D}, chi={chi}, i.i.d. seed 0",
           "workspace_bytes": workspace_size(2, D, chi)}
    for prec in ("bf16x3", "fp64"):
        torch.cuda.reset_peak_memory_stats()
        g = CTMRG(A, chi, precision=prec, profile=True)
        g.step(warmup)
        torch.cuda.synchronize()
        g.gemm_stats(reset=True)
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = g.gemm_stats()
        r = {"ms_per_step": 1e3 * (t1 - t0) / steps, "value": steps / (t1 - t0), "unit": "CTMRG iterations/s",
             "phases_ms_per_step": {k: 1e3 * v / steps for k, v in zip(PHASES, g.timing().tolist())},
             "kept_last": list(g.records()[-1]["kept"]), "svd_health": list(g.svd_health()),
             "peak_device_bytes": int(torch.cuda.max_memory_allocated()),
             "gemm_algorithmic_tflops": st["flops"] / st["seconds"] / 1e12 if st["seconds"] > 0 else None,
             "gemm_share_of_step": st["seconds"] / (t1 - t0), "note": "profiled pass (HIP events per GEMM launch)"}
        g.close()
        res[prec] = r
    return res


def complex_case(D=5, chi=100, warmup=5, steps=10):
    """Complex iPEPS tensors (Sec. II C) in the real representation of their
    Hermitian structure: Z2 FP64 time per iteration of a complex i.i.d.
    tensor (real and imaginary parts N(0,1), seed 0) against the real path on
    a real i.i.d. tensor of the same shape (seed 0), after `warmup`
    iterations, with the iterations' subspace iterations and kept sizes."""
    import torch

    from paper_2410_11596_amd import CTMRG, inputs

    res = {"workload": f"Z2 directional CTMRG, 1x1 cell, d=2 D={D}, chi={chi}, FP64: complex i.i.d. tensor "
                       f"(real and imaginary parts N(0,1), seed 0) against a real i.i.d. tensor (seed 0)"}
    for label, A in (("complex", inputs.complex_iid_tensor(2, D, 0)), ("real", inputs.iid_tensor(2, D, 0))):
        g = CTMRG(A, chi)
        g.step(warmup)
        torch.cuda.synchronize()
        n0 = g.num_records()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        recs = [g.record(m) for m in range(n0, g.num_records())]
        res[label] = {"ms_per_step": 1e3 * (t1 - t0) / steps, "value": steps / (t1 - t0), "unit": "CTMRG iterations/s",
                      "kept_last": list(recs[-1]["kept"]),
                      "subspace_iterations_mean": float(np.mean([max(r["iters"]) for r in recs]))}
        g.close()
    res["complex_over_real_time"] = res["complex"]["ms_per_step"] / res["real"]["ms_per_step"]
    return res


def c4v_scheme(D, chi, steps, warmup, tol=1e-10, max_iter=200):
    """The C4v scheme (one corner, one edge, one truncation per iteration)
    against the directional moves, both Z2 FP64, on a C4v-symmetric tensor of
    the same size: time per iteration, then iterations and wall time to
    delta < tol from the start and the largest RDM difference there."""
    import torch

    from paper_2410_11596_amd import CTMRG, inputs

    A = inputs.c4v_iid_tensor(2, D, 0)
    res = {"workload": f"C4v-symmetrised real iPEPS d=2 D={D}, chi={chi}, Z2 FP64"}
    conv = {}
    for name, c4 in (("c4v", True), ("directional", False)):
        g = CTMRG(A, chi, c4v=c4)
        g.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res[name + "_ms_per_iteration"] = 1e3 * (t1 - t0) / steps
        g.close()
        g = CTMRG(A, chi, c4v=c4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 0
        while n < max_iter:
            g.step(1)
            n += 1
            if g.converged(tol)[0]:
                break
        t1 = time.perf_counter()
        res[name + "_iterations_to_delta_1e-10"] = n
        res[name + "_seconds_to_delta_1e-10"] = t1 - t0
        conv[name] = np.concatenate([g.rdm1().ravel(), g.rdm2("h").ravel(), g.rdm2("v").ravel()])
        g.close()
    res["speedup_per_iteration"] = res["directional_ms_per_iteration"] / res["c4v_ms_per_iteration"]
    res["speedup_to_solution"] = res["directional_seconds_to_delta_1e-10"] / res["c4v_seconds_to_delta_1e-10"]
    res["max_abs_rdm_diff_at_solution"] = float(np.abs(conv["c4v"] - conv["directional"]).max())
    return res


def hotrg_speedup(chis=(32, 48, 64), D=2, steps=4, warmup=6, probe_chi=32):
    """HOTRG (include/hctm_hotrg.h): time per step of the Z2 and the plain
    form once the bonds have reached chi, and their ratio, for several chi
    (Fig. 4(c) of the paper); at probe_chi the symmetry error of both forms
    with the probe b and their Heisenberg bond energies (Fig. 3)."""
    import torch

    from paper_2410_11596_amd import HOTRG, inputs

    A = inputs.iid_tensor(2, D, 0)
    res = {"workload": f"HOTRG on the double layer of an i.i.d. d=2 D={D} tensor, FP64; {warmup} steps to "
                       f"reach chi, then {steps} timed steps", "chi": list(chis)}
    for form in ("z2", "dense"):
        ms, kept = [], []
        for chi in chis:
            h = HOTRG(A, chi, form=form)
            h.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.step(steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms.append(1e3 * (t1 - t0) / steps)
            kept.append(list(h.records()[-1]["kept"]))
            h.close()
        res[form + "_ms_per_step"] = ms
        res[form + "_kept_last"] = kept
        p = HOTRG(A, probe_chi, form=form, probes=True, bond=inputs.heisenberg_bond_matrix())
        p.step(warmup + steps)
        res[form + "_sym_error_chi%d" % probe_chi] = p.sym_error()
        res[form + "_log_z_chi%d" % probe_chi] = p.log_z()
        res[form + "_energy_chi%d" % probe_chi] = p.energy()
        p.close()
    res["z2_over_dense"] = [d / z for d, z in zip(res["dense_ms_per_step"], res["z2_ms_per_step"])]
    res["abs_energy_difference_chi%d" % probe_chi] = abs(res["z2_energy_chi%d" % probe_chi] -
                                                          res["dense_energy_chi%d" % probe_chi])
    return res


def hotrg_by_d(Ds=(2, 4, 6), chi=64, steps=4, warmup=6):
    """HOTRG Z2 / plain time per step at one chi for several D (the paper:
    the speed-up hardly depends on D, which only enters the first step)."""
    import torch

    from paper_2410_11596_amd import HOTRG, inputs

    res = {"chi": chi, "D": list(Ds), "z2_ms_per_step": [], "dense_ms_per_step": []}
    for D in Ds:
        A = inputs.iid_tensor(2, D, 0)
        for form in ("z2", "dense"):
            h = HOTRG(A, chi, form=form)
            h.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.step(steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            res[form + "_ms_per_step"].append(1e3 * (t1 - t0) / steps)
            h.close()
    res["z2_over_dense"] = [d / z for d, z in zip(res["dense_ms_per_step"], res["z2_ms_per_step"])]
    return res


SERVE_CHI = (16, 32, 64, 100, 144, 196)


def serving_requests(n_req, seed=11, complex_share=0.1):
    """The mixed-solve stream: D uniform in {2, ..., 7}, chi uniform in
    {16, 32, 64, 100, 144, 196} redrawn until chi >= D^2, i.i.d. N(0,1)
    tensors (seed 1000 + i), and with probability complex_share a complex
    tensor (real and imaginary parts N(0,1)) when D <= 5."""
    from paper_2410_11596_amd import inputs

    rng = np.random.default_rng(seed)
    reqs = []
    while len(reqs) < n_req:
        D = int(rng.integers(2, 8))
        chi = int(rng.choice(SERVE_CHI))
        if chi < D * D:
            continue
        cplx = D <= 5 and rng.random() < complex_share
        i = len(reqs)
        A = inputs.complex_iid_tensor(2, D, 1000 + i) if cplx else inputs.iid_tensor(2, D, 1000 + i)
        reqs.append((D, chi, cplx, A))
    return reqs


def serving(n_req, rate, max_active=8, tol=1e-10, max_iter=60, seed=11, baseline_n=None):
    """A stream of n_req solves (serving_requests) with Poisson arrivals at
    `rate` per second, each run to delta < tol (at most max_iter iterations)
    and its RDMs read: latency = result ready - arrival.  Served: the Z2 form
    through the server, up to max_active solves at a time, admitted by
    workspace.  Baseline: the first baseline_n requests of the same stream,
    one at a time, in the plain (dense) FP64 form (the complex ones, which
    have no plain GPU form, in their Z2 form), queued behind each other."""
    import ctypes

    import torch

    from paper_2410_11596_amd import Server, workspace_size
    from paper_2410_11596_amd.binding import lib, CtmOpts, _check

    torch.cuda.init()  # before the server's streams: the baseline runs through torch's device
    reqs = serving_requests(n_req, seed)
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0 / rate, n_req)

    def ws(D, chi, cplx, form):
        if not cplx:
            return workspace_size(2, D, chi, form=form)
        o = CtmOpts()
        _check(lib().ctm_opts_default(ctypes.byref(o)))
        n = ctypes.c_size_t()
        _check(lib().ctm_workspace_size_complex(2, D, chi, ctypes.byref(o), ctypes.byref(n)))
        return n.value

    big = max(ws(D, chi, c, "z2") for D, chi, c, _ in reqs)
    out = {"requests": n_req, "arrival_rate_per_s": rate, "tol": tol, "max_iter": max_iter,
           "mix": "D uniform in {2..7}, chi uniform in {16,32,64,100,144,196} with chi >= D^2, i.i.d. N(0,1) "
                  "tensors, 10% complex (real and imaginary parts N(0,1)) at D <= 5",
           "complex_requests": int(sum(c for _, _, c, _ in reqs))}
    nb = n_req if baseline_n is None else min(baseline_n, n_req)
    arrive = np.cumsum(gaps)
    # served: the Z2 form through the server, up to max_active at a time
    pool = max_active * big + (1 << 24)
    srv = Server(pool, max_active=max_active)
    t0 = time.perf_counter()
    ids = []
    for (D, chi, cplx, A), at in zip(reqs, arrive):
        time.sleep(max(0.0, t0 + at - time.perf_counter()))
        ids.append(srv.submit(A, chi, form="z2", tol=tol, max_iter=max_iter))
        if len(ids) % 32 == 0:
            print(f"serving concurrent_z2: {len(ids)}/{n_req} submitted", file=sys.stderr, flush=True)
    res = []
    for i in ids:
        res.append(srv.wait(i))
        if len(res) % 32 == 0:
            print(f"serving concurrent_z2: {len(res)}/{n_req} done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    srv.close()
    lat = np.array([r["t_end"] - r["t_submit"] for r in res])
    out["concurrent_z2"] = {"requests": n_req, "max_active": max_active,
                            "p50_latency_s": float(np.percentile(lat, 50)),
                            "p99_latency_s": float(np.percentile(lat, 99)), "solves_per_s": n_req / (t1 - t0),
                            "wall_s": t1 - t0, "failed": int(sum(r["status"] != 0 for r in res)),
                            "converged": int(sum(r["converged"] for r in res)),
                            "iterations": int(sum(r["iterations"] for r in res)), "pool_bytes": int(pool)}
    if 0 < nb < n_req:
        out["concurrent_z2"]["first_%d" % nb] = {"p50_latency_s": float(np.percentile(lat[:nb], 50)),
                                                 "p99_latency_s": float(np.percentile(lat[:nb], 99))}
    print(json.dumps({"concurrent_z2": out["concurrent_z2"]}), file=sys.stderr, flush=True)
    if nb > 0:
        # baseline: one solve at a time in the plain FP64 form (complex
        # requests, which have no plain form, in their Z2 form), the same
        # arrivals: solve i starts when it has arrived and solve i-1 is done
        from paper_2410_11596_amd import CTMRG

        end = 0.0
        lat_b, iters, conv_n = [], 0, 0
        for i, ((D, chi, cplx, A), at) in enumerate(zip(reqs[:nb], arrive[:nb])):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            g = CTMRG(A, chi, form="z2" if cplx else "dense")
            it, conv = 0, False
            while it < max_iter and not conv:
                g.step(1)
                it += 1
                conv = g.converged(tol)[0]
                if it % 10 == 0:
                    print(f"baseline solve {i + 1}/{nb} (D={D}, chi={chi}): {it} iterations", file=sys.stderr,
                          flush=True)
            g.rdm1()
            g.rdm2("h")
            g.rdm2("v")
            g.close()
            torch.cuda.synchronize()
            dur = time.perf_counter() - s0
            end = max(at, end) + dur
            lat_b.append(end - at)
            iters += it
            conv_n += int(conv)
            print(f"baseline solve {i + 1}/{nb} done in {dur:.2f} s", file=sys.stderr, flush=True)
        lat_b = np.array(lat_b)
        out["one_at_a_time_dense"] = {"requests": nb, "max_active": 1,
                                      "p50_latency_s": float(np.percentile(lat_b, 50)),
                                      "p99_latency_s": float(np.percentile(lat_b, 99)),
                                      "solves_per_s": nb / end, "wall_s": end, "converged": conv_n,
                                      "iterations": iters,
                                      "queue": "one server: solve i starts at max(arrival i, end of solve i-1); "
                                               "solves run back to back, arrivals on the same clock"}
    return out


def _oracle_saturated_env(ctmrg, basis, run, D, chi, split, seed):
    """A seeded random environment with every bond at chi: split (even, odd)
    in the Z2 form (blocks of odd total parity zero), one sector in the plain
    form."""
    rng = np.random.default_rng(seed + 1)
    q = D * D
    if run.form == "z2":
        pq = run.par_q
        pb = np.array([0] * split[0] + [1] * split[1])
    else:
        pq = np.zeros(q, dtype=np.int64)
        pb = np.zeros(chi, dtype=np.int64)
    ts = []
    for shape, pars in [((chi, chi), [pb, pb]), ((chi, q, chi), [pb, pq, pb])] * 4:
        x = rng.standard_normal(shape)
        ts.append(np.where(basis.parity_mask(pars), x, 0.0))
    return ctmrg.Env(ts, [pb.copy() for _ in range(4)] if run.form == "z2" else None)


def small_configs(steps, warmup):
    """The small shapes of the parity tests, timed like the headline one: the
    Z2 and plain forms at D = 2, chi = 16 and D = 4, chi = 64 (i.i.d. seed 0,
    FP64), warmup untimed iterations, then steps timed.  At these sizes a
    step is bound by launches and host checks, not by the matrix cores."""
    from paper_2410_11596_amd import inputs

    out = []
    for D, chi in ((2, 16), (4, 64)):
        A = inputs.iid_tensor(2, D, 0)
        row = {"D": D, "chi": chi, "iterations_timed": [warmup + 1, warmup + steps]}
        for form in ("z2", "dense"):
            t, st, _, _ = time_form(A, chi, form, steps, warmup, profile=False)
            row[form] = {"value": steps / t, "unit": "CTMRG iterations/s", "ms_per_step": 1e3 * t / steps,
                         "iteration_ms": st["iteration_ms"]}
        row["z2_over_dense"] = row["z2"]["value"] / row["dense"]["value"]
        out.append(row)
    return out


def cpu_baseline(D, chi, split, seed=0, z2_repeats=3):
    """The oracle as it stands, on the host cores: one left move of its plain
    (dense) form -- the authority -- on a seeded random environment with every
    bond at chi, timed once (about 15-25 s on 16 cores), scaled x4 to one
    iteration; beside it the median of z2_repeats left moves of its Z2 form on
    the same kind of environment split (even, odd)."""
    from oracle import basis, ctmrg

    from paper_2410_11596_amd import inputs

    A = inputs.iid_tensor(2, D, seed)
    threads = len(os.sched_getaffinity(0))
    rd = ctmrg.Run(chi, "dense", A=A)
    env = _oracle_saturated_env(ctmrg, basis, rd, D, chi, split, seed)
    t0 = time.perf_counter()
    ctmrg.left_move(env, rd.a, chi, rd.tau, None)
    t_dense = time.perf_counter() - t0
    rz = ctmrg.Run(chi, "z2", A=A)
    tz = []
    for r in range(z2_repeats):
        env = _oracle_saturated_env(ctmrg, basis, rz, D, chi, split, seed + r)
        t0 = time.perf_counter()
        ctmrg.left_move(env, rz.a, chi, rz.tau, rz.par_q)
        tz.append(time.perf_counter() - t0)
    t_z2 = float(np.median(tz))
    small = small_config_oracle_times()
    return {
        "value": 1.0 / (4.0 * t_dense),
        "unit": "CTMRG iterations/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one left move of the oracle's plain (dense) form (numpy + the host BLAS/LAPACK, FP64, "
                  f"{threads} threads) on a seeded random D={D}, chi={chi} environment with every bond at chi, "
                  f"{t_dense:.1f} s, scaled x4 to one iteration",
        "z2_form": {"value": 1.0 / (4.0 * t_z2), "unit": "CTMRG iterations/s",
                    "sample": f"median of {z2_repeats} left moves of the oracle's Z2 form on such environments "
                              f"split {split[0]}+{split[1]}: {', '.join(f'{t:.2f}' for t in tz)} s"},
        "small_configs": small,
    }


def small_config_oracle_times(warm=3):
    """Seconds per iteration of the oracle's solve (i.i.d. seed 0) at
    D = 2, chi = 16 and D = 4, chi = 64, both forms, after warm iterations
    (the bonds at chi): the next iteration with every host thread, the one
    after it with the BLAS/LAPACK pools held to one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import ctmrg

    from paper_2410_11596_amd import inputs

    out = []
    for D, chi in ((2, 16), (4, 64)):
        A = inputs.iid_tensor(2, D, 0)
        for form in ("dense", "z2"):
            r = ctmrg.Run(chi, form, A=A)
            r.step(warm)
            t0 = time.perf_counter()
            r.step(1)
            t_all = time.perf_counter() - t0
            with threadpool_limits(1):
                t0 = time.perf_counter()
                r.step(1)
                t_one = time.perf_counter() - t0
            out.append({"D": D, "chi": chi, "form": form, "s_per_iteration": t_all,
                        "s_per_iteration_one_thread": t_one, "threads": len(os.sched_getaffinity(0))})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed iterations (the window is warmup+1 .. warmup+steps)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed iterations before the window")
    ap.add_argument("--dense-steps", type=int, default=None,
                    help="timed iterations of the plain form (default: --steps, the same window as the Z2 form)")
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-block-product run")
    ap.add_argument("--no-late", action="store_true", help="skip the later-iterations timing of the same solve")
    ap.add_argument("--no-c4v", action="store_true", help="skip the C4v-scheme comparison")
    ap.add_argument("--no-small", action="store_true", help="skip the D = 2 and D = 4 timings")
    ap.add_argument("--no-complex", action="store_true", help="skip the complex-tensor timing")
    ap.add_argument("--no-large", action="store_true", help="skip the D = 8, chi = 256 run")
    ap.add_argument("--no-hotrg", action="store_true", help="skip the HOTRG Z2/plain comparison")
    ap.add_argument("--hotrg-by-d", action="store_true", help="run only the HOTRG comparison over D at chi 64")
    ap.add_argument("--hotrg-only", type=int, default=0, metavar="CHI",
                    help="run only the HOTRG comparison at this chi and print its JSON")
    ap.add_argument("--serve", type=int, default=24, metavar="N",
                    help="solves in the serving run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="Poisson arrival rate of the serving run (1/s)")
    ap.add_argument("--serve-baseline", type=int, default=None, metavar="N",
                    help="requests of the one-at-a-time plain-form baseline (default: all of the serving run)")
    ap.add_argument("--serve-max-iter", type=int, default=60, help="iteration cap of a served solve")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving comparison and print its JSON")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip measuring the chip's own MFMA rate and copy bandwidth")
    ap.add_argument("--copy-check", type=int, default=0, metavar="BYTES",
                    help="before timing, copy BYTES three times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.dense_steps is None:
        args.dense_steps = args.steps
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver is built for a single GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.serve_only:
        print(json.dumps(serving(args.serve, args.serve_rate, max_iter=args.serve_max_iter,
                                 baseline_n=args.serve_baseline)), flush=True)
        return
    if args.hotrg_only:
        print(json.dumps(hotrg_speedup(chis=(args.hotrg_only,), probe_chi=min(args.hotrg_only, 32))))
        return
    if args.hotrg_by_d:
        print(json.dumps(hotrg_by_d()))
        return

    import torch

    from paper_2410_11596_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.copy_check > 0:
        copy_check(args.copy_check)
    A = inputs.iid_tensor(2, args.D, 0)
    # value: the timed iterations without instrumentation; roofline: the
    # same iterations again (the run is deterministic) with a HIP event pair
    # around every GEMM launch
    tz, zstats, phases, split = time_form(A, args.chi, "z2", args.steps, args.warmup, profile=False)
    tz_prof, stats, _, _ = time_form(A, args.chi, "z2", args.steps, args.warmup, profile=True)
    z2_rate = args.steps / tz
    out = {
        "metric": METRIC,
        "value": z2_rate,
        "unit": "CTMRG iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * tz / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"Z2 directional CTMRG, 1x1 cell, real iPEPS d=2 D={args.D}, chi={args.chi}, "
                        f"i.i.d. N(0,1) tensor seed 0, FP64",
            "form": "z2",
            "D": args.D,
            "chi": args.chi,
            "precision": "fp64",
        },
        "sector_split": list(split),
        "phases_ms_per_step": {k: 1e3 * v / args.steps for k, v in zip(PHASES, phases.tolist())},
        "phases_sum_ms_per_step": 1e3 * float(np.sum(phases)) / args.steps,
        "svd_health_in_window": {k: zstats[k] for k in ("truncations_in_window", "svd_unconverged_in_window",
                                                        "multiplet_splits_in_window")},
        "svd_in_window": zstats["svd_in_window"],
        "iteration_ms": zstats["iteration_ms"],
    }
    if stats["launches"] > 0 and stats["seconds"] > 0:
        # mean algorithmic flops per launch over the mean launch duration of
        # the GEMM kernel (a HIP event right before and right after each of
        # its launches, on the library's stream); an event pair costs a fixed
        # few microseconds even around no work, which is measured on the same
        # stream and taken off every launch.  The split-K reductions that
        # follow some launches are timed apart and reported beside.
        ev = event_pair_overhead()
        kernel_s = stats["seconds"] - stats["launches"] * ev
        red_s = stats["reduce_seconds"] - stats["reduce_launches"] * ev
        achieved = stats["flops"] / kernel_s / 1e12
        out["roofline"] = {
            "bound": "mfma",
            "kernel": "gemm_f64_kernel",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": gemm_traffic(),
            "launches": stats["launches"],
            "flops_per_launch": stats["flops"] / stats["launches"],
            "avg_launch_us": 1e6 * kernel_s / stats["launches"],
            "event_pair_overhead_us": 1e6 * ev,
            "achieved_uncorrected": stats["flops"] / stats["seconds"] / 1e12,
            "with_splitk_reduce": {"achieved": stats["flops"] / (kernel_s + red_s) / 1e12,
                                   "frac": stats["flops"] / (kernel_s + red_s) / 1e12 / FP64_PEAK_TFLOPS,
                                   "reduce_launches": stats["reduce_launches"],
                                   "avg_reduce_us": 1e6 * red_s / max(1, stats["reduce_launches"])},
            "gemm_share_of_step": kernel_s / tz_prof,
            "profiled_pass_ms_per_step": 1e3 * tz_prof / args.steps,
        }
        if not args.no_peaks:
            mp = measured_peaks()
            out["roofline"]["measured_peaks"] = mp
            out["roofline"]["frac_of_measured_mfma"] = achieved / mp["fp64_mfma_tflops"]
    if not args.no_late:
        out["late_iterations"] = late_iterations(A, args.chi, args.warmup + args.steps, args.steps)
    if not args.no_dense:
        # the plain form over the same window: the same warm-up, the same
        # number of timed iterations (unless --dense-steps says otherwise)
        td, dstats, dphases, _ = time_form(A, args.chi, "dense", args.dense_steps, args.warmup, profile=False)
        dense_rate = args.dense_steps / td
        dph = {k: 1e3 * v / args.dense_steps for k, v in zip(PHASES, dphases.tolist())}
        out["dense"] = {
            "iterations_timed": [args.warmup + 1, args.warmup + args.dense_steps],
            "z2_iterations_timed": [args.warmup + 1, args.warmup + args.steps],
            "value": dense_rate,
            "ms_per_step": 1e3 * td / args.dense_steps,
            "phases_ms_per_step": dph,
            "svd_health_in_window": {k: dstats[k] for k in ("truncations_in_window", "svd_unconverged_in_window",
                                                            "multiplet_splits_in_window")},
            "svd_in_window": dstats["svd_in_window"],
            "iteration_ms": dstats["iteration_ms"],
            "phases_sum_ms_per_step": sum(dph.values()),
            "z2_over_dense": z2_rate / dense_rate,
            "matched_window": args.dense_steps == args.steps,
            "phase_ratio_dense_over_z2": {k: (dph[k] / out["phases_ms_per_step"][k])
                                          if out["phases_ms_per_step"][k] > 0 else None for k in PHASES},
        }
        out["z2_over_dense"] = out["dense"]["z2_over_dense"]
    if not args.no_mixed and args.D == 6 and args.chi == 144:
        gold = _golden("seed0")
        out["mixed"] = mixed_precision(A, args.chi, args.steps, args.warmup, gold)
        out["mixed_bf16x3"] = mixed_precision(A, args.chi, args.steps, args.warmup, gold, precision="bf16x3")
        out["mixed_perturbed"] = mixed_precision(inputs.perturbed_product(2, 6, 20), args.chi, args.steps,
                                                 args.warmup, _golden("perturbed"))
    if not args.no_large:
        out["large_d8_chi256"] = large_shape()
    if not args.no_small:
        out["small_configs"] = small_configs(args.steps, args.warmup)
    if not args.no_c4v:
        out["c4v"] = c4v_scheme(args.D, args.chi, args.steps, args.warmup)
    if not args.no_complex:
        out["complex"] = complex_case()
    if not args.no_hotrg:
        out["hotrg"] = hotrg_speedup()
        out["hotrg"]["by_D"] = hotrg_by_d()
    if args.serve > 0:
        out["serving"] = serving(args.serve, args.serve_rate, max_iter=args.serve_max_iter,
                                 baseline_n=args.serve_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.D, args.chi, (84, 60))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
