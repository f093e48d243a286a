"""GPU parity: the HIP CTMRG (Z2 and plain forms) against the CPU oracle.

Both sides start from the same seeded tensor and run the same number of
iterations; only gauge-invariant outputs are compared (RDMs, energy, the
one-site environment in the plain basis, the kept spectrum of every move,
ln kappa, sector sizes).  Tolerance: 1e-10 on RDM entries and energies.
"""
import numpy as np
import pytest

from oracle import basis, ctmrg
from paper_2410_11596_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


def _gpu_run(A, chi, form, iters, **kw):
    from paper_2410_11596_amd import CTMRG

    c = CTMRG(A, chi, form=form, **kw)
    c.step(iters)
    return c


def _gpu_launch(A, chi, form, **kw):
    from paper_2410_11596_amd import CTMRG

    return CTMRG(A, chi, form=form, **kw)


# delta and the corner spectra are distances and entries of sum-normalised
# spectra of corners renormalised with projectors that divide by singular
# values down to 1e-12 of the largest: FP64 rounding is amplified to about
# 1e-10 there.  The oracle itself moves by that much when only its LAPACK
# SVD driver changes (gesdd -> gesvd at D = 2, chi = 16: delta by 2.5e-10,
# corner spectra by 6e-11), so parity is asked to 1e-9.
DELTA_TOL = 1e-9
SPEC_TOL = 1e-9


def _compare_corner_spectra(g, o, atol=SPEC_TOL):
    """The four current corner spectra (sum-normalised, zero padded) against
    the oracle's on their common length; the rest is zero on both sides."""
    for c in range(4):
        sg = g.corner_spectrum(c)
        so = o._spec[c]
        n = min(len(sg), len(so))
        assert np.abs(sg[:n] - so[:n]).max() < atol, c
        assert not np.any(sg[n:]) and not np.any(so[n:])


def _compare(g, o, spectra_rtol=1e-6, tol=TOL):
    assert np.abs(g.rdm1() - o.rho1()).max() < tol
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < tol
    assert np.abs(g.rdm2("v") - o.rho2("v")).max() < tol
    h = ctmrg.heisenberg_bond()
    assert abs(g.energy(h) - o.energy(h)) < tol * max(1.0, abs(o.energy(h)))
    eo = o.epsilon()
    assert np.abs(g.epsilon() - eo).max() < 1e3 * tol * np.abs(eo).max()
    recs = g.records()
    assert len(recs) == len(o.records)
    for rg, ro in zip(recs, o.records):
        k = sum(rg["kept"])
        assert k == sum(ro["kept"])
        assert np.allclose(rg["spectrum"][:k], ro["spectrum"][:k], rtol=spectra_rtol, atol=1e-13)


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_first_moves_d2(form):
    A = inputs.iid_tensor(2, 2, 1)
    o = ctmrg.Run(16, form, A=A).step(1)
    g = _gpu_run(A, 16, form, 1)
    _compare(g, o)


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_config1_d2_chi16_50_iterations(form):
    """D=2, chi=16, 50 iterations: the Z2 and plain forms side by side; delta
    after every iteration against the oracle's."""
    A = inputs.iid_tensor(2, 2, 0)
    o = ctmrg.Run(16, form, A=A)
    g = _gpu_launch(A, 16, form)
    _compare_corner_spectra(g, o)  # the initial environment
    for it in range(50):
        o.step(1)
        g.step(1)
        assert abs(g.converged(0.0)[1] - o.deltas[-1]) < DELTA_TOL, it
    _compare_corner_spectra(g, o)
    _compare(g, o)
    if form == "z2":
        assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
        assert g.s_err() <= 1e-15
        r1, r2 = g.rdm1(), g.rdm2("h")
        assert np.array_equal(r1, r1.T) and np.array_equal(r2, r2.T)
    assert abs(g.log_kappa() - o.log_kappa()) < 1e-10


def test_dense_and_z2_gpu_forms_agree_d3():
    # chi = 16 keeps the cut well above the 1e-12 cutoff for this tensor
    A = inputs.iid_tensor(2, 3, 4)
    gz = _gpu_run(A, 16, "z2", 6)
    gd = _gpu_run(A, 16, "dense", 6)
    assert np.abs(gz.rdm2("h") - gd.rdm2("h")).max() < TOL
    assert np.abs(gz.rdm1() - gd.rdm1()).max() < TOL


def test_product_state():
    v = np.array([0.6, -0.8])
    A = inputs.product_state(v, 3)
    g = _gpu_run(A, 8, "z2", 3)
    assert all(tuple(r["kept"]) == (1, 0) for r in g.records())
    r1 = g.rdm1()
    assert np.allclose(r1, np.outer(v, v) / (v @ v), atol=1e-14)
    assert np.allclose(g.rdm2("h"), np.kron(r1, r1), atol=1e-14)


def test_ising_peps_up_boundary():
    beta = 0.45
    A = inputs.ising_peps(beta)
    b = inputs.ising_up_boundary(beta)
    o = ctmrg.Run(16, "z2", A=A, boundary=b).step(40)
    g = _gpu_run(A, 16, "z2", 40, boundary=b)
    assert all(r["kept"][1] == 0 for r in g.records())
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL
    assert abs(g.log_kappa() - o.log_kappa()) < 1e-10


@pytest.mark.parametrize("form_m", [False, True])
@pytest.mark.parametrize("form", ["z2", "dense"])
def test_config2_d4_chi64(form, form_m):
    """D=4 (10+6), chi=64: subspace-iteration SVD path against the oracle,
    with the decomposed matrix applied through the enlarged corners (default)
    or always formed (form_m); the convergence measure delta after every
    iteration and the final corner spectra against the oracle's."""
    A = inputs.iid_tensor(2, 4, 0)
    o = ctmrg.Run(64, form, A=A)
    g = _gpu_launch(A, 64, form, form_m=form_m)
    for it in range(8):
        o.step(1)
        g.step(1)
        assert abs(g.converged(0.0)[1] - o.deltas[-1]) < DELTA_TOL, it
    _compare(g, o)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
    _compare_corner_spectra(g, o)
    if form_m:
        assert not any(r["implicit"] for r in g.records())
    assert g.svd_health()[0] == 0


def test_metric_shape_d6_chi144_one_iteration():
    """D=6 (21+15), chi=144, the benchmark shape: one iteration (4 moves)."""
    A = inputs.iid_tensor(2, 6, 0)
    o = ctmrg.Run(144, "z2", A=A).step(1)
    g = _gpu_run(A, 144, "z2", 1)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
    for rg, ro in zip(g.records(), o.records):
        assert np.allclose(rg["spectrum"], ro["spectrum"][: len(rg["spectrum"])], rtol=1e-6, atol=1e-13)
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < TOL


def test_corner_applied_matrix_matches_formed_matrix_d6():
    """D=6, chi=144: once the subspace iteration is short, M is applied
    through the enlarged corners instead of being formed; both ways give the
    same environment (RDMs to 1e-10, identical kept sector sizes)."""
    A = inputs.iid_tensor(2, 6, 0)
    ga = _gpu_run(A, 144, "z2", 12)
    gf = _gpu_run(A, 144, "z2", 12, form_m=True)
    ra, rf = ga.records(), gf.records()
    assert any(r["implicit"] for r in ra) and not any(r["implicit"] for r in rf)
    assert [tuple(r["kept"]) for r in ra] == [tuple(r["kept"]) for r in rf]
    assert np.abs(ga.rdm1() - gf.rdm1()).max() < TOL
    assert np.abs(ga.rdm2("h") - gf.rdm2("h")).max() < TOL
    assert np.abs(ga.rdm2("v") - gf.rdm2("v")).max() < TOL
    assert ga.s_err() <= 1e-15


@pytest.mark.parametrize("D,chi", [(1, 1), (1, 4), (2, 1), (3, 2)])
@pytest.mark.parametrize("form", ["z2", "dense"])
def test_degenerate_sizes(D, chi, form):
    """Bond dimension one (a product state: no odd sector at all), and
    truncation to one or two states (the kept count below the sector sizes)."""
    A = inputs.iid_tensor(2, D, 3)
    o = ctmrg.Run(chi, form, A=A).step(3)
    g = _gpu_run(A, chi, form, 3)
    _compare(g, o)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
    if D == 1:
        a = A.reshape(2)
        assert np.abs(g.rdm1() - np.outer(a, a) / (a @ a)).max() < 1e-14


def test_largest_shape_d8_chi256_forms_agree():
    """D = 8 (36 + 28), chi = 256, the largest configuration: two iterations
    of the Z2 and plain forms agree (kept spectra, sector sizes, RDMs), and
    the Z2 RDMs are Hermitian bit for bit with S_err = 0.  Too large for the
    oracle; the two forms share the code but not the block structure."""
    A = inputs.iid_tensor(2, 8, 0)
    gz = _gpu_run(A, 256, "z2", 2)
    gd = _gpu_run(A, 256, "dense", 2)
    rz, rd = gz.records(), gd.records()
    assert len(rz) == len(rd) == 8
    for a, b in zip(rz, rd):
        k = sum(a["kept"])
        assert k == sum(b["kept"])
        assert np.allclose(a["spectrum"][:k], b["spectrum"][:k], rtol=1e-8, atol=1e-13)
    for dr in ("h", "v"):
        assert np.abs(gz.rdm2(dr) - gd.rdm2(dr)).max() < TOL
        r2 = gz.rdm2(dr)
        assert np.array_equal(r2, r2.T) and abs(np.trace(r2) - 1.0) < 1e-12
    assert np.abs(gz.rdm1() - gd.rdm1()).max() < TOL
    assert gz.s_err() == 0.0
    gz.close()
    gd.close()


def test_runs_are_bitwise_reproducible_with_and_without_instrumentation():
    """Two solves of the benchmark shape from the same tensor, one with a HIP
    event pair around every GEMM launch: the same records and bit-identical
    RDMs after the same iterations (fixed reduction orders, no atomics in the
    results), so a timing pass and a profiled pass do the same work."""
    from paper_2410_11596_amd import CTMRG

    A = inputs.iid_tensor(2, 6, 0)
    a = CTMRG(A, 144, form="z2")
    a.step(3)
    b = CTMRG(A, 144, form="z2", profile=True)
    b.step(3)
    assert np.array_equal(a.rdm1(), b.rdm1())
    assert np.array_equal(a.rdm2("h"), b.rdm2("h"))
    ra, rb = a.records(), b.records()
    assert [r["kept"] for r in ra] == [r["kept"] for r in rb]
    assert [r["iters"] for r in ra] == [r["iters"] for r in rb]
    assert all(np.array_equal(x["spectrum"], y["spectrum"]) for x, y in zip(ra, rb))
    assert b.gemm_stats()["launches"] > 0


def test_subspace_iteration_cap_is_reported():
    """With one subspace iteration allowed, the truncations that take the
    subspace path cannot pass their residual test: each is flagged in its
    record and counted by ctm_svd_health, and the solve itself still runs."""
    A = inputs.iid_tensor(2, 4, 0)
    g = _gpu_launch(A, 64, "z2", svd_iters=1)
    g.step(2)
    recs = g.records()
    sub = [r for r in recs if r["iters"][0] > 0 or r["iters"][1] > 0]
    assert sub, "no truncation took the subspace path"
    assert all(any(r["unconverged"]) for r in sub)
    assert all(not any(r["unconverged"]) for r in recs if r["iters"] == (0, 0))
    assert g.svd_health()[0] == sum(1 for r in recs if any(r["unconverged"]))
    r1 = g.rdm1()
    assert np.isfinite(r1).all() and abs(np.trace(r1) - 1.0) < 1e-12
    # the default cap converges on the same input
    h = _gpu_launch(A, 64, "z2")
    h.step(2)
    assert h.svd_health()[0] == 0


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_retry_that_needs_the_formed_matrix(form):
    """D = 2, chi = 100 (a request of the serving stream, seed 1033): while
    the bonds grow, a kept count passes the trusted part of a subspace that
    was applied through the corners, and the retry with the larger block
    reaches the sector size, so that block is decomposed directly on M formed
    from the enlarged corners.  The solve completes and matches the oracle.

    This input keeps singular values down to the 1e-12 cutoff from the first
    iteration on and is ill-conditioned at that level: a 1e-15 relative
    perturbation of the tensor moves the oracle's own delta by up to 2e-8,
    its corner spectra by up to 6e-8 and its rho1 by up to 2.8e-10 (measured
    over three iterations).  So delta is compared to 1e-6 and the RDMs to
    1e-9; the kept sector sizes exactly."""
    iters = 6
    A = inputs.iid_tensor(2, 2, 1033)
    o = ctmrg.Run(100, form, A=A).step(iters)
    g = _gpu_launch(A, 100, form)
    for it in range(iters):
        g.step(1)
        assert abs(g.converged(0.0)[1] - o.deltas[it]) < 1e-6, it
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
    assert np.abs(g.rdm1() - o.rho1()).max() < 1e-9
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < 1e-9
    assert np.abs(g.rdm2("v") - o.rho2("v")).max() < 1e-9
    if form == "dense":  # the Z2 sectors of this input are small enough to be decomposed directly
        assert any(max(r["iters"]) > 0 for r in g.records())  # the subspace path ran


def test_product_state_has_zero_delta():
    """A product state's corners have rank one from the start: delta is zero
    after the first iteration, the corner spectra are (1, 0, ...)."""
    v = np.array([0.6, -0.8])
    A = inputs.product_state(v, 3)
    g = _gpu_launch(A, 8, "z2")
    g.step(1)
    conv, dl = g.converged(1e-14)
    assert conv and dl < 1e-14
    for c in range(4):
        s = g.corner_spectrum(c)
        assert abs(s[0] - 1.0) < 1e-14 and np.abs(s[1:]).max() < 1e-14


def _golden_d6(name="seed0"):
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", f"ctmrg_d6_chi144_{name}.json")
    with open(path) as f:
        return json.load(f)


def _compare_golden_observables(g, ob):
    assert np.abs(g.rdm1() - np.array(ob["rho1"])).max() < TOL
    assert np.abs(g.rdm2("h") - np.array(ob["rho2_h"])).max() < TOL
    assert np.abs(g.rdm2("v") - np.array(ob["rho2_v"])).max() < TOL
    e = g.energy(ctmrg.heisenberg_bond())
    assert abs(e - ob["energy"]) < TOL * max(1.0, abs(ob["energy"]))
    assert abs(g.log_kappa() - ob["log_kappa"]) < TOL
    eps = g.epsilon().reshape(-1)
    got = eps[np.array(ob["eps_index"])]
    assert np.abs(got - np.array(ob["eps_value"])).max() < 1e-7 * ob["eps_max_abs"]


@pytest.mark.parametrize("form_m", [False, True])
def test_benchmark_regime_d6_chi144_against_oracle(form_m):
    """The benchmark shape (D = 6, chi = 144, seed 0) through the iterations
    the benchmark times: warm starts, small oversampling once the cuts
    converge, the matrix applied through the corners (default) or always
    formed (form_m), both Jacobi phases and the redo with a larger subspace.
    Every record's kept sector sizes exactly and kept spectrum, delta after
    every iteration, the final corner spectra, RDMs and energy (1e-10), ln
    kappa and sampled entries of the one-site environment against the
    oracle's values stored by tests/golden/make_ctmrg_d6_chi144.py."""
    gold = _golden_d6("seed0")
    A = inputs.iid_tensor(2, 6, 0)
    g = _gpu_launch(A, gold["chi"], "z2", form_m=form_m)
    for it in range(gold["iterations"]):
        g.step(1)
        assert abs(g.converged(0.0)[1] - gold["deltas"][it]) < DELTA_TOL, it
    recs = g.records()
    assert len(recs) == len(gold["records"])
    for m, (rg, ro) in enumerate(zip(recs, gold["records"])):
        assert list(rg["kept"]) == ro["kept"], m
        # values near the 1e-12 cutoff carry absolute errors of about 1e-13
        assert np.allclose(rg["spectrum"], ro["spectrum"], rtol=1e-8, atol=1e-12), m
        assert not rg["multiplet_split"]
    # the regimes the benchmark's iterations run in were all exercised
    if form_m:
        assert not any(r["implicit"] for r in recs)
    else:
        assert any(r["implicit"] for r in recs[8:]) and any(not r["implicit"] for r in recs)
    assert any(0 < max(r["iters"]) <= 3 for r in recs)
    # truncations whose subspace iteration stopped at the cap (the early,
    # unconverged cuts) are reported, and are among the ones compared above
    print("records (iterations even/odd, unconverged):",
          [(r["iters"], r["unconverged"]) for r in recs], flush=True)
    assert g.svd_health()[0] == sum(1 for r in recs if any(r["unconverged"]))
    assert all(max(r["iters"]) == 12 for r in recs if any(r["unconverged"]))
    for c in range(4):
        sg = g.corner_spectrum(c)
        so = np.array(gold["corner_spectra"][c])
        n = min(len(sg), len(so))
        assert np.abs(sg[:n] - so[:n]).max() < SPEC_TOL
    _compare_golden_observables(g, gold["observables"][str(gold["iterations"])])
    assert g.s_err() <= 1e-15
    g.close()


def test_perturbed_product_state_d6_chi144_against_oracle():
    """The perturbed product state of the mixed-precision workload (e_0 plus
    1e-2 noise, D = 6, chi = 144): strongly uneven sectors and a fast-decaying
    spectrum; records, delta and the observables against the oracle."""
    gold = _golden_d6("perturbed")
    A = inputs.perturbed_product(2, 6, 20)
    g = _gpu_launch(A, gold["chi"], "z2")
    for it in range(gold["iterations"]):
        g.step(1)
        assert abs(g.converged(0.0)[1] - gold["deltas"][it]) < DELTA_TOL, it
    recs = g.records()
    for m, (rg, ro) in enumerate(zip(recs, gold["records"])):
        assert list(rg["kept"]) == ro["kept"], m
        assert np.allclose(rg["spectrum"], ro["spectrum"], rtol=1e-8, atol=1e-12), m
    print("kept (even, odd):", [r["kept"] for r in recs[-4:]], flush=True)
    _compare_golden_observables(g, gold["observables"][str(gold["iterations"])])
    g.close()
