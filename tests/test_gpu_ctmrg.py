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
    """D=2, chi=16, 50 iterations: the Z2 and plain forms side by side."""
    A = inputs.iid_tensor(2, 2, 0)
    o = ctmrg.Run(16, form, A=A).step(50)
    g = _gpu_run(A, 16, form, 50)
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


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_config2_d4_chi64(form):
    """D=4 (10+6), chi=64: subspace-iteration SVD path against the oracle."""
    A = inputs.iid_tensor(2, 4, 0)
    o = ctmrg.Run(64, form, A=A).step(8)
    g = _gpu_run(A, 64, form, 8)
    _compare(g, o)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]


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
