"""GPU parity of the C4v-symmetric scheme (Sec. II A, one corner and one
edge): the HIP path with c4v=True against the C4v oracle (oracle/c4v.py) on
seeded tensors symmetrised over the eight symmetries of the square, in the Z2
and plain forms; and its fixed point against the directional scheme's on the
GPU and against Onsager's free energy for the Ising PEPS.  Only
gauge-invariant outputs are compared (RDMs, energy, the plain-basis
environment of a site, ln kappa, the kept spectrum and sector sizes of every
iteration); tolerance 1e-10 on RDM entries."""
import numpy as np
import pytest

from oracle import c4v, ctmrg
from paper_2410_11596_amd import inputs
from test_gpu_ctmrg import _compare
from test_oracle_pins import onsager_log_z

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


def c4v_tensor(D, seed):
    return inputs.c4v_iid_tensor(2, D, seed)


def _gpu(A, chi, form, iters, **kw):
    from paper_2410_11596_amd import CTMRG

    c = CTMRG(A, chi, form=form, c4v=True, **kw)
    c.step(iters)
    return c


@pytest.mark.parametrize("form", ["z2", "dense"])
@pytest.mark.parametrize("iters", [1, 30])
def test_d2_chi16(form, iters):
    A = c4v_tensor(2, 0)
    o = c4v.C4vRun(16, form, A=A).step(iters)
    g = _gpu(A, 16, form, iters)
    _compare(g, o)
    assert len(g.records()) == iters  # one truncation per iteration
    if form == "z2":
        assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]


def test_d3_chi30_ragged_sectors():
    """D=3 (6+3): sectors of unequal size, chi not a multiple of either."""
    A = c4v_tensor(3, 2)
    o = c4v.C4vRun(30, "z2", A=A).step(12)
    g = _gpu(A, 30, "z2", 12)
    _compare(g, o)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]


def test_d4_chi64_subspace_iteration():
    """D=4 (10+6), chi=64: enlarged corner of 1024 rows, decomposed by the
    subspace iteration."""
    A = c4v_tensor(4, 3)
    o = c4v.C4vRun(64, "z2", A=A).step(6)
    g = _gpu(A, 64, "z2", 6)
    _compare(g, o)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
    assert any(max(r["iters"]) > 0 for r in g.records())


def test_d6_chi144_two_iterations():
    """D=6 (21+15), chi=144: the enlarged corner reaches 5184 rows."""
    A = c4v_tensor(6, 0)
    o = c4v.C4vRun(144, "z2", A=A).step(2)
    g = _gpu(A, 144, "z2", 2)
    assert [tuple(r["kept"]) for r in g.records()] == [tuple(r["kept"]) for r in o.records]
    for rg, ro in zip(g.records(), o.records):
        assert np.allclose(rg["spectrum"], ro["spectrum"][: len(rg["spectrum"])], rtol=1e-6, atol=1e-13)
    info = [(r["iters"], r["sweeps"]) for r in g.records()]
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL, info
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < TOL, info
    assert np.abs(g.rdm2("v") - g.rdm2("h")).max() < TOL  # the symmetry of the square


def test_fixed_point_is_the_directional_one():
    from paper_2410_11596_amd import CTMRG

    A = c4v_tensor(2, 1)
    g = _gpu(A, 16, "z2", 0)
    g.run(300, tol=1e-12)
    d = CTMRG(A, 16, form="z2")
    d.run(200, tol=1e-12)
    assert g.converged(1e-12)[0] and d.converged(1e-12)[0]
    assert np.abs(g.rdm1() - d.rdm1()).max() < 1e-11
    assert np.abs(g.rdm2("h") - d.rdm2("h")).max() < 1e-11
    assert np.abs(g.rdm2("v") - d.rdm2("v")).max() < 1e-11
    assert abs(g.log_kappa() - d.log_kappa()) < 1e-11


def test_ising_peps_onsager():
    beta = 0.40
    A = inputs.ising_peps(beta)
    g = _gpu(A, 16, "z2", 0)
    g.run(400, tol=1e-13)
    assert abs(g.log_kappa() - onsager_log_z(beta)) < 1e-10
    o = c4v.C4vRun(16, "z2", A=A).run(400, tol=1e-13)
    assert abs(g.log_kappa() - o.log_kappa()) < 1e-11
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL


def test_mixed_precision_refines_to_the_fp64_fixed_point():
    A = c4v_tensor(3, 6)
    ref = _gpu(A, 24, "z2", 0)
    ref.run(300, tol=1e-12)
    g = _gpu(A, 24, "z2", 0, precision="bf16x3")
    g.step(40)
    g.set_precision("fp64")
    g.run(300, tol=1e-12)
    assert np.abs(g.rdm1() - ref.rdm1()).max() < 1e-10
    assert np.abs(g.rdm2("h") - ref.rdm2("h")).max() < 1e-10


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_degenerate_sizes(form):
    """chi = 1, D = 1 and a product state: exact RDMs and the oracle."""
    A = c4v_tensor(2, 5)
    o = c4v.C4vRun(1, form, A=A).step(5)
    g = _gpu(A, 1, form, 5)
    _compare(g, o)
    A1 = inputs.iid_tensor(3, 1, 2)
    g = _gpu(A1, 4, form, 3)
    r1 = g.rdm1()
    v = A1.reshape(3)
    assert np.allclose(r1, np.outer(v, v) / (v @ v), atol=1e-14)
    P = inputs.product_state(np.array([0.6, -0.8]), 2)
    g = _gpu(P, 4, form, 3)
    w = np.array([0.6, -0.8])
    assert np.allclose(g.rdm1(), np.outer(w, w), atol=1e-14)
    assert all(sum(r["kept"]) == 1 for r in g.records())
