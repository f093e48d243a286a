"""GPU parity for complex tensors (Sec. II C) against the oracle.

The GPU holds every structured complex tensor as its real even-total blocks
and the imaginary parts of its odd-total blocks; the oracle's real
representation (oracle/complex_z2.py, the q leg and f of the paper) and its
plain complex128 form (oracle/ctmrg.py on complex tensors) are the
references.  Compared: kept sizes and spectra of every truncation, delta
after every iteration, the Hermitian one- and two-site RDMs and the energy
(1e-10), exact Hermiticity of the GPU RDMs, a real tensor given as complex
against the real GPU path, a global phase, a complex product state, and the
calls that a complex context refuses."""
import numpy as np
import pytest

from oracle import complex_z2, ctmrg
from paper_2410_11596_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10
DELTA_TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


def _gpu(A, chi, **kw):
    from paper_2410_11596_amd import CTMRG

    return CTMRG(A, chi, **kw)


@pytest.mark.parametrize("D,chi,iters", [(2, 12, 4), (2, 9, 6), (3, 20, 2), (4, 30, 2)])
def test_complex_tensor_against_the_oracle(D, chi, iters):
    A = inputs.complex_iid_tensor(2, D, 10 + D)
    print(f"complex D={D} chi={chi} iterations={iters}", flush=True)
    z = complex_z2.Run(chi, A)
    g = _gpu(A, chi)
    for it in range(iters):
        z.step(1)
        g.step(1)
        assert abs(g.converged(0.0)[1] - z.deltas[-1]) < DELTA_TOL, it
    recs = g.records()
    assert len(recs) == len(z.records)
    for rg, ro in zip(recs, z.records):
        assert tuple(rg["kept"]) == tuple(ro["kept"])
        k = rg["kept"][0]
        assert np.allclose(rg["spectrum"][:k], ro["spectrum"][:k], rtol=1e-8, atol=1e-12)
    r1 = g.rdm1()
    assert np.array_equal(r1, r1.conj().T)  # Hermitian by construction
    assert np.abs(r1 - z.rho1()).max() < TOL
    for f in ("h", "v"):
        r2 = g.rdm2(f)
        assert np.array_equal(r2, r2.conj().T)
        assert np.abs(r2 - z.rho2(f)).max() < TOL
    h = ctmrg.heisenberg_bond()
    assert abs(g.energy(h) - z.energy(h)) < TOL
    # the plain complex form reaches the same state within its own
    # (truncation-broken) Hermiticity
    p = ctmrg.Run(chi, "dense", A=A).step(iters)
    assert np.abs(r1 - p.rho1()).max() < 1e-8
    g.close()


def test_real_tensor_as_complex_equals_the_real_path():
    A = inputs.iid_tensor(2, 3, 4)
    gc = _gpu(A.astype(np.complex128), 16).step(4)
    gr = _gpu(A, 16).step(4)
    assert [r["kept"][0] for r in gc.records()] == [sum(r["kept"]) for r in gr.records()]
    assert np.abs(gc.rdm1() - gr.rdm1()).max() < TOL
    assert np.abs(gc.rdm2("h") - gr.rdm2("h")).max() < TOL
    assert np.abs(gc.rdm1().imag).max() == 0.0


def test_global_phase_and_product_state():
    A = inputs.complex_iid_tensor(2, 2, 4)
    ga = _gpu(A, 12).step(3)
    gb = _gpu(A * np.exp(0.7j), 12).step(3)
    assert np.abs(ga.rdm1() - gb.rdm1()).max() < 1e-12
    assert np.abs(ga.rdm2("v") - gb.rdm2("v")).max() < 1e-12
    v = np.array([0.6, 0.8j])
    P = np.zeros((2, 2, 2, 2, 2), dtype=np.complex128)
    P[:, 0, 0, 0, 0] = v
    gp = _gpu(P, 4).step(2)
    rho = gp.rdm1()
    assert np.abs(rho - np.outer(v, v.conj())).max() < 1e-14
    assert np.abs(gp.rdm2("h") - np.kron(rho, rho)).max() < 1e-14


def test_complex_context_refuses_real_only_calls():
    from paper_2410_11596_amd import binding

    g = _gpu(inputs.complex_iid_tensor(2, 2, 1), 8).step(1)
    with pytest.raises(binding.HctmError):
        binding._check(binding.lib().ctm_s_err(g._ctx, (binding.ctypes.c_double * 1)()), g._ctx)
    with pytest.raises(binding.HctmError):
        g.set_precision("fp32")
    with pytest.raises(binding.HctmError):
        _gpu(inputs.complex_iid_tensor(2, 2, 1), 8, form="dense")
    g.close()
