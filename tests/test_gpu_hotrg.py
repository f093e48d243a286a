"""GPU parity of HOTRG (include/hctm_hotrg.h) against the HOTRG oracle
(oracle/hotrg.py) on the same seeded tensors, Z2 and plain forms: ln Z per
site within 1e-10 (relative to max(1, |ln Z|)), the kept sector sizes and the
chosen side of every step exactly, the kept spectra within 1e-8 relative and
the discarded weights within 1e-6 relative; the probe ratios Z_b / Z and
Z_|b| / Z within 1e-10 of |Z_|b| / Z|, and Z_b exactly zero in the Z2 form.
At sizes the oracle cannot hold (its joined tensor has chi^6 entries) the
two GPU forms are compared with each other."""
import numpy as np
import pytest

from oracle import hotrg
from paper_2410_11596_amd import inputs
from test_oracle_pins import onsager_log_z

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


def _gpu(A, chi, form, steps, **kw):
    from paper_2410_11596_amd import HOTRG

    h = HOTRG(A, chi, form=form, **kw)
    h.step(steps)
    return h


def _compare(g, o, tol=1e-10):
    lz = o.log_z()
    assert abs(g.log_z() - lz) < tol * max(1.0, abs(lz))
    recs = g.records()
    assert len(recs) == len(o.records)
    for rg, ro in zip(recs, o.records):
        assert tuple(rg["kept"]) == tuple(ro["kept"])
        assert rg["side"] == ro["side"]
        assert np.allclose(rg["spectrum"], ro["spectrum"], rtol=1e-8, atol=1e-14)
        assert np.allclose(rg["discarded"], ro["discarded"], rtol=1e-6, atol=1e-13)


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_untruncated_two_steps(form):
    A = inputs.iid_tensor(2, 2, 0)
    o = hotrg.Run(16, form, A=A, tau=0.0).step(2)
    g = _gpu(A, 16, form, 2, svd_rel_cutoff=0.0)
    assert abs(g.log_z() - o.log_z()) < 1e-13


@pytest.mark.parametrize("form", ["z2", "dense"])
@pytest.mark.parametrize("D,chi,steps", [(2, 8, 12), (3, 12, 8), (4, 16, 4)])
def test_truncated_steps(form, D, chi, steps):
    A = inputs.iid_tensor(2, D, 5)
    o = hotrg.Run(chi, form, A=A).step(steps)
    g = _gpu(A, chi, form, steps)
    _compare(g, o)


@pytest.mark.parametrize("beta", [0.30, 0.60])
def test_ising_free_energy_onsager(beta):
    k = 20
    g = _gpu(inputs.ising_peps(beta), 10, "z2", k)
    degeneracy = np.log(2.0) / 2**k if beta > 0.5 * np.log(1 + np.sqrt(2)) else 0.0
    assert abs(g.log_z() - onsager_log_z(beta) - degeneracy) < 2e-8


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_symmetry_probe(form):
    A = inputs.iid_tensor(2, 3, 1)
    o = hotrg.Run(10, form, A=A, probes=True).step(5)
    g = _gpu(A, 10, form, 5, probes=True)
    _compare(g, o)
    zb, zab = g.impurity_ratios()
    ob, oab = o.impurity_ratios()
    assert abs(zab - oab) < 1e-10 * abs(oab)
    assert abs(zb - ob) < 1e-10 * abs(oab)
    if form == "z2":
        assert zb == 0.0 and g.sym_error() == 0.0


def test_forms_agree_at_chi32():
    """chi = 32 (Gram matrices of 1024 rows in the plain form, two sectors of
    about 512 in the Z2 form): the largest plain size."""
    A = inputs.iid_tensor(2, 2, 7)
    z = _gpu(A, 32, "z2", 8, probes=True)
    p = _gpu(A, 32, "dense", 8, probes=True)
    assert abs(z.log_z() - p.log_z()) < 1e-9 * max(1.0, abs(p.log_z()))
    for rz, rp in zip(z.records(), p.records()):
        assert sum(rz["kept"]) == sum(rp["kept"])
    assert z.sym_error() == 0.0
    assert np.isfinite(p.sym_error())


def test_d6_chi36_z2():
    """D = 6 (21 + 15): the Gram sectors of the first step hold 666 and 630
    rows."""
    A = inputs.iid_tensor(2, 6, 0)
    g = _gpu(A, 36, "z2", 3, probes=True)
    assert all(sum(r["kept"]) <= 36 for r in g.records())
    assert np.isfinite(g.log_z())
    assert g.sym_error() == 0.0


@pytest.mark.parametrize("form,chi,steps", [("dense", 18, 6), ("z2", 24, 5)])
def test_subspace_eigensolver_against_oracle(form, chi, steps):
    """Gram sectors above 256 rows (324 in the plain form at chi = 18, 320 in
    the Z2 form at chi = 24) go to the subspace iteration."""
    A = inputs.iid_tensor(2, 2, 9)
    o = hotrg.Run(chi, form, A=A).step(steps)
    g = _gpu(A, chi, form, steps)
    _compare(g, o)


def test_forms_agree_at_chi48_subspace_sectors():
    """chi = 48: plain Gram matrices of 2304 rows, Z2 sectors of about 1150,
    all by subspace iteration."""
    A = inputs.iid_tensor(2, 2, 11)
    z = _gpu(A, 48, "z2", 6)
    p = _gpu(A, 48, "dense", 6)
    assert abs(z.log_z() - p.log_z()) < 1e-9 * max(1.0, abs(p.log_z()))
    for rz, rp in zip(z.records(), p.records()):
        assert sum(rz["kept"]) == sum(rp["kept"])
        k = len(rz["spectrum"])
        assert np.allclose(rz["spectrum"], rp["spectrum"][:k], rtol=1e-7, atol=1e-13)


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_degenerate_sizes(form):
    """D = 1 (the double layer is a number: ln Z = ln a exactly), chi = 1
    (one state per step) and a product state (rank-one network) against the
    oracle and the closed forms."""
    A1 = inputs.iid_tensor(3, 1, 2)
    g = _gpu(A1, 4, form, 3)
    a = float(np.sum(A1.reshape(3) ** 2))
    assert abs(g.log_z() - np.log(a)) < 1e-13
    A = inputs.iid_tensor(2, 2, 4)
    o = hotrg.Run(1, form, A=A).step(6)
    g = _gpu(A, 1, form, 6)
    _compare(g, o)
    assert all(sum(r["kept"]) == 1 for r in g.records())
    v = np.array([0.6, -0.8, 0.3])
    P = inputs.product_state(v, 3)
    g = _gpu(P, 8, form, 5, probes=True)
    assert abs(g.log_z() - np.log(v @ v)) < 1e-13
    assert all(sum(r["kept"]) == 1 for r in g.records())


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_bond_energy_against_oracle(form):
    h = inputs.heisenberg_bond_matrix()
    A = inputs.iid_tensor(2, 2, 6)
    o = hotrg.Run(16, form, A=A, tau=0.0, bond=h).step(2)
    g = _gpu(A, 16, form, 2, svd_rel_cutoff=0.0, bond=h)
    assert abs(g.energy() - o.energy()) < 1e-13  # untruncated: the 2 x 2 torus
    A = inputs.iid_tensor(2, 3, 8)
    o = hotrg.Run(12, form, A=A, bond=h).step(6)
    g = _gpu(A, 12, form, 6, bond=h)
    _compare(g, o)
    assert abs(g.energy() - o.energy()) < 1e-10


def test_ising_correlation_and_plain_z2_energy_difference():
    zz = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
    from test_oracle_pins import ising_nn_corr

    g = _gpu(inputs.ising_peps(0.3), 10, "z2", 20, bond=zz)
    assert abs(g.energy() - ising_nn_corr(0.3)) < 5e-6
    h = inputs.heisenberg_bond_matrix()
    A = inputs.iid_tensor(2, 2, 7)
    z = _gpu(A, 32, "z2", 10, bond=h)
    p = _gpu(A, 32, "dense", 10, bond=h)
    assert abs(z.energy() - p.energy()) < 1e-9


def test_api_misuse_is_an_argument_error_and_leaves_the_context_usable():
    from paper_2410_11596_amd import HctmError, binding

    h = inputs.heisenberg_bond_matrix()
    A = inputs.iid_tensor(2, 2, 3)
    g = _gpu(A, 8, "z2", 0)
    with pytest.raises(HctmError) as e:
        g.energy()  # no bond operator
    assert e.value.code == binding.CTM_E_ARG
    with pytest.raises(HctmError) as e:
        g.sym_error()  # no probes
    assert e.value.code == binding.CTM_E_ARG
    g2 = _gpu(A, 8, "z2", 0, bond=h)
    with pytest.raises(HctmError):
        g2.energy()  # no step yet
    g2.step(2)
    e2 = g2.energy()
    with pytest.raises(HctmError) as e:
        binding._hcheck(binding.lib().hotrg_set_bond(g2._ctx, binding._dptr(np.ascontiguousarray(h))), g2._ctx)
    assert e.value.code == binding.CTM_E_ARG  # after the first step
    g2.step(1)  # still usable
    assert np.isfinite(g2.energy()) and np.isfinite(e2)
    A5 = inputs.iid_tensor(5, 2, 1)
    with pytest.raises(HctmError):
        _gpu(A5, 8, "z2", 0, bond=np.eye(25))  # d > 4


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_rho1_against_oracle(form):
    A = inputs.iid_tensor(3, 2, 9)
    o = hotrg.Run(16, form, A=A, tau=0.0, rdm1=True).step(2)
    g = _gpu(A, 16, form, 2, svd_rel_cutoff=0.0, rdm1=True)
    assert np.abs(g.rho1() - o.rho1()).max() < 1e-13  # untruncated: the 2 x 2 torus
    A = inputs.iid_tensor(2, 3, 4)
    o = hotrg.Run(10, form, A=A, rdm1=True, probes=True, bond=inputs.heisenberg_bond_matrix()).step(6)
    g = _gpu(A, 10, form, 6, rdm1=True, probes=True, bond=inputs.heisenberg_bond_matrix())
    _compare(g, o)
    r = g.rho1()
    assert np.abs(r - o.rho1()).max() < 1e-10
    assert abs(g.energy() - o.energy()) < 1e-10
    if form == "z2":
        assert np.array_equal(r, r.T)  # Hermitian by construction
    assert abs(np.trace(r) - 1.0) < 1e-14
