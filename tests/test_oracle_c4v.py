"""Pins of the C4v oracle (oracle/c4v.py) against what the paper and the
mathematics fix: the symmetrised tensor has all eight symmetries; the C4v
environment is symmetric (C = C^T, T symmetric in its two boundary legs);
its fixed point is that of the directional CTMRG (the same network, another
truncation scheme); the Ising PEPS gives Onsager's free energy and
nearest-neighbour correlation and Yang's magnetisation; the plain and Z2
forms agree."""
import numpy as np
import pytest

from oracle import c4v, ctmrg
from paper_2410_11596_amd import inputs
from test_oracle_pins import ising_nn_corr, onsager_log_z, yang_m


def c4v_tensor(D, seed):
    return c4v.c4v_symmetrize(inputs.iid_tensor(2, D, seed))


def test_symmetrised_tensor_has_the_eight_symmetries():
    A = c4v_tensor(3, 1)
    assert c4v.is_c4v(A)
    assert not c4v.is_c4v(inputs.iid_tensor(2, 3, 1))
    # a symmetric tensor is its own symmetrisation
    assert np.abs(c4v.c4v_symmetrize(A) - A).max() < 1e-15


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_fixed_point_is_the_directional_one(form):
    A = c4v_tensor(2, 0)
    r = c4v.C4vRun(16, form, A=A).run(200, tol=1e-12)
    d = ctmrg.Run(16, form, A=A).run(120, tol=1e-12)
    assert r.deltas[-1] < 1e-12
    assert np.abs(r.rho1() - d.rho1()).max() < 1e-12
    assert np.abs(r.rho2("h") - d.rho2("h")).max() < 1e-12
    assert np.abs(r.rho2("v") - d.rho2("v")).max() < 1e-12
    C, T = r.env.t[0], r.env.t[1]
    assert np.abs(C - C.T).max() < 1e-14
    assert np.abs(T - T.transpose(2, 1, 0)).max() < 1e-14
    # one corner and one edge for the whole environment
    assert all(x is C for x in r.env.t[0::2]) and all(x is T for x in r.env.t[1::2])


@pytest.mark.parametrize("beta", [0.40, 0.45])
def test_ising_peps_against_onsager_and_yang(beta):
    A = inputs.ising_peps(beta)
    assert c4v.is_c4v(A)
    bnd = inputs.ising_up_boundary(beta) if beta > 0.44 else None
    r = c4v.C4vRun(16, "z2", A=A, boundary=bnd).run(400, tol=1e-13)
    assert abs(r.log_kappa() - onsager_log_z(beta)) < 1e-10
    zz = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
    assert abs(np.trace(r.rho2("h") @ zz) - ising_nn_corr(beta)) < 1e-8
    r1 = r.rho1()
    assert abs((r1[0, 0] - r1[1, 1]) - yang_m(beta)) < 1e-7


@pytest.mark.parametrize("D,chi", [(2, 12), (3, 20)])
def test_dense_and_z2_forms_agree(D, chi):
    A = c4v_tensor(D, 5)
    z = c4v.C4vRun(chi, "z2", A=A).step(6)
    p = c4v.C4vRun(chi, "dense", A=A).step(6)
    assert np.abs(z.rho1() - p.rho1()).max() < 1e-10
    assert np.abs(z.rho2("h") - p.rho2("h")).max() < 1e-10
    for rz, rp in zip(z.records, p.records):
        k = sum(rz["kept"])
        assert k == sum(rp["kept"])
        assert np.allclose(rz["spectrum"][:k], rp["spectrum"][:k], rtol=1e-8, atol=1e-13)


@pytest.mark.parametrize("form", ["dense", "z2"])
@pytest.mark.parametrize("chi", [10, 25])
def test_truncation_keeps_the_largest_moduli(form, chi):
    """One C4v truncation (Sec. II A, reading R16) against an eigendecomposition
    of the enlarged corner contracted independently: the corner is symmetric;
    the kept count is min(chi, #{|lambda| > tau |lambda|_max}) over both
    sectors and the recorded spectrum is the largest moduli; the new corner
    P^T Q P is diagonal with those moduli (normalised).  Keeping by value
    instead of modulus, or one sector only, fails these."""
    A = inputs.c4v_iid_tensor(2, 3, 1)
    run = c4v.C4vRun(12, form, A=A).step(3)
    env = run.env.copy()
    C1, T1, _, _, _, _, _, T4 = env.t
    Q = np.einsum("cx,xut,wlc,uldr->wdtr", C1, T1, T4, run.a)
    n = Q.shape[0] * Q.shape[1]
    M = Q.reshape(n, n)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    lam = np.linalg.eigvalsh(M)
    assert lam.min() < 0 < lam.max()  # both signs occur, so value and modulus orders differ
    mod = np.sort(np.abs(lam))[::-1]
    rec = c4v.c4v_move(env, run.a, chi, 1e-12, run.par_q)
    k = sum(rec["kept"])
    assert k == min(chi, int(np.sum(mod > 1e-12 * mod[0])))
    assert np.allclose(rec["spectrum"][:k], mod[:k] / mod[0], rtol=1e-9, atol=1e-13)
    Cn = env.t[0]
    assert np.abs(Cn - np.diag(np.diag(Cn))).max() < 1e-10
    assert np.allclose(np.sort(np.abs(np.diag(Cn)))[::-1], mod[:k] / np.linalg.norm(mod[:k]), rtol=1e-8, atol=1e-13)
