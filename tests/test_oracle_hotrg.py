"""Pins of the HOTRG oracle (oracle/hotrg.py) against what the mathematics
fixes: without truncation a step is exact, so after one and two steps ln Z is
that of the 1 x 2 and 2 x 2 tori contracted directly, and for the Ising PEPS
that of the spin sum on the 2 x 2 and 2 x 4 tori; with truncation the Ising
free energy converges to Onsager's; the probe b is antisymmetric under the
bra-ket swap (odd in the rotated basis), so an untruncated network gives
Z_b = 0, and |b| placed on one site of the 2 x 2 torus gives the direct
contraction; the plain and Z2 forms agree."""
import itertools

import numpy as np
import pytest

from oracle import basis, ctmrg, hotrg
from paper_2410_11596_amd import inputs
from test_oracle_pins import ising_nn_corr, onsager_log_z

EXACT = dict(chi=10**6, tau=0.0)


def torus_1x2(a):
    return np.einsum("ABCB,CEAE->", a, a)


def torus_2x2(a00, a10, a01, a11):
    """Sites (x, y) with legs [u, l, d, r]; right and down neighbours modulo 2."""
    return np.einsum("ABCD,EDFB,CGAH,FHEG->", a00, a10, a01, a11, optimize=True)


def ising_spin_sum(beta, Lx, Ly):
    """Z of the Ising model (J = 1) on an Lx x Ly torus by enumeration."""
    n = Lx * Ly
    Z = 0.0
    for bits in itertools.product((1, -1), repeat=n):
        s = np.array(bits).reshape(Ly, Lx)
        e = np.sum(s * np.roll(s, 1, axis=0)) + np.sum(s * np.roll(s, 1, axis=1))
        Z += np.exp(beta * e)
    return Z


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_untruncated_steps_are_the_tori(form):
    A = inputs.iid_tensor(2, 2, 0)
    a = basis.double_layer(A)
    r = hotrg.Run(form=form, A=A, **EXACT).step(1)
    assert abs(2 * r.log_z() - np.log(torus_1x2(a))) < 1e-13
    r.step(1)
    assert abs(4 * r.log_z() - np.log(torus_2x2(a, a, a, a))) < 1e-13


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_ising_peps_spin_sums(form):
    beta = 0.4
    A = inputs.ising_peps(beta)
    r = hotrg.Run(form=form, A=A, **EXACT).step(2)
    assert abs(4 * r.log_z() - np.log(ising_spin_sum(beta, 2, 2))) < 1e-12
    r.step(1)
    assert abs(8 * r.log_z() - np.log(ising_spin_sum(beta, 2, 4))) < 1e-12


@pytest.mark.parametrize("beta", [0.30, 0.60])
def test_ising_free_energy_onsager(beta):
    """20 steps: a torus of 2^20 sites.  In the ordered phase (beta = 0.6)
    its Z counts both magnetised states, ln Z / N = -beta f + ln 2 / N."""
    k = 20
    r = hotrg.Run(10, "z2", A=inputs.ising_peps(beta)).step(k)
    degeneracy = np.log(2.0) / 2**k if beta > 0.5 * np.log(1 + np.sqrt(2)) else 0.0
    assert abs(r.log_z() - onsager_log_z(beta) - degeneracy) < 2e-8


def test_probe_b_is_swap_odd():
    D = 2
    b = hotrg.probe_b(D)
    ab = hotrg.probe_b(D, absolute=True)
    S = basis.swap_matrix(D)
    sb = basis.apply_on_all_legs(S, b)
    assert np.array_equal(sb, -b)  # ket <-> bra on every leg is the matrix transpose
    assert np.array_equal(basis.apply_on_all_legs(S, ab), ab)
    assert np.count_nonzero(b) == D ** 8 - D ** 4
    U = basis.hermitian_basis(D)
    p = basis.leg_parity(D)
    bt = basis.rotate(b, U)
    assert np.abs(hotrg._mask_parity(bt, [p] * 4, 0)).max() < 1e-15  # no even block


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_probe_untruncated(form):
    A = inputs.iid_tensor(2, 2, 3)
    a = basis.double_layer(A)
    r = hotrg.Run(form=form, A=A, probes=True, **EXACT).step(2)
    rb, rab = r.impurity_ratios()
    z = torus_2x2(a, a, a, a)
    assert abs(rab - torus_2x2(hotrg.probe_b(2, absolute=True), a, a, a) / z) < 1e-12 * abs(rab)
    assert abs(torus_2x2(hotrg.probe_b(2), a, a, a) / z) < 1e-13  # the exact network is Hermitian
    assert abs(rb) < 1e-13 * abs(rab)
    if form == "z2":
        assert rb == 0.0


def test_probe_with_truncation_z2_exact_zero():
    r = hotrg.Run(10, "z2", A=inputs.iid_tensor(2, 3, 1), probes=True).step(5)
    assert r.sym_error() == 0.0
    assert abs(r.impurity_ratios()[1]) > 0.0


def test_rotation_invariance_untruncated():
    A = inputs.iid_tensor(2, 2, 4)
    a = basis.double_layer(A)
    r0 = hotrg.Run(form="dense", a=a, **EXACT).step(2)
    r1 = hotrg.Run(form="dense", a=ctmrg.rot_a(a, 1), **EXACT).step(2)
    assert abs(r0.log_z() - r1.log_z()) < 1e-13


@pytest.mark.parametrize("D,chi", [(2, 8), (3, 12)])
def test_plain_and_z2_forms_agree(D, chi):
    A = inputs.iid_tensor(2, D, 5)
    z = hotrg.Run(chi, "z2", A=A).step(6)
    p = hotrg.Run(chi, "dense", A=A).step(6)
    assert abs(z.log_z() - p.log_z()) < 1e-10
    for rz, rp in zip(z.records, p.records):
        assert sum(rz["kept"]) == sum(rp["kept"])
        k = len(rz["spectrum"])
        assert np.allclose(rz["spectrum"], rp["spectrum"][:k], rtol=1e-8, atol=1e-13)
        assert np.allclose(rz["discarded"], rp["discarded"], rtol=1e-6, atol=1e-13)


def heis():
    return inputs.heisenberg_bond_matrix()


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_bond_energy_untruncated_is_the_torus_expectation(form):
    """Two exact steps: <h> on the vertical bond (0,0)-(0,1) of the 2 x 2
    torus, against the direct contraction with the physical indices open."""
    A = inputs.iid_tensor(2, 2, 6)
    a = basis.double_layer(A)
    h = heis().reshape(2, 2, 2, 2)
    num = 0.0
    for s1, s2, t1, t2 in itertools.product(range(2), repeat=4):
        if h[s1, s2, t1, t2] != 0.0:
            num += h[s1, s2, t1, t2] * torus_2x2(basis.impurity(A, s1, t1), a, basis.impurity(A, s2, t2), a)
    e_exact = num / torus_2x2(a, a, a, a)
    r = hotrg.Run(form=form, A=A, bond=heis(), **EXACT).step(2)
    assert abs(r.energy() - e_exact) < 1e-13


@pytest.mark.parametrize("beta", [0.30, 0.60])
def test_ising_nearest_neighbour_correlation(beta):
    """Onsager's <s_i s_j>: an impurity observable carries the truncation
    error to first order (2.6e-6 at chi = 10, 8e-7 at chi = 16 for
    beta = 0.3), so the bound is looser than the free energy's."""
    zz = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
    r = hotrg.Run(10, "z2", A=inputs.ising_peps(beta), bond=zz).step(20)
    assert abs(r.energy() - ising_nn_corr(beta)) < 5e-6


def test_bond_energy_forms_agree():
    A = inputs.iid_tensor(2, 3, 8)
    z = hotrg.Run(12, "z2", A=A, bond=heis()).step(6)
    p = hotrg.Run(12, "dense", A=A, bond=heis()).step(6)
    assert abs(z.energy() - p.energy()) < 1e-10


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_rho1_untruncated_is_the_torus_rdm(form):
    A = inputs.iid_tensor(3, 2, 9)
    a = basis.double_layer(A)
    z = torus_2x2(a, a, a, a)
    exact = np.array([[torus_2x2(basis.impurity(A, s, t), a, a, a) / z for t in range(3)] for s in range(3)])
    r = hotrg.Run(form=form, A=A, rdm1=True, **EXACT).step(2)
    assert np.abs(r.rho1() - exact).max() < 1e-13


def test_rho1_symmetric_in_z2_and_forms_agree():
    A = inputs.iid_tensor(2, 3, 4)
    z = hotrg.Run(10, "z2", A=A, rdm1=True).step(6)
    p = hotrg.Run(10, "dense", A=A, rdm1=True).step(6)
    rz, rp = z.rho1(), p.rho1()
    assert np.array_equal(rz, rz.T) and abs(np.trace(rz) - 1.0) < 1e-14
    assert np.abs(rz - rp).max() < 1e-10
    v = np.array([0.6, -0.8])
    r = hotrg.Run(8, "z2", A=inputs.product_state(v, 2), rdm1=True).step(4).rho1()
    assert np.abs(r - np.outer(v, v)).max() < 1e-14


@pytest.mark.parametrize("form", ["dense", "z2"])
@pytest.mark.parametrize("chi", [6, 12])
def test_isometry_is_the_best_rank_k_cut(form, chi):
    """One truncated HOTRG step (H2, H3) against a plain SVD of both
    matricisations of the joined tensor M: U has orthonormal columns; the
    discarded weight of each side is ||M - U U^T M||^2 with that side's U,
    and equals the sum of the squared singular values past the kept count
    (Eckart-Young), k = min(chi, #{s^2 > tau s_max^2}); the side taken is
    the one that discards less (the left one on a tie); the kept spectrum is
    that side's s^2 / s_max^2; in the Z2 form every column of U lies in one
    parity sector.  A Gram matrix of the wrong side, keeping the wrong
    eigenvectors or taking the worse side fails one of these."""
    A = inputs.iid_tensor(2, 2, 6)
    r = hotrg.Run(chi, form, A=A).step(2)
    M = hotrg.join_vertical(r.T, r.T)
    ph = r.ph if form == "z2" else None
    U, side, kept, spec, errs = hotrg.isometry(M, chi, 1e-12, ph)
    n = M.shape[1] * M.shape[2]
    k = U.shape[1]
    assert sum(kept) == k
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12

    mats = (M.transpose(1, 2, 0, 3, 4, 5).reshape(n, -1), M.transpose(4, 5, 0, 1, 2, 3).reshape(n, -1))
    want = []
    for Mm in mats:
        s = np.linalg.svd(Mm, compute_uv=False)
        kk = min(chi, int(np.sum(s ** 2 > 1e-12 * s[0] ** 2)))
        assert kk == k
        want.append((float(np.sum(s[kk:] ** 2)), s[:kk] ** 2 / s[0] ** 2))
    total = float(np.sum(mats[0] ** 2))
    for sd in (0, 1):
        assert abs(errs[sd] - want[sd][0]) < 1e-10 * total
    assert want[0][0] > 1e-8 * total and want[1][0] > 1e-8 * total  # both sides truncate
    best = 0 if want[0][0] <= want[1][0] + 1e-10 * total else 1
    assert side == best
    assert np.allclose(spec, want[side][1], rtol=1e-9, atol=1e-14)
    Mm = mats[side]
    assert abs(np.sum((Mm - U @ (U.T @ Mm)) ** 2) - want[side][0]) < 1e-10 * total
    if form == "z2":
        pf = ((ph[:, None] + ph[None, :]) % 2).reshape(-1)
        newp = np.array([0] * kept[0] + [1] * kept[1])
        assert np.all(U[pf[:, None] != newp[None, :]] == 0)
