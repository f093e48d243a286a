"""Pins of the complex-tensor oracle (paper Sec. II C).

The plain complex CTMRG (oracle/ctmrg.py on complex128 tensors, the bra layer
conjugated) is pinned to: an exact brute-force contraction of the finite
patch its first iteration represents, the real oracle on real input, the
invariance of every observable under a global phase of A, and a complex
product state.  The real representation of Sec. II C (oracle/complex_z2.py:
the q leg of dimension 2 and the tensor f) is pinned to the paper's
statement that the rotated double layer has real even-total and imaginary
odd-total blocks, to complex multiplication, and to the plain complex form.
"""
import numpy as np
import pytest

from oracle import basis, bruteforce, complex_z2, ctmrg
from paper_2410_11596_amd import inputs


def _ctensor(d, D, seed):
    return inputs.complex_iid_tensor(d, D, seed)


@pytest.mark.parametrize("D,seed", [(2, 0), (3, 1), (4, 2)])
def test_rotated_double_layer_blocks_real_and_imaginary(D, seed):
    """Sec. II C: in the eigenbasis of S the blocks of even total parity are
    real and those of odd total parity imaginary."""
    A = _ctensor(2, D, seed)
    at = basis.rotate(basis.double_layer(A), basis.hermitian_basis(D))
    even = basis.parity_mask([basis.leg_parity(D)] * 4)
    m = np.abs(at).max()
    assert np.abs(at.imag[even]).max() <= 1e-15 * m
    assert np.abs(at.real[~even]).max() <= 1e-15 * m
    # both parts are really there (a complex tensor, not a real one)
    assert np.abs(at.imag[~even]).max() > 1e-3 * m


def test_f_is_the_complex_product():
    """The paper's f: f(1,1,1) = 1, f(2,2,1) = -1, f(1,2,2) = f(2,1,2) = 1
    (1-based), zero otherwise; contracting two structured matrices through it
    is their complex product."""
    F = complex_z2.F
    want = {(0, 0, 0): 1.0, (1, 1, 0): -1.0, (0, 1, 1): 1.0, (1, 0, 1): 1.0}
    for idx in np.ndindex(2, 2, 2):
        assert F[idx] == want.get(idx, 0.0)
    rng = np.random.default_rng(5)
    pa, pb, pc = (rng.integers(0, 2, n) for n in (7, 9, 5))

    def structured(pr, pc_):
        x = rng.standard_normal((len(pr), len(pc_)))
        odd = (pr[:, None] + pc_[None, :]) % 2 == 1
        return np.where(odd, 1j * x, x)

    X, Y = structured(pa, pb), structured(pb, pc)
    Z = complex_z2.from_rep(complex_z2.bmul(complex_z2.to_rep(X, [pa, pb]), complex_z2.to_rep(Y, [pb, pc]),
                                            [1], [0]))
    assert np.abs(Z - X @ Y).max() < 1e-13
    # and the product keeps the structure
    complex_z2.to_rep(Z, [pa, pc])


def test_real_input_gives_the_real_oracle():
    """A real tensor stored as complex: the plain complex oracle and the real
    representation reproduce the real oracle."""
    A = inputs.iid_tensor(2, 2, 0)
    r = ctmrg.Run(16, "dense", A=A).step(4)
    c = ctmrg.Run(16, "dense", A=A.astype(np.complex128)).step(4)
    z = complex_z2.Run(16, A).step(4)
    for o in (c, z):
        assert np.abs(o.rho1() - r.rho1()).max() < 1e-12
        assert np.abs(o.rho2("h") - r.rho2("h")).max() < 1e-12
        assert abs(o.energy() - r.energy()) < 1e-12
        for ra, rb in zip(o.records, r.records):
            k = sum(rb["kept"])
            assert sum(ra["kept"]) == k
            assert np.allclose(ra["spectrum"][:k], rb["spectrum"][:k], rtol=1e-8, atol=1e-12)


def test_first_iteration_is_exact_for_complex_tensors():
    """One iteration at D = 2, chi = 16 represents the 5 x 5 patch exactly;
    the complex brute-force contraction (bra layer conjugated) agrees."""
    A = _ctensor(2, 2, 3)
    a = basis.double_layer(A)
    b = np.eye(2).reshape(-1)
    run = ctmrg.Run(16, "dense", A=A).step(1)
    eps_bf = bruteforce.epsilon(a, b, 5)
    assert np.abs(run.epsilon() - eps_bf).max() <= 1e-10 * np.abs(eps_bf).max()
    assert np.abs(run.rho1() - bruteforce.rdm1(a, A, b, 5)).max() < 1e-11
    assert np.abs(run.rho2("h") - bruteforce.rdm2_h(a, A, b, 5, 6)).max() < 1e-11
    z = complex_z2.Run(16, A).step(1)
    assert np.abs(z.epsilon() - eps_bf).max() <= 1e-10 * np.abs(eps_bf).max()
    assert np.abs(z.rho1() - bruteforce.rdm1(a, A, b, 5)).max() < 1e-11


def test_global_phase_changes_nothing():
    A = _ctensor(2, 2, 4)
    B = A * np.exp(0.7j)
    assert np.abs(basis.double_layer(A) - basis.double_layer(B)).max() < 1e-15
    ra, rb = complex_z2.Run(12, A).step(3), complex_z2.Run(12, B).step(3)
    assert np.abs(ra.rho1() - rb.rho1()).max() < 1e-13
    assert np.abs(ra.rho2("v") - rb.rho2("v")).max() < 1e-13


def test_complex_product_state():
    """A = v (x) e_0 (x) e_0 (x) e_0 (x) e_0 with complex v: rho1 = v v^dagger / |v|^2."""
    v = np.array([0.6, 0.8j])
    A = np.zeros((2, 2, 2, 2, 2), dtype=np.complex128)
    A[:, 0, 0, 0, 0] = v
    z = complex_z2.Run(4, A).step(2)
    rho = z.rho1()
    assert np.abs(rho - np.outer(v, v.conj())).max() < 1e-14
    assert np.abs(z.rho2("h") - np.kron(rho, rho)).max() < 1e-14


@pytest.mark.parametrize("D,chi,iters", [(2, 12, 4), (2, 9, 6), (3, 20, 2)])
def test_real_representation_equals_plain_complex(D, chi, iters):
    """Sec. II C: the real representation reaches the same result as complex
    arithmetic (kept spectra, delta, RDMs, energy), and its environment and
    RDMs are Hermitian by construction while the plain form's are only
    approximately so after a truncation.  chi is below the bond growth of
    the first iteration, so that no kept value lies near the 1e-12 cutoff
    (whose inverse square root would amplify the rounding of either form to
    about 1e-8)."""
    A = _ctensor(2, D, 10 + D)
    p = ctmrg.Run(chi, "dense", A=A).step(iters)
    z = complex_z2.Run(chi, A).step(iters)
    for ra, rb in zip(z.records, p.records):
        k = sum(rb["kept"])
        assert sum(ra["kept"]) == k
        assert np.allclose(ra["spectrum"][:k], rb["spectrum"][:k], rtol=1e-8, atol=1e-12)
    assert np.abs(np.array(z.deltas) - np.array(p.deltas)).max() < 1e-9
    for f in ("h", "v"):
        assert np.abs(z.rho2(f) - p.rho2(f)).max() < 1e-10
    r1 = z.rho1()
    assert np.abs(r1 - p.rho1()).max() < 1e-10
    assert abs(z.energy() - p.energy()) < 1e-10
    assert np.abs(r1 - r1.conj().T).max() < 1e-15
    assert z.s_err() < 1e-14


@pytest.mark.parametrize("chi", [6, 14])
def test_truncated_cut_is_the_best_rank_k_cut(chi):
    """One cut of the real representation (reading: M decomposed through the
    real R = D^-1 M D) against a complex SVD of the whole loop: with the
    halves contracted independently from the complex tensors, P_b P_a = 1,
    ||M - H_d P_a P_b H_u|| is the discarded weight (Eckart-Young), k =
    min(chi, #{s > tau s_max}) and the recorded spectrum is M's.  A sign of
    D^-1 M D, or of the imaginary part of V or W, fails these."""
    from test_oracle_pins import _halves_by_einsum

    A = _ctensor(2, 3, 21)
    run = complex_z2.Run(12, A).step(3)
    env = run.env
    top, right, bottom, left = env.par
    pq = run.par_q
    pW = ((left[:, None] + pq[None, :]) % 2).reshape(-1)
    pE = ((right[:, None] + pq[None, :]) % 2).reshape(-1)
    Q = complex_z2.quadrants(env.t, run.at)
    Pa, Pb, rec = complex_z2.cut_projectors(*Q, chi, 1e-12, pW, pE)
    k = Pa.shape[2]
    Pa = complex_z2.from_rep(Pa).reshape(-1, k)
    Pb = complex_z2.from_rep(Pb).reshape(k, -1)

    plain = ctmrg.Env([complex_z2.from_rep(x) for x in env.t])
    Hu, Hd = _halves_by_einsum(plain, complex_z2.from_rep(run.at))
    M = Hd @ Hu
    s = np.linalg.svd(M, compute_uv=False)
    assert k == max(1, min(chi, int(np.sum(s > 1e-12 * s[0]))))
    assert np.allclose(rec["spectrum"][:k], s[:k] / s[0], rtol=1e-9, atol=1e-13)
    assert np.abs(Pb @ Pa - np.eye(k)).max() < 1e-9
    err = np.linalg.norm(M - Hd @ Pa @ Pb @ Hu)
    want = np.sqrt(np.sum(s[k:] ** 2))
    assert abs(err - want) <= 1e-8 * s[0] + 1e-6 * want
