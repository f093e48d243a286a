"""Pin of the oracle's converged fixed point against an infinite cylinder.

An independent route to the same infinite network: roll the plane into a
cylinder of circumference L, find the leading left and right eigenvectors
of its row transfer matrix (ARPACK on a matrix-free product), and read the
free energy per site and the reduced density matrices from them.  On a
state with a short correlation length the cylinder reaches the plane
exponentially fast in L.  The perturbed product state used here (D = 2,
eps = 0.1; second transfer eigenvalue 0.073 of the first) is correlated
(its Heisenberg energy differs from the product state's 1/2 by 3e-5), and
at L = 7 the cylinder agrees with the plane to about 1e-11 in ln kappa and
1e-9 in the RDMs.  Nothing here calls the oracle's contractions: only
basis.double_layer (pinned against the paper's example elsewhere) forms
the transfer tensor.
"""
import functools

import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, eigs

from oracle import basis, ctmrg
from paper_2410_11596_amd import inputs

L_CYL = 7


def _row_apply(sites, v):
    """One periodic row of 4-leg tensors [u, l, d, r] applied to v[u_1..u_L].

    Returns w[d_1..d_L]: the row is absorbed site by site, carrying the
    first site's left leg and the current right leg, and closed at the end.
    """
    L = len(sites)
    q = sites[0].shape[0]
    t = np.tensordot(sites[0], v.reshape((q,) * L), ([0], [0]))   # [l1, d1, r1, u2..uL]
    t = np.moveaxis(t, 2, 1)                                      # [l1, r1, d1, u2..uL]
    for i in range(1, L):
        t = np.tensordot(t, sites[i], ([1, 2 + i], [1, 0]))       # [l1, d1..di, u.., d, r]
        t = np.moveaxis(t, -1, 1)
        t = np.moveaxis(t, -1, 2 + i)                             # [l1, r, d1..d_{i+1}, u..]
    return np.trace(t, axis1=0, axis2=1).reshape(-1)


def _leading(a, L):
    n = a.shape[0] ** L
    op = LinearOperator((n, n), matvec=lambda v: _row_apply([a] * L, v), dtype=np.float64)
    w, v = eigs(op, k=1, which="LM", tol=1e-14, maxiter=10000)
    v = v[:, 0]
    v = v / v[np.argmax(np.abs(v))]          # the Perron vector, made real
    assert abs(w[0].imag) < 1e-12 * abs(w[0]) and np.abs(v.imag).max() < 1e-10
    return w[0].real, v.real


def _cylinder_of(A, L):
    """ln kappa, rho1, rho2 (horizontal, vertical) on the cylinder."""
    d = A.shape[0]
    a = basis.double_layer(A)
    lam, R = _leading(a, L)                          # the half plane above a row
    _, Lv = _leading(a.transpose(2, 1, 0, 3), L)     # the half plane below it

    def opened(s, t):
        # the double layer with the physical legs fixed: ket s, bra t
        return np.einsum("ijkl,mnop->imjnkolp", A[s], A[t]).reshape(a.shape)

    z = Lv @ _row_apply([a] * L, R)
    r1 = np.array([[Lv @ _row_apply([opened(s, t)] + [a] * (L - 1), R) for t in range(d)]
                   for s in range(d)])
    rh = np.zeros((d, d, d, d))
    rv = np.zeros((d, d, d, d))
    for s1 in range(d):
        for t1 in range(d):
            top = _row_apply([opened(s1, t1)] + [a] * (L - 1), R)
            for s2 in range(d):
                for t2 in range(d):
                    rh[s1, s2, t1, t2] = Lv @ _row_apply([opened(s1, t1), opened(s2, t2)] + [a] * (L - 2), R)
                    rv[s1, s2, t1, t2] = Lv @ _row_apply([opened(s2, t2)] + [a] * (L - 1), top)
    rh = rh.reshape(d * d, d * d)
    rv = rv.reshape(d * d, d * d)
    assert abs(np.trace(r1) / z - 1) < 1e-12 and abs(np.trace(rh) / z - 1) < 1e-12
    return np.log(lam) / L, r1 / np.trace(r1), rh / np.trace(rh), rv / np.trace(rv)


@functools.lru_cache(maxsize=None)
def _cylinder(eps, seed, L):
    return _cylinder_of(inputs.perturbed_product(2, 2, seed, eps=eps), L)


def test_cylinder_on_a_product_state():
    """The cylinder itself: a normalised product state has one state per row,
    so ln kappa = 0 and its RDMs are v v^T and (v v^T) (x) (v v^T), at any L."""
    v = np.array([0.6, 0.8])
    A = inputs.product_state(v, 2)
    one = np.outer(v, v)
    for L in (3, 4):
        f, r1, rh, rv = _cylinder_of(A, L)
        assert abs(f) < 1e-13
        assert np.abs(r1 - one).max() < 1e-13
        assert np.abs(rh - np.kron(one, one)).max() < 1e-13
        assert np.abs(rv - np.kron(one, one)).max() < 1e-13


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_fixed_point_matches_the_cylinder(form):
    """Converged CTMRG (chi = 8, run to delta < 1e-14) against the cylinder at
    L = 7: ln kappa within 5e-11, rho1 within 1e-9, both bond RDMs within
    3e-9, the Heisenberg energy within 1e-10."""
    eps, seed = 0.1, 0
    A = inputs.perturbed_product(2, 2, seed, eps=eps)
    run = ctmrg.Run(8, form, A=A).run(100, tol=1e-14)
    assert run.deltas[-1] < 1e-14
    f, r1, rh, rv = _cylinder(eps, seed, L_CYL)
    h = ctmrg.heisenberg_bond()
    assert abs(run.log_kappa() - f) < 5e-11
    assert np.abs(run.rho1() - r1).max() < 1e-9
    assert np.abs(run.rho2("h") - rh).max() < 3e-9
    assert np.abs(run.rho2("v") - rv).max() < 3e-9
    e_cyl = np.trace(rh @ h) + np.trace(rv @ h)
    assert abs(run.energy() - e_cyl) < 1e-10
    # the state is not a product state: a product state's energy is 1/2
    assert abs(e_cyl - 0.5) > 1e-5
