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
import itertools

import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, eigs

from oracle import basis, c4v, cell, complex_z2, ctmrg, hotrg
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


def _leading(rows):
    """Leading eigenpair of the transfer matrix of a stack of periodic rows
    (applied top row first), as a real Perron vector."""
    L = len(rows[0])
    n = rows[0][0].shape[0] ** L

    def mv(v):
        for r in rows:
            v = _row_apply(r, v)
        return v

    cplx = np.iscomplexobj(rows[0][0])
    op = LinearOperator((n, n), matvec=mv, dtype=np.complex128 if cplx else np.float64)
    w, v = eigs(op, k=1, which="LM", tol=1e-14, maxiter=10000)
    v = v[:, 0]
    v = v / v[np.argmax(np.abs(v))]
    # the leading eigenvalue of a row of double layers is real and positive
    assert abs(w[0].imag) < 1e-12 * abs(w[0]) and w[0].real > 0
    if cplx:
        return w[0].real, v
    assert np.abs(v.imag).max() < 1e-10
    return w[0].real, v.real


def _flipped(rows):
    """The same stack seen from below: rows in reverse order, up and down swapped."""
    return [[s.transpose(2, 1, 0, 3) for s in r] for r in reversed(rows)]


def _opened(A, s, t):
    """The double layer of A with the physical legs fixed: ket s, bra t
    (the bra layer conjugated)."""
    D = A.shape[1]
    return np.einsum("ijkl,mnop->imjnkolp", A[s], np.conj(A[t])).reshape((D * D,) * 4)


def _cylinder_cell(As, Lx, Ly, L):
    """RDMs of every site and bond of an Lx x Ly cell on a cylinder of
    circumference L (a multiple of Lx), and ln of the leading eigenvalue of
    one period of rows per site.

    Each value is a ratio of two contractions of the same stack of 2 Ly rows
    between the leading vectors above and below it, one with physical legs
    opened where the RDM sits and one closed.
    """
    d = next(iter(As.values())).shape[0]
    a = {s: basis.double_layer(A) for s, A in As.items()}

    def row(y, opened=None):
        opened = opened or {}
        return [opened.get(x, a[(x % Lx, y % Ly)]) for x in range(L)]

    lam, R = _leading([row(y) for y in range(Ly)])        # the half plane above row 0
    _, Lv = _leading(_flipped([row(y) for y in range(Ly)]))  # the half plane below row Ly-1

    def Z(opened):
        v = R
        for y in range(2 * Ly):
            v = _row_apply(row(y, opened.get(y)), v)
        return Lv @ v

    rho1, rh, rv = {}, {}, {}
    for y in range(Ly):
        for x in range(Lx):
            A0, A1, A2 = As[(x, y)], As[((x + 1) % Lx, y)], As[(x, (y + 1) % Ly)]
            r1 = np.array([[Z({y: {x: _opened(A0, s, t)}}) for t in range(d)] for s in range(d)])
            h = np.zeros((d,) * 4, dtype=a[(x, y)].dtype)
            v = np.zeros((d,) * 4, dtype=a[(x, y)].dtype)
            for s1, t1, s2, t2 in itertools.product(range(d), repeat=4):
                o1 = _opened(A0, s1, t1)
                h[s1, s2, t1, t2] = Z({y: {x: o1, x + 1: _opened(A1, s2, t2)}})
                v[s1, s2, t1, t2] = Z({y: {x: o1}, y + 1: {x: _opened(A2, s2, t2)}})
            h = h.reshape(d * d, d * d)
            v = v.reshape(d * d, d * d)
            z = Z({})
            assert abs(np.trace(r1) / z - 1) < 1e-12 and abs(np.trace(h) / z - 1) < 1e-12
            rho1[(x, y)], rh[(x, y)], rv[(x, y)] = r1 / np.trace(r1), h / np.trace(h), v / np.trace(v)
    return np.log(lam) / (L * Ly), rho1, rh, rv


def _cylinder_of(A, L):
    """ln kappa, rho1, rho2 (horizontal, vertical) of one tensor on the cylinder."""
    f, r1, rh, rv = _cylinder_cell({(0, 0): A}, 1, 1, L)
    return f, r1[(0, 0)], rh[(0, 0)], rv[(0, 0)]


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


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_cell_fixed_point_matches_the_cylinder(form):
    """A 3x2 cell of six different perturbed product states (eps = 0.05) after
    30 iterations at chi = 8, against a cylinder of circumference 6 holding
    two copies of the cell per row: every site's rho1 and every horizontal
    and vertical bond RDM within 1e-8, the energy per site within 5e-10 (the
    cylinder itself is off by about 2e-9 and 7e-11 at this circumference).
    A tensor placed at the wrong site, a bond RDM read across the wrong pair
    or a frame turned the wrong way round fails at the size of the
    correlations, 1e-3 (three columns, so that a reflection of the cell is
    not also a translation of it)."""
    Lx, Ly = 3, 2
    As = {(x, y): inputs.perturbed_product(2, 2, 10 * y + x, eps=0.05) for y in range(Ly) for x in range(Lx)}
    run = cell.CellRun(8, form, As, Lx, Ly).step(30)
    _, r1, rh, rv = _cylinder_cell(As, Lx, Ly, 6)
    h = ctmrg.heisenberg_bond()
    for (x, y) in r1:
        assert np.abs(run.rho1(x, y) - r1[(x, y)]).max() < 1e-8
        assert np.abs(run.rho2(x, y, "h") - rh[(x, y)]).max() < 1e-8
        assert np.abs(run.rho2(x, y, "v") - rv[(x, y)]).max() < 1e-8
    e_cyl = np.mean([np.trace(rh[s] @ h) + np.trace(rv[s] @ h) for s in r1])
    assert abs(run.energy() - e_cyl) < 5e-10
    assert abs(e_cyl - 0.5) > 1e-3


def test_complex_fixed_point_matches_the_cylinder():
    """Sec. II C: a complex perturbed product state (the product state plus
    0.1 times a complex i.i.d. tensor), solved in the real representation of
    its Hermitian structure at chi = 8, against the complex cylinder of
    circumference 7 with conjugated bra layers: rho1 and both bond RDMs
    within 1e-10, the energy within 1e-11 (measured: 2e-11 and 7e-15; the
    imaginary parts of the RDMs are 4e-3).  A bra layer that is not conjugated,
    or an imaginary part with the wrong sign, fails at the size of the
    imaginary parts of the RDMs."""
    A = inputs.product_state([1.0, 0.0], 2) + 0.1 * inputs.complex_iid_tensor(2, 2, 3)
    run = complex_z2.Run(8, A).step(30)
    _, r1, rh, rv = _cylinder_of(A, 7)
    assert np.abs(r1.imag).max() > 1e-3           # a genuinely complex state
    h = ctmrg.heisenberg_bond()
    assert np.abs(run.rho1() - r1).max() < 1e-10
    assert np.abs(run.rho2("h") - rh).max() < 1e-10
    assert np.abs(run.rho2("v") - rv).max() < 1e-10
    e_cyl = np.real(np.trace(rh @ h) + np.trace(rv @ h))
    assert abs(run.energy() - e_cyl) < 1e-11


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_c4v_fixed_point_matches_the_cylinder(form):
    """The C4v scheme (one corner, one edge) on the product state plus 0.2
    times a C4v-symmetrised i.i.d. tensor, run to delta < 1e-14 at chi = 8,
    against the cylinder at circumference 7: ln kappa within 5e-11, rho1
    within 2e-10, both bond RDMs within 5e-10, the energy within 2e-10
    (measured: 5e-12, 3e-11, 2e-10 and 5e-11; the energy differs from the
    product state's by 1.2e-4)."""
    A = inputs.product_state([1.0, 0.0], 2) + 0.2 * inputs.c4v_iid_tensor(2, 2, 5)
    assert c4v.is_c4v(A)
    run = c4v.C4vRun(8, form, A=A).run(100, tol=1e-14)
    assert run.deltas[-1] < 1e-14
    f, r1, rh, rv = _cylinder_of(A, 7)
    h = ctmrg.heisenberg_bond()
    assert abs(run.log_kappa() - f) < 5e-11
    assert np.abs(run.rho1() - r1).max() < 2e-10
    assert np.abs(run.rho2("h") - rh).max() < 5e-10
    assert np.abs(run.rho2("v") - rv).max() < 5e-10
    e_cyl = np.trace(rh @ h) + np.trace(rv @ h)
    assert abs(run.energy() - e_cyl) < 2e-10
    assert abs(e_cyl - 0.5) > 1e-4


def test_iid_fixed_point_between_the_cylinders():
    """An i.i.d. tensor (D = 2, seed 0, chi = 16; its energy 0.073 is far
    from a product state's): the cylinders converge slowly here (their
    error alternates in sign and shrinks about threefold per site), so this
    pin is loose: at circumference 8 the converged CTMRG is within 2e-4 of
    the cylinder in ln kappa, the RDMs and the energy, and the gap shrinks
    from circumference 7 to 8 by at least half in every one of them, i.e.
    the cylinders close in on the CTMRG value.  A wrong projector side or a
    misplaced tensor moves these numbers by 1e-2 or more."""
    A = inputs.iid_tensor(2, 2, 0)
    run = ctmrg.Run(16, "z2", A=A).run(60, tol=1e-11)
    assert run.deltas[-1] < 1e-11
    h = ctmrg.heisenberg_bond()
    got = [run.log_kappa(), run.rho1(), run.rho2("h"), run.rho2("v"), run.energy()]
    gaps = []
    for L in (7, 8):
        f, r1, rh, rv = _cylinder_of(A, L)
        ref = [f, r1, rh, rv, np.trace(rh @ h) + np.trace(rv @ h)]
        gaps.append([float(np.abs(np.asarray(g) - np.asarray(r)).max()) for g, r in zip(got, ref)])
    assert max(gaps[1]) < 2e-4
    assert all(g8 < 0.5 * g7 for g7, g8 in zip(*gaps))


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_hotrg_free_energy_matches_the_cylinder(form):
    """HOTRG (30 steps, a torus of 2^30 sites) on a perturbed product state
    (eps = 0.05, whose ln kappa is -9.3e-4) against the cylinder at
    circumference 7: ln Z per site within 2e-7 at chi = 12 and closer than
    at chi = 8 (measured 6e-8 and 1.5e-6; HOTRG keeps less of the network
    per step than CTMRG, so its error at a given chi is larger)."""
    A = inputs.perturbed_product(2, 2, 0, eps=0.05)
    f = _cylinder_of(A, 7)[0]
    e8 = abs(hotrg.Run(8, form, A=A).step(30).log_z() - f)
    e12 = abs(hotrg.Run(12, form, A=A).step(30).log_z() - f)
    assert e12 < 2e-7 and e12 < e8
