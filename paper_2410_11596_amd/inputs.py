"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws and assembles input tensors; it holds none of the
contraction method's arithmetic.  The paper benchmarks converged Heisenberg
ground states (Sec. III); those tensors are not available, so i.i.d.
Gaussian tensors of the same shapes stand in for them.

Leg order of a single-layer tensor: [s, u, l, d, r] (physical first).
"""
import numpy as np


def iid_tensor(d, D, seed):
    """Real tensor with i.i.d. N(0,1) entries, divided by its largest |entry|."""
    A = np.random.default_rng(seed).standard_normal((d, D, D, D, D))
    return A / np.abs(A).max()


def complex_iid_tensor(d, D, seed):
    """Complex tensor whose real and imaginary parts are i.i.d. N(0,1) (both
    drawn from one seeded generator, real part first), divided by its largest
    |entry|."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((d, D, D, D, D))
    im = rng.standard_normal((d, D, D, D, D))
    A = re + 1j * im
    return A / np.abs(A).max()


def c4v_iid_tensor(d, D, seed):
    """iid_tensor(d, D, seed) averaged over the eight symmetries of the square
    (the rotations of the virtual legs [u, l, d, r], each with and without the
    left-right reflection): a tensor with the C4v symmetry."""
    A = iid_tensor(d, D, seed)
    out = np.zeros_like(A)
    for B in (A, A.transpose(0, 1, 4, 3, 2)):
        for r in range(4):
            out += B.transpose((0,) + tuple(1 + (np.arange(4) + r) % 4))
    return out / 8.0


def iid_cell(d, D, seeds):
    """Several independent tensors (one per unit-cell site)."""
    return [iid_tensor(d, D, s) for s in seeds]


def perturbed_product(d, D, seed, eps=1e-2):
    """e_{s=0} x e_0 x e_0 x e_0 x e_0 plus eps times an N(0,1) tensor, max-abs normalised."""
    A = np.zeros((d, D, D, D, D))
    A[0, 0, 0, 0, 0] = 1.0
    A = A + eps * np.random.default_rng(seed).standard_normal((d, D, D, D, D))
    return A / np.abs(A).max()


def product_state(v, D):
    """A[s, 0, 0, 0, 0] = v[s], all other entries zero (a product state)."""
    v = np.asarray(v, dtype=np.float64)
    A = np.zeros((len(v), D, D, D, D))
    A[:, 0, 0, 0, 0] = v
    return A


def _sym_sqrt(m):
    w, V = np.linalg.eigh(m)
    return (V * np.sqrt(w)) @ V.T


def ising_bond_sqrt(beta):
    """Symmetric M with M M^T = [[e^(b/2), e^(-b/2)], [e^(-b/2), e^(b/2)]]."""
    eb = np.exp(beta / 2.0)
    return _sym_sqrt(np.array([[eb, 1.0 / eb], [1.0 / eb, eb]]))


def ising_peps(beta):
    """Ising PEPS, D = d = 2: A[s,u,l,d,r] = M[s,u] M[s,l] M[s,d] M[s,r].

    Its norm network is the partition function of the 2D classical Ising
    model at inverse temperature beta (J = 1); s = 0 is spin up.
    """
    M = ising_bond_sqrt(beta)
    return np.einsum("su,sl,sd,sr->suldr", M, M, M, M)


def ising_up_boundary(beta):
    """Boundary vector b[(u, ub)] = M[0,u] M[0,ub]: spins fixed up outside."""
    M = ising_bond_sqrt(beta)
    return np.outer(M[0], M[0]).reshape(-1)


def ising_classical(beta):
    """Single-layer classical Ising tensor with bond 2.

    a[u,l,d,r] = sum_s Q[s,u] Q[s,l] Q[s,d] Q[s,r], Q Q^T = [[e^b, e^-b], [e^-b, e^b]].
    """
    eb = np.exp(beta)
    Q = _sym_sqrt(np.array([[eb, 1.0 / eb], [1.0 / eb, eb]]))
    return np.einsum("su,sl,sd,sr->uldr", Q, Q, Q, Q)


def heisenberg_bond_matrix():
    """The Heisenberg bond S.S (J = 1) of two spins 1/2 in the basis
    |uu>, |ud>, |du>, |dd>: 1/4 on the aligned states, -1/4 and the exchange
    1/2 on the antialigned pair."""
    return np.array([[0.25, 0.0, 0.0, 0.0],
                     [0.0, -0.25, 0.5, 0.0],
                     [0.0, 0.5, -0.25, 0.0],
                     [0.0, 0.0, 0.0, 0.25]])
