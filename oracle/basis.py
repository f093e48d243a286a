"""Swap operator, Hermitian eigenbasis and double layer (paper Sec. II A-B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions
-----------
* A single-layer iPEPS tensor A has shape (d, D, D, D, D), legs [s, u, l, d, r].
* The double layer joins ket leg k and bra leg kbar into one index of size
  q = D*D, numbered K = k*D + kbar ("ket-major").  The paper lists the D = 2
  basis in another order; this is a relabelling only.
* S swaps bra and ket on one joined leg: S |k kbar> = |kbar k>  (Sec. II B,
  definition of the swap tensor).
* U has the eigenvectors of S as ROWS: first the D states |k k>, then the
  symmetric combinations (|k l> + |l k>)/sqrt2 for k < l (lexicographic),
  these are the even sector (eigenvalue +1); then the antisymmetric
  combinations (|k l> - |l k>)/sqrt2 for k < l, the odd sector (-1).
  Sector sizes follow the paper's count: D + (D^2 - D)/2 and (D^2 - D)/2.
"""
import numpy as np


def sector_dims(D):
    """(dim even, dim odd) of the joined bra-ket leg (Sec. II B)."""
    return D + (D * D - D) // 2, (D * D - D) // 2


def swap_matrix(D):
    """S as a q x q permutation matrix: S[K', K] = 1 iff K=(k,kb), K'=(kb,k)."""
    q = D * D
    S = np.zeros((q, q))
    for k in range(D):
        for kb in range(D):
            S[kb * D + k, k * D + kb] = 1.0
    return S


def hermitian_basis(D):
    """Orthogonal U (rows = eigenvectors of S, even sector first)."""
    q = D * D
    U = np.zeros((q, q))
    r2 = 1.0 / np.sqrt(2.0)
    row = 0
    for k in range(D):
        U[row, k * D + k] = 1.0
        row += 1
    for k in range(D):
        for l in range(k + 1, D):
            U[row, k * D + l] = r2
            U[row, l * D + k] = r2
            row += 1
    for k in range(D):
        for l in range(k + 1, D):
            U[row, k * D + l] = r2
            U[row, l * D + k] = -r2
            row += 1
    return U


def leg_parity(D):
    """Parity (0 even, 1 odd) of each rotated basis state of a joined leg."""
    qe, qo = sector_dims(D)
    return np.array([0] * qe + [1] * qo, dtype=np.int64)


def double_layer(A):
    """a[U,L,Dn,R] = sum_s A[s,u,l,d,r] conj(A[s,ub,lb,db,rb]), U = u*D + ub
    (Fig. 1b: the ket layer A and the bra layer A^dagger).

    For real A the conjugate is A itself (Sec. II B), for complex A (Sec. II C)
    the bra layer is conjugated.
    """
    d, D = A.shape[0], A.shape[1]
    q = D * D
    a = np.einsum("sabcd,sefgh->aebfcgdh", A, np.conj(A), optimize=True)
    return a.reshape(q, q, q, q)


def impurity(A, s, sp):
    """Double layer with fixed physical indices: ket s, bra sp (for RDMs)."""
    D = A.shape[1]
    q = D * D
    x = np.einsum("abcd,efgh->aebfcgdh", A[s], np.conj(A[sp]))
    return x.reshape(q, q, q, q)


def apply_on_all_legs(X, a):
    """Apply the q x q matrix X to every leg of a 4-leg tensor."""
    return np.einsum("ia,jb,kc,ld,abcd->ijkl", X, X, X, X, a, optimize=True)


def rotate(a, U):
    """Tensor in the eigenbasis of S: a~ = (U x U x U x U) a."""
    return apply_on_all_legs(U, a)


def unrotate(at, U):
    """Inverse of `rotate` (U is orthogonal)."""
    return apply_on_all_legs(U.T, at)


def parity_mask(par_legs):
    """Boolean mask of the entries whose leg parities sum to an even number."""
    tot = np.zeros([len(p) for p in par_legs], dtype=np.int64)
    for i, p in enumerate(par_legs):
        shape = [1] * len(par_legs)
        shape[i] = len(p)
        tot = tot + p.reshape(shape)
    return (tot % 2) == 0
