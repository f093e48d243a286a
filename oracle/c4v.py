"""C4v-symmetric CTMRG, plain and Z2 forms (paper Sec. II A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a tensor invariant under the rotations and reflections of the square
lattice the paper's CTMRG keeps one corner C and one edge T: the environment
of every site has C1 = C2 = C3 = C4 = C and T1 = T2 = T3 = T4 = T, each in its
own leg convention (counter-clockwise, as in ctmrg).  One iteration:

  * the enlarged corner Q = C T T a, a symmetric matrix between its two cuts
    (the chi leg and the q leg of each cut);
  * its eigendecomposition, per parity sector in the Z2 form (Q is block
    diagonal there, Sec. II B), keeping the chi eigenvalues of largest modulus
    over the merged spectrum (same cutoff and ties as the directional
    truncation, on |lambda|); P = their eigenvectors;
  * C' = P^T Q P (diagonal: the kept eigenvalues), T' = P^T (T a) P;
  * both divided by their Frobenius norm.

The eigendecomposition is that of the symmetrised block (Q + Q^T) / 2: the
enlarged corner of a C4v-symmetric network is symmetric up to rounding.
"""
import numpy as np

from . import ctmrg


def c4v_symmetrize(A):
    """Mean of A[s,u,l,d,r] over the eight symmetries of the square (the four
    rotations, each with and without the left-right reflection)."""
    out = np.zeros_like(A)
    for refl in (False, True):
        B = A.transpose(0, 1, 4, 3, 2) if refl else A  # swap left and right
        for r in range(4):
            out += ctmrg.rot_A(B, r)
    return out / 8.0


def is_c4v(A, tol=1e-14):
    return all(np.abs(ctmrg.rot_A(A, r) - A).max() <= tol for r in range(4)) and \
        np.abs(A.transpose(0, 1, 4, 3, 2) - A).max() <= tol


def c4v_move(env, a, chi, tau=1e-12, par_q=None):
    """One C4v iteration in place; returns the record (spectrum of |lambda|
    merged and divided by the largest, kept sector sizes)."""
    z2 = env.par is not None
    Q1 = ctmrg.quadrants(env, a)[0]  # [w, d, t, r]: rows (T4's lower leg, a's down), cols (T1's right leg, a's right)
    chiW, q = Q1.shape[0], Q1.shape[1]
    n = chiW * q
    M = Q1.reshape(n, n)
    if z2:
        left = env.par[3]
        prow = ((left[:, None] + par_q[None, :]) % 2).reshape(-1)
        sectors = [0, 1]
    else:
        prow = np.zeros(n, dtype=np.int64)
        sectors = [0]
    parts = []
    for P in sectors:
        idx = np.nonzero(prow == P)[0]
        if len(idx) == 0:
            continue
        Ms = M[np.ix_(idx, idx)]
        lam, U = np.linalg.eigh(0.5 * (Ms + Ms.T))
        order = np.argsort(-np.abs(lam), kind="stable")  # by modulus, descending
        parts.append((P, idx, lam[order], U[:, order]))
    svals = np.concatenate([np.abs(p[2]) for p in parts])
    sec = np.concatenate([np.full(len(p[2]), p[0]) for p in parts])
    loc = np.concatenate([np.arange(len(p[2])) for p in parts])
    kept = ctmrg._select(svals, sec, chi, tau)
    kept = kept[np.lexsort((loc[kept], sec[kept]))]  # even sector first, then by modulus
    k = len(kept)
    Pm = np.zeros((n, k))
    kcount = [0, 0]
    col = 0
    for (P, idx, lam, U) in parts:
        sel = loc[kept[sec[kept] == P]]
        kP = len(sel)
        kcount[P] = kP
        if kP:
            Pm[np.ix_(idx, np.arange(col, col + kP))] = U[:, sel]
        col += kP
    Cn = Pm.T @ M @ Pm
    P3 = Pm.reshape(chiW, q, k)
    T4 = env.t[7]
    Tn = ctmrg.absorb_t4(P3, T4, a, P3.transpose(2, 0, 1))  # [k_down, r, k_up]
    Cn = ctmrg._fro_normalise(Cn)
    Tn = ctmrg._fro_normalise(Tn)
    if z2:
        newpar = np.array([0] * kcount[0] + [1] * kcount[1], dtype=np.int64)
        Cn = ctmrg._mask(Cn, [newpar, newpar])
        Tn = ctmrg._mask(Tn, [newpar, par_q, newpar])
        env.par = [newpar.copy() for _ in range(4)]
    env.t = [Cn, Tn] * 4
    order = np.argsort(-svals)
    rec = {"spectrum": svals[order] / svals[order[0]], "kept": (kcount[0], kcount[1]) if z2 else (k, 0)}
    return rec


class C4vRun(ctmrg.Run):
    """C4v CTMRG on a C4v-symmetric tensor (plain or Z2 form); observables as
    in ctmrg.Run."""

    def __init__(self, chi, form="dense", A=None, a=None, boundary=None, tau=1e-12):
        super().__init__(chi, form, A=A, a=a, boundary=boundary, tau=tau)

    def step(self, n=1):
        for _ in range(n):
            rec = c4v_move(self.env, self.a, self.chi, self.tau, self.par_q)
            rec["iteration"] = self.iterations
            self.records.append(rec)
            self.iterations += 1
            new = ctmrg.corner_spectra(self.env, self.chi)
            self.deltas.append(ctmrg.spectra_delta(self._spec, new))
            self._spec = new
        return self
