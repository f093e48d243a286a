"""Complex iPEPS in the real representation of Sec. II C (the q leg and f).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a complex tensor A the double layer a = sum_s A[s] (x) conj(A[s]) is not
swap invariant, but in the eigenbasis of the swap S its blocks of even total
parity are real and those of odd total parity are imaginary (Sec. II C).
Every tensor b of the contraction keeps that structure; it is stored as the
real tensor bt with one extra leg q of dimension 2, bt[..., 0] = Re b (even
total parity) and bt[..., 1] = Im b (odd total parity), and two such tensors
are multiplied by contracting their q legs with the tensor f of the complex
multiplication rule, f[0,0,0] = 1, f[1,1,0] = -1, f[0,1,1] = f[1,0,1] = 1:
c~[.., r] = sum b~[.., p] b~[.., q] f[p, q, r].  The q leg times [1, i]
gives the complex tensor back.

The directional CTMRG move is that of oracle/ctmrg.py (its readings hold)
with every product taken this way.  Readings for the truncation, where the
paper names the representation but not the decomposition:
  * M = H_d H_u is decomposed through the real R = D^-1 M D with
    D = diag(i^p), p the parity of each index of the cut: R holds M's real
    (even-total) blocks and the imaginary parts of its odd-total blocks, the
    block (even row, odd column) negated.  R = U S V^T gives
    M = (D U) S (D V)^dagger: the same singular values, and singular vectors
    D U, D V with real entries on even and imaginary entries on odd indices,
    i.e. every new bond state is even;
  * kept states as in the real case: min(chi, #{s > tau s_max}) over the one
    spectrum of R (it couples the sectors);
  * P_a = H_u (D V) S^-1/2, P_b = S^-1/2 (D U)^dagger H_d, in the
    representation (D V)~[j, k, p_j] = V[j, k] and
    (D U)^dagger~[k, i, p_i] = (-1)^p_i U[i, k];
  * Frobenius normalisation over both parts.
Observables are taken from the environment converted back to complex numbers
and to the plain basis, with the functions of oracle/ctmrg.py.
"""
import numpy as np

from . import basis, ctmrg

# f[p, q, r]: the product of parts p and q lands in part r with this sign
F = np.zeros((2, 2, 2))
F[0, 0, 0] = 1.0
F[1, 1, 0] = -1.0
F[0, 1, 1] = 1.0
F[1, 0, 1] = 1.0


def bmul(X, Y, ax_x, ax_y):
    """c~ = sum over the listed legs (and the q legs through f) of X~ Y~.

    X and Y carry their q leg last; the result has X's free legs, then Y's,
    then its q leg."""
    fx = X.ndim - len(ax_x)  # free legs of X including q
    Z = np.tensordot(X, Y, (ax_x, ax_y))
    return np.tensordot(Z, F, ([fx - 1, Z.ndim - 1], [0, 1]))


def tp(X, *perm):
    """Transpose the ordinary legs, keeping q last."""
    return X.transpose(list(perm) + [X.ndim - 1])


def to_rep(c, pars, tol=1e-13):
    """Real representation of a structured complex tensor; the parts that the
    structure says vanish (imaginary even-total, real odd-total entries) must
    be below tol relative to the largest entry."""
    even = basis.parity_mask(pars)
    scale = max(np.abs(c).max(), 1e-300)
    assert np.abs(np.where(even, c.imag, 0.0)).max() <= tol * scale, "imaginary even-total entries"
    assert np.abs(np.where(even, 0.0, c.real)).max() <= tol * scale, "real odd-total entries"
    return np.stack([np.where(even, c.real, 0.0), np.where(even, 0.0, c.imag)], axis=-1)


def from_rep(bt):
    """The q leg times [1, i]."""
    return bt[..., 0] + 1j * bt[..., 1]


def _fro(x):
    return x / np.linalg.norm(x)


def quadrants(t, at):
    """ctmrg.quadrants with structured products (q legs last)."""
    C1, T1, C2, T2, C3, T3, C4, T4 = t
    y = bmul(T4, bmul(C1, T1, [1], [0]), [2], [0])               # [w,l,u,t]
    Q1 = tp(bmul(y, at, [2, 1], [0, 1]), 0, 2, 1, 3)              # [w,d,t,r]
    y = bmul(bmul(T1, C2, [2], [0]), T2, [2], [0])               # [t,u,r,e]
    Q2 = tp(bmul(y, at, [1, 2], [0, 3]), 0, 2, 1, 3)              # [t,l,e,d]
    y = bmul(bmul(T2, C3, [2], [0]), T3, [2], [0])               # [e,r,d,m]
    Q3 = tp(bmul(y, at, [1, 2], [3, 2]), 0, 2, 1, 3)              # [e,u,m,l]
    y = bmul(bmul(T3, C4, [2], [0]), T4, [2], [0])               # [m,d,l,w]
    Q4 = tp(bmul(y, at, [1, 2], [2, 1]), 0, 3, 1, 2)              # [m,r,w,u]
    return Q1, Q2, Q3, Q4


def _mat(Q):
    s = Q.shape
    return Q.reshape(s[0] * s[1], s[2] * s[3], 2)


def cut_projectors(Q1, Q2, Q3, Q4, chi, tau, pW, pE):
    """Projectors of one cut (see the module docstring); pW, pE: parities of
    the indices of the west and east cuts."""
    chiW, q = Q1.shape[0], Q1.shape[1]
    m1, m2, m3, m4 = (_mat(Q) for Q in (Q1, Q2, Q3, Q4))
    Hu = bmul(m1, m2, [1], [0])   # [W, E]
    Hd = bmul(m3, m4, [1], [0])   # [E, W]
    M = bmul(Hd, Hu, [1], [0])    # [E, E]
    R = M[..., 0] + M[..., 1]
    R = np.where((pE[:, None] == 0) & (pE[None, :] == 1), -R, R)
    Ur, s, Vt = np.linalg.svd(R)
    kept = ctmrg._select(s, np.zeros(len(s), dtype=np.int64), chi, tau)
    kept = np.sort(kept)
    k = len(kept)
    isq = 1.0 / np.sqrt(s[kept])
    V = Vt[kept].T                # [E, k]
    U = Ur[:, kept]               # [E, k]
    Vc = np.zeros(V.shape + (2,))
    Vc[pE == 0, :, 0] = V[pE == 0]
    Vc[pE == 1, :, 1] = V[pE == 1]
    WH = np.zeros((k, len(pE), 2))
    WH[:, pE == 0, 0] = U[pE == 0].T
    WH[:, pE == 1, 1] = -U[pE == 1].T
    Pa = bmul(Hu, Vc, [1], [0]) * isq[None, :, None]     # [W, k]
    Pb = bmul(WH, Hd, [1], [0]) * isq[:, None, None]     # [k, W]
    spec = s / s[0]
    return Pa.reshape(chiW, q, k, 2), Pb.reshape(k, chiW, q, 2), {"spectrum": spec, "kept": (k, 0)}


def left_move(env, at, chi, tau, par_q):
    """One left move (C1, T4, C4 replaced), as ctmrg.left_move."""
    top, right, bottom, left = env.par
    Q1, Q2, Q3, Q4 = quadrants(env.t, at)
    pW = ((left[:, None] + par_q[None, :]) % 2).reshape(-1)
    pE = ((right[:, None] + par_q[None, :]) % 2).reshape(-1)
    Pa, Pb, rec = cut_projectors(Q1, Q2, Q3, Q4, chi, tau, pW, pE)
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    # C1'[k,r] = Pb[k,(c,u)] C1[c,x] T1[x,u,r]
    env.t[0] = _fro(bmul(Pb, bmul(C1, T1, [1], [0]), [1, 2], [0, 1]))
    # T4'[i,r,j] = Pa[(c,u),j] T4[w,l,c] a[u,l,e,r] Pb[i,(w,e)]
    z = bmul(bmul(T4, Pa, [2], [0]), at, [1, 2], [1, 0])        # [w,j,e,r]
    env.t[7] = _fro(tp(bmul(Pb, z, [1, 2], [0, 2]), 0, 2, 1))  # [i,j,r] -> [i,r,j]
    # C4'[r,j] = T3[r,u,x] C4[x,c] Pa[(c,u),j]
    env.t[6] = _fro(bmul(bmul(T3, C4, [2], [0]), Pa, [2, 1], [0, 1]))
    env.par[3] = np.zeros(rec["kept"][0], dtype=np.int64)     # every new state even
    return rec


class Run:
    """Directional CTMRG of a complex tensor A (d, D, D, D, D) in the real
    representation; the same outputs as ctmrg.Run(form="dense") on complex A."""

    def __init__(self, chi, A, tau=1e-12):
        self.chi, self.tau, self.A = chi, tau, np.asarray(A, dtype=np.complex128)
        D = self.A.shape[1]
        self.U = basis.hermitian_basis(D)
        self.par_q = basis.leg_parity(D)
        self.a_plain = basis.double_layer(self.A)
        self.at = to_rep(basis.rotate(self.a_plain, self.U), [self.par_q] * 4)
        b = self.U @ np.eye(D).reshape(-1)           # the traced boundary, even and real
        bt = to_rep(b.astype(np.complex128), [self.par_q])
        td = lambda X, Y, ax, ay: bmul(X, Y, ax, ay)
        at = self.at
        # initial environment: the boundary legs of the 3x3 patch traced with b
        C1 = td(bt, td(bt, at, [0], [0]), [0], [0])                          # [Dn,R]   (u, l traced)
        T1 = td(bt, at, [0], [0])                                            # [L,Dn,R]
        C2 = td(bt, tp(td(bt, at, [0], [0]), 2, 0, 1), [0], [0])            # r, u traced -> [L,Dn]
        T2 = tp(td(bt, at, [0], [3]), 0, 1, 2)                              # [U,L,Dn]
        C3 = td(bt, td(bt, at, [0], [2]), [0], [2])                         # d, r traced -> [U,L]
        T3 = tp(td(bt, at, [0], [2]), 2, 0, 1)                              # [R,U,L]
        C4 = tp(td(bt, td(bt, at, [0], [1]), [0], [1]), 1, 0)               # l, d traced -> [R,U]
        T4 = tp(td(bt, at, [0], [1]), 1, 2, 0)                              # [Dn,R,U]
        self.env = ctmrg.Env([_fro(x) for x in (C1, T1, C2, T2, C3, T3, C4, T4)],
                             [self.par_q.copy() for _ in range(4)])
        self.records, self.deltas = [], []
        self._spec = self.corner_spectra()

    def corner_spectra(self):
        return ctmrg.corner_spectra(ctmrg.Env([from_rep(x) for x in self.env.t]), self.chi)

    def step(self, n=1):
        for _ in range(n):
            for dname, r in ctmrg.MOVE_ROTATIONS:
                env_r = self.env.rotated(r)
                at_r = self.at
                for _ in range(r % 4):
                    at_r = tp(at_r, 3, 0, 1, 2)
                rec = left_move(env_r, at_r, self.chi, self.tau, self.par_q)
                self.env.store_rotated(env_r, r)
                rec["move"] = dname
                self.records.append(rec)
            new = self.corner_spectra()
            self.deltas.append(ctmrg.spectra_delta(self._spec, new))
            self._spec = new
        return self

    def plain(self):
        """The environment as complex tensors in the plain basis (the q leg
        times [1, i], then U^T on the edge tensors' double-layer legs)."""
        t = [from_rep(x) for x in self.env.t]
        U = self.U
        for i, eq in ((1, "lar,ab->lbr"), (3, "uad,ab->ubd"), (5, "rau,ab->rbu"), (7, "dau,ab->dbu")):
            t[i] = np.einsum(eq, t[i], U)
        return ctmrg.Env(t)

    def epsilon(self):
        eps = ctmrg.epsilon_of(self.plain())
        return eps / np.sum(eps * self.a_plain)

    def rho1(self):
        return ctmrg.rho1_of(self.epsilon(), self.A)

    def rho2(self, direction="h"):
        r = 0 if direction == "h" else 1
        return ctmrg.rho2_h_of(self.plain().rotated(r), ctmrg.rot_A(self.A, r))

    def energy(self, h=None):
        h = ctmrg.heisenberg_bond() if h is None else h
        return float(np.real(np.trace(self.rho2("h") @ h) + np.trace(self.rho2("v") @ h)))

    def s_err(self):
        return ctmrg.s_err_of(self.epsilon())
