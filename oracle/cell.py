"""Directional CTMRG on an Lx x Ly unit cell, plain and Z2 forms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper treats a one-site translation-invariant network; a unit cell of
Lx x Ly different tensors A(x, y) (x to the right, y downwards, periodic) is
the usual extension of directional CTMRG and is read here as follows:

  * every site carries its own eight environment tensors C1..C4, T1..T4
    (legs as in `ctmrg`), C1(x, y) being the corner up-left of site (x, y),
    T1(x, y) the edge above it, and so on counter-clockwise;
  * the initial environment of site (x, y) is its 3x3 patch with the outer
    legs traced with b: C1(x, y) comes from a(x-1, y-1), T1(x, y) from
    a(x, y-1), ..., T4(x, y) from a(x-1, y);
  * a move in frame r (left 0, top 1, right 2, bottom 3, as in `ctmrg`) sweeps
    the frame columns X = 0 .. LX-1 in turn.  At column X, for every frame row
    Y, the cut between rows Y and Y+1 left of the column gets its projector
    pair from the four enlarged corners of the 2x2 block of sites with
    top-left (X, Y): Q1 at (X, Y), Q2 at (X+1, Y), Q3 at (X+1, Y+1), Q4 at
    (X, Y+1) (`ctmrg.cut_projectors`).  Once all rows have their pair, the
    left environment of column X+1 is replaced:
        C1(X+1, Y) = P_b(Y-1) C1(X, Y) T1(X, Y)
        T4(X+1, Y) = P_a(Y-1) T4(X, Y) a(X, Y) P_b(Y)
        C4(X+1, Y) = T3(X, Y) C4(X, Y) P_a(Y)
    each divided by its Frobenius norm;
  * frame coordinates map to the cell by the quarter turns of `ctmrg`
    (`site_of`); with Lx = Ly = 1 everything reduces to `ctmrg.Run`.

In the Z2 form every leg of every environment tensor carries its own parity
vector, since on a unit cell the two legs of an edge tensor can belong to
different bonds.
"""
import numpy as np

from . import basis
from .ctmrg import (_fro_normalise, _mask, absorb_c1, absorb_c4, absorb_t4, corner_spectra, cut_projectors,
                    epsilon_of, heisenberg_bond, initial_environment, quadrants, rho1_of, rho2_h_of, rot_A, rot_a,
                    s_err_of, spectra_delta, Env)

# neighbour of site (x, y) whose traced double layer gives the initial slot i
INIT_OFFSET = [(-1, -1), (0, -1), (1, -1), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0)]
MOVES = (("L", 0), ("R", 2), ("T", 1), ("B", 3))


def to_cell(r, X, Y):
    """Unwrapped cell coordinates of frame-r coordinates (X, Y).

    Frame r is the lattice turned r quarter turns so that the old right leg
    is the new up leg: its right is the cell's direction (3 - r) mod 4 and its
    down the direction (2 - r) mod 4 (0 up, 1 left, 2 down, 3 right).
    """
    r %= 4
    if r == 0:
        return X, Y
    if r == 1:
        return -Y, X
    if r == 2:
        return -X, -Y
    return Y, -X


def frame_dims(Lx, Ly, r):
    return (Lx, Ly) if r % 2 == 0 else (Ly, Lx)


class CellRun:
    """State of one CTMRG solve on an Lx x Ly cell (plain or Z2 form).

    tensors: dict (x, y) -> A(x, y) of shape (d, D, D, D, D), legs [s,u,l,d,r].
    """

    def __init__(self, chi, form, tensors, Lx, Ly, boundary=None, tau=1e-12):
        if form not in ("dense", "z2"):
            raise ValueError(form)
        self.form, self.chi, self.tau, self.Lx, self.Ly = form, chi, tau, Lx, Ly
        self.sites = [(x, y) for y in range(Ly) for x in range(Lx)]
        self.A = {s: np.asarray(tensors[s], dtype=np.float64) for s in self.sites}
        self.a_plain = {s: basis.double_layer(self.A[s]) for s in self.sites}
        q = self.a_plain[(0, 0)].shape[0]
        D = int(round(np.sqrt(q)))
        if form == "z2":
            self.U = basis.hermitian_basis(D)
            self.par_q = basis.leg_parity(D)
            self.a = {s: _mask(basis.rotate(self.a_plain[s], self.U), [self.par_q] * 4) for s in self.sites}
        else:
            self.U = None
            self.par_q = None
            self.a = dict(self.a_plain)
        if boundary is None:
            boundary = np.eye(D).reshape(-1)
        b = np.asarray(boundary, dtype=np.float64)
        if form == "z2":
            b = self.U @ b
        # environments: 8 tensors per site and (Z2) one parity vector per leg
        self.t = {}
        self.lp = {}
        pq = self.par_q
        for s in self.sites:
            ts = []
            for i, (dx, dy) in enumerate(INIT_OFFSET):
                nb = self.wrap(s[0] + dx, s[1] + dy)
                ts.append(initial_environment(self.a[nb], b, pq).t[i])
            self.t[s] = ts
            if form == "z2":
                self.lp[s] = [[pq.copy() for _ in range(2 if i % 2 == 0 else 3)] for i in range(8)]
        self.records = []
        self.deltas = []
        self.iterations = 0
        self._spec = self.corner_spectra()

    def wrap(self, x, y):
        return (x % self.Lx, y % self.Ly)

    def site_of(self, r, X, Y):
        return self.wrap(*to_cell(r, X, Y))

    # ---------------------------------------------------------- moves ----
    def _frame_env(self, s, r):
        return Env([self.t[s][(i + 2 * r) % 8] for i in range(8)])

    def _frame_lp(self, s, r):
        return [self.lp[s][(i + 2 * r) % 8] for i in range(8)]

    def move(self, r):
        """Sweep the frame-r columns once (a left move of frame r)."""
        LX, LY = frame_dims(self.Lx, self.Ly, r)
        z2 = self.form == "z2"
        pq = self.par_q
        for X in range(LX):
            proj = []
            for Y in range(LY):
                s1, s2 = self.site_of(r, X, Y), self.site_of(r, X + 1, Y)
                s3, s4 = self.site_of(r, X + 1, Y + 1), self.site_of(r, X, Y + 1)
                Q1 = quadrants(self._frame_env(s1, r), rot_a(self.a[s1], r))[0]
                Q2 = quadrants(self._frame_env(s2, r), rot_a(self.a[s2], r))[1]
                Q3 = quadrants(self._frame_env(s3, r), rot_a(self.a[s3], r))[2]
                Q4 = quadrants(self._frame_env(s4, r), rot_a(self.a[s4], r))[3]
                pars = None
                if z2:
                    l1, l2, l3, l4 = (self._frame_lp(s, r) for s in (s1, s2, s3, s4))
                    # the two ends of every cut are the same bond
                    for u, v in ((l1[7][0], l4[7][2]), (l1[1][2], l2[1][0]), (l2[3][2], l3[3][0]),
                                 (l3[5][2], l4[5][0])):
                        assert np.array_equal(u, v), "inconsistent bond parities"
                    pars = [((p[:, None] + pq[None, :]) % 2).reshape(-1)
                            for p in (l1[7][0], l1[1][2], l2[3][2], l3[5][2])]
                Pa3, Pb3, kc, rec = cut_projectors(Q1, Q2, Q3, Q4, self.chi, self.tau, pars)
                rec.update(frame=r, column=X, row=Y)
                self.records.append(rec)
                newpar = np.array([0] * kc[0] + [1] * kc[1], dtype=np.int64) if z2 else None
                proj.append((Pa3, Pb3, newpar))
            updates = []
            for Y in range(LY):
                s, t = self.site_of(r, X, Y), self.site_of(r, X + 1, Y)
                e = self._frame_env(s, r).t
                Pa_up, Pb_up, np_up = proj[(Y - 1) % LY]
                Pa_dn, Pb_dn, np_dn = proj[Y]
                c1 = _fro_normalise(absorb_c1(Pb_up, e[0], e[1]))
                t4 = _fro_normalise(absorb_t4(Pa_up, e[7], rot_a(self.a[s], r), Pb_dn))
                c4 = _fro_normalise(absorb_c4(e[5], e[6], Pa_dn))
                lps = None
                if z2:
                    ls = self._frame_lp(s, r)
                    lps = ([np_up, ls[1][2]], [np_dn, pq, np_up], [ls[5][0], np_dn])
                    c1 = _mask(c1, lps[0])
                    t4 = _mask(t4, lps[1])
                    c4 = _mask(c4, lps[2])
                updates.append((t, (c1, t4, c4), lps))
            for t, (c1, t4, c4), lps in updates:
                for i, x, j in ((0, c1, 0), (7, t4, 1), (6, c4, 2)):
                    slot = (i + 2 * r) % 8
                    self.t[t][slot] = x
                    if z2:
                        self.lp[t][slot] = lps[j]

    def step(self, n=1):
        for _ in range(n):
            for _name, r in MOVES:
                self.move(r)
            self.iterations += 1
            new = self.corner_spectra()
            self.deltas.append(spectra_delta(self._spec, new))
            self._spec = new
        return self

    def corner_spectra(self):
        out = []
        for s in self.sites:
            out += corner_spectra(Env(self.t[s]), self.chi)
        return out

    # ---------------------------------------------------- observables ----
    def plain_env(self, s):
        t = list(self.t[s])
        if self.form == "z2":
            U = self.U
            t[1] = np.einsum("lar,ab->lbr", t[1], U)
            t[3] = np.einsum("uad,ab->ubd", t[3], U)
            t[5] = np.einsum("rau,ab->rbu", t[5], U)
            t[7] = np.einsum("dau,ab->dbu", t[7], U)
        return Env(t)

    def epsilon(self, x, y):
        s = self.wrap(x, y)
        eps = epsilon_of(Env(self.t[s]))
        if self.form == "z2":
            eps = basis.unrotate(eps, self.U)
        return eps / np.sum(eps * self.a_plain[s])

    def rho1(self, x, y):
        rho = rho1_of(self.epsilon(x, y), self.A[self.wrap(x, y)])
        if self.form == "z2":
            rho = 0.5 * (rho + rho.T)
        return rho

    def rho2(self, x, y, direction="h"):
        """Pair (x, y)-(x+1, y) ("h") or (x, y)-(x, y+1) ("v"), first site first."""
        r = 0 if direction == "h" else 1
        s = self.wrap(x, y)
        t = self.wrap(x + 1, y) if r == 0 else self.wrap(x, y + 1)
        rho = rho2_h_of(self.plain_env(s).rotated(r), rot_A(self.A[s], r),
                        self.plain_env(t).rotated(r), rot_A(self.A[t], r))
        if self.form == "z2":
            rho = 0.5 * (rho + rho.T)
        return rho

    def energy(self, h=None):
        """Bond energy per site: the mean over sites of E_h + E_v."""
        if h is None:
            h = heisenberg_bond()
        e = 0.0
        for (x, y) in self.sites:
            e += float(np.trace(self.rho2(x, y, "h") @ h) + np.trace(self.rho2(x, y, "v") @ h))
        return e / len(self.sites)

    def s_err(self):
        return max(s_err_of(self.epsilon(x, y)) for (x, y) in self.sites)
