"""HOTRG on the double-layer network, plain and Z2 forms (the coarse-graining
method the paper treats beside CTMRG: Sec. II A; the symmetry probe b of
Sec. III A; the speed-up of Fig. 4(c), (d)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names HOTRG (higher-order tensor renormalisation group) and states
that the Z2 structure of the rotated double layer applies to its steps; the
steps themselves are those of the standard method.  Readings where the paper
is silent:

  H1  A step joins two tensors along the vertical bond: the upper T[u,l1,m,r1]
      and the lower T[m,l2,d,r2] give M[u,l1,l2,d,r1,r2].  The two left legs
      (l1,l2) and the two right legs (r1,r2) are each fused and cut back to
      chi by one isometry U applied to both:
      T'[u,x,d,y] = sum U[(l1 l2),x] M[u,l1,l2,d,r1,r2] U[(r1 r2),y].
  H2  U holds the dominant eigenvectors of the left Gram matrix
      ML = M_L M_L^T (M_L = M as a matrix with rows (l1,l2)) or of the right
      one MR (rows (r1,r2)), whichever discards the smaller weight (the sum
      of the eigenvalues not kept); on a tie the left one.  Both Gram
      matrices have the trace ||M||_F^2; weights within 1e-10 of it count
      as tied (a side that keeps every state discards exactly nothing, which
      rounding must not turn into a preference).
  H3  Kept: min(chi, #{lambda > tau lambda_max}) over the merged spectrum of
      both sectors, ties even sector first (as in the CTMRG truncation).
      Columns of U: even sector first, each by decreasing eigenvalue.
  H4  The new tensor is divided by its Frobenius norm n_j and then rotated by
      a quarter turn, T[u,l,d,r] <- T[r,u,l,d] on the legs, so that the next
      step joins along the other direction.
  H5  After k steps the tensor stands for a torus of 2^k sites:
      ln Z / N = ln n_0 + sum_{j=1..k} ln(n_j) / 2^j + ln(Tr T_k) / 2^k,
      Tr T = sum_{u,l} T[u,l,u,l], n_0 the norm of the initial tensor.
  H7  The energy of a vertical bond: the bond operator h[(s1 s2),(s1' s2')]
      (site 1 above site 2) is written as sum_k c_k O_k (x) O'_k by the SVD of
      h reshuffled to [(s1 s1'), (s2 s2')]; each term puts the impurities
      a[O] = sum_{s s'} O[s,s'] A[s] (x) A[s'] (ket s, bra s') above a[O']
      in the first step, which joins them into one impurity carried like the
      probe.  E = sum_k c_k Z_k / Z.  In the Z2 form each O is split into its
      symmetric (even impurity) and antisymmetric (odd) part; the mixed
      products are odd and contribute nothing.
  H8  The one-site RDM: rho[s,s'] = Z[a(E_ss')] / Z with E_ss' = |s><s'|, each
      impurity carried like the probe; in the Z2 form only the symmetric
      parts (E_ss' + E_s's)/2 are even, so rho is symmetric by construction.
      Divided by its trace.
  H6  The probe: one tensor of the network is replaced by an impurity (b or
      |b|).  In every step the impurity takes the upper place and a pure
      tensor the lower one, with the pure step's U and n_j, so that
      Tr(T^imp_k) / Tr(T_k) = Z_imp / Z.  The symmetry error is
      |Z_b| / Z_|b|.  b, as a D^4 x D^4 matrix between the ket and the bra
      indices (u,l,d,r), is +1 above the diagonal and -1 below; |b| is 1 off
      the diagonal (Sec. III A).

In the Z2 form every tensor is stored dense in the rotated basis with leg
parities; the pure tensors are even, b is odd (it is antisymmetric under the
bra-ket swap), |b| even; parity masks keep only the allowed blocks, and the
Gram matrices are decomposed per sector.
"""
import numpy as np

from . import basis
from .ctmrg import _select


def probe_b(D, absolute=False):
    """The symmetry probe of Sec. III A as a double-layer tensor [U,L,Dn,R]
    (joined index K = k*D + kbar per leg)."""
    n = D ** 4
    i, j = np.indices((n, n))
    B = np.where(i < j, 1.0, np.where(i > j, -1.0, 0.0))
    if absolute:
        B = np.abs(B)
    b = B.reshape((D,) * 8)  # [ku, kl, kd, kr, bu, bl, bd, br]
    q = D * D
    return b.transpose(0, 4, 1, 5, 2, 6, 3, 7).reshape(q, q, q, q)


def _mask_parity(x, pars, tp):
    tot = np.zeros(x.shape, dtype=np.int64)
    for i, p in enumerate(pars):
        shape = [1] * x.ndim
        shape[i] = len(p)
        tot = tot + p.reshape(shape)
    return np.where(tot % 2 == tp, x, 0.0)


def join_vertical(Tu, Tl):
    """M[u,l1,l2,d,r1,r2] = sum_m Tu[u,l1,m,r1] Tl[m,l2,d,r2] (H1)."""
    return np.einsum("uamb,mcde->uacdbe", Tu, Tl)


def isometry(M, chi, tau, ph=None):
    """U of H2/H3 for M[u,l1,l2,d,r1,r2]; returns (U, side, kept per sector,
    spectrum kept (descending, divided by the largest), discarded weight of
    both sides)."""
    Dh1, Dh2 = M.shape[1], M.shape[2]
    n = Dh1 * Dh2
    ML = M.transpose(1, 2, 0, 3, 4, 5).reshape(n, -1)
    MR = M.transpose(4, 5, 0, 1, 2, 3).reshape(n, -1)
    if ph is not None:
        pf = ((ph[:, None] + ph[None, :]) % 2).reshape(-1)
        sectors = [0, 1]
    else:
        pf = np.zeros(n, dtype=np.int64)
        sectors = [0]
    best = None
    errs = []
    for side, Mm in enumerate((ML, MR)):
        G = Mm @ Mm.T
        parts = []
        for P in sectors:
            idx = np.nonzero(pf == P)[0]
            if len(idx) == 0:
                continue
            lam, V = np.linalg.eigh(G[np.ix_(idx, idx)])
            order = np.argsort(-lam, kind="stable")
            parts.append((P, idx, lam[order], V[:, order]))
        lam_all = np.concatenate([p[2] for p in parts])
        sec = np.concatenate([np.full(len(p[2]), p[0]) for p in parts])
        loc = np.concatenate([np.arange(len(p[2])) for p in parts])
        kept = _select(lam_all, sec, chi, tau)
        kept = kept[np.lexsort((loc[kept], sec[kept]))]
        err = float(np.sum(lam_all) - np.sum(lam_all[kept]))
        errs.append(err)
        U = np.zeros((n, len(kept)))
        kcount = [0, 0]
        col = 0
        for (P, idx, lam, V) in parts:
            sel = loc[kept[sec[kept] == P]]
            kcount[P] = len(sel)
            if len(sel):
                U[np.ix_(idx, np.arange(col, col + len(sel)))] = V[:, sel]
            col += len(sel)
        spec = np.sort(lam_all[kept])[::-1]
        cand = (U, side, tuple(kcount), spec / spec[0])
        if best is None or err < errs[0] - 1e-10 * np.sum(lam_all):
            best = cand
    return best + (tuple(errs),)


def contract_step(M, U):
    """T'[u,x,d,y] = sum U[(l1 l2),x] M[u,l1,l2,d,r1,r2] U[(r1 r2),y] (H1)."""
    Dh1, Dh2 = M.shape[1], M.shape[2]
    U3 = U.reshape(Dh1, Dh2, -1)
    return np.einsum("abx,uabdce,cey->uxdy", U3, M, U3, optimize=True)


def rotate_quarter(T):
    """T[u,l,d,r] <- T[r,u,l,d] (H4): the right leg becomes the upper one."""
    return T.transpose(3, 0, 1, 2)


class Run:
    """HOTRG on the double layer of A (or on a given network tensor a), plain
    or Z2 form; optional impurities (H6) carried along."""

    def __init__(self, chi, form="dense", A=None, a=None, tau=1e-12, probes=False, bond=None, rdm1=False):
        if form not in ("dense", "z2"):
            raise ValueError(form)
        self.form, self.chi, self.tau = form, chi, tau
        if a is None:
            a = basis.double_layer(A)
        q = a.shape[0]
        D = int(round(np.sqrt(q)))
        imps = []
        if probes:
            imps = [probe_b(D), probe_b(D, absolute=True)]
        if form == "z2":
            U = basis.hermitian_basis(D)
            p = basis.leg_parity(D)
            a = _mask_parity(basis.rotate(a, U), [p] * 4, 0)
            # b is odd under the swap, |b| even: only those blocks are kept
            imps = [_mask_parity(basis.rotate(x, U), [p] * 4, tp) for x, tp in zip(imps, (1, 0))]
            self.pv = p.copy()
            self.ph = p.copy()
            self.tp = [1, 0][: len(imps)]
        else:
            self.pv = self.ph = None
            self.tp = [0] * len(imps)
        # bond energy (H7): pairs (coefficient, upper, lower) of impurities
        pairs = []
        if bond is not None:
            d = A.shape[0]
            H = np.asarray(bond, dtype=np.float64).reshape(d, d, d, d)  # [s1, s2, s1', s2']
            Hr = H.transpose(0, 2, 1, 3).reshape(d * d, d * d)       # [(s1 s1'), (s2 s2')]
            Uh, sh, Vh = np.linalg.svd(Hr)
            for k in range(len(sh)):
                if sh[k] <= 1e-14 * sh[0]:
                    continue
                O1 = Uh[:, k].reshape(d, d)
                O2 = Vh[k].reshape(d, d)
                if form == "z2":
                    parts = [((O1 + O1.T) / 2, (O2 + O2.T) / 2, 0), ((O1 - O1.T) / 2, (O2 - O2.T) / 2, 1)]
                else:
                    parts = [(O1, O2, 0)]
                for P1, P2, tp in parts:
                    if not (np.abs(P1).max() > 0 and np.abs(P2).max() > 0):
                        continue
                    i1 = np.einsum("st,sabcd,tefgh->aebfcgdh", P1, A, A).reshape(a.shape)
                    i2 = np.einsum("st,sabcd,tefgh->aebfcgdh", P2, A, A).reshape(a.shape)
                    if form == "z2":
                        i1 = _mask_parity(basis.rotate(i1, U), [p] * 4, tp)
                        i2 = _mask_parity(basis.rotate(i2, U), [p] * 4, tp)
                    pairs.append((sh[k], i1, i2))
        # one-site RDM (H8): impurities of E_ss' (plain) or of the symmetric
        # parts (Z2, s <= s'), with their places in rho
        self.rdm_places = []
        if rdm1:
            d = A.shape[0]
            for s1 in range(d):
                for s2 in range(d):
                    if form == "z2" and s2 < s1:
                        continue
                    E = np.zeros((d, d))
                    E[s1, s2] = 1.0
                    if form == "z2":
                        E = 0.5 * (E + E.T)
                    x = np.einsum("st,sabcd,tefgh->aebfcgdh", E, A, A).reshape(a.shape)
                    if form == "z2":
                        x = _mask_parity(basis.rotate(x, U), [p] * 4, 0)
                    imps.append(x)
                    self.tp.append(0)
                    self.rdm_places.append((s1, s2))
        n0 = np.linalg.norm(a)
        self.T = a / n0
        self.imps = [x / n0 for x in imps]
        self.pairs = [(c, x / n0, y / n0) for c, x, y in pairs]
        self.bond_imps = []  # joined pairs after the first step
        self.log_norms = [np.log(n0)]
        self.records = []
        self.steps = 0

    def step(self, n=1):
        z2 = self.form == "z2"
        for _ in range(n):
            M = join_vertical(self.T, self.T)
            U, side, kept, spec, errs = isometry(M, self.chi, self.tau, self.ph if z2 else None)
            Tn = contract_step(M, U)
            imps = [contract_step(join_vertical(x, self.T), U) for x in self.imps]
            if self.steps == 0:
                bimps = [contract_step(join_vertical(x, y), U) for _, x, y in self.pairs]
            else:
                bimps = [contract_step(join_vertical(x, self.T), U) for x in self.bond_imps]
            if z2:
                newp = np.array([0] * kept[0] + [1] * kept[1], dtype=np.int64)
                Tn = _mask_parity(Tn, [self.pv, newp, self.pv, newp], 0)
                imps = [_mask_parity(x, [self.pv, newp, self.pv, newp], tp) for x, tp in zip(imps, self.tp)]
                bimps = [_mask_parity(x, [self.pv, newp, self.pv, newp], 0) for x in bimps]
                # after the quarter turn the new bond is vertical
                self.pv, self.ph = newp, self.pv
            nj = np.linalg.norm(Tn)
            self.T = rotate_quarter(Tn / nj)
            self.imps = [rotate_quarter(x / nj) for x in imps]
            self.bond_imps = [rotate_quarter(x / nj) for x in bimps]
            self.log_norms.append(np.log(nj))
            self.records.append({"kept": kept if z2 else (sum(kept), 0), "side": side, "spectrum": spec,
                                 "discarded": errs})
            self.steps += 1
        return self

    def trace(self, T=None):
        T = self.T if T is None else T
        return float(np.einsum("ulul->", T))

    def log_z(self):
        """ln Z per site of the torus of 2^k sites (H5)."""
        k = self.steps
        s = sum(ln / 2.0 ** j for j, ln in enumerate(self.log_norms))
        return s + np.log(self.trace()) / 2.0 ** k

    def impurity_ratios(self):
        """Z_imp / Z for the carried impurities (H6)."""
        t = self.trace()
        return [self.trace(x) / t for x in self.imps]

    def energy(self):
        """<h> on a vertical bond (H7); needs at least one step."""
        t = self.trace()
        return sum(c * self.trace(x) / t for (c, _, _), x in zip(self.pairs, self.bond_imps))

    def sym_error(self):
        """|Z_b| / Z_|b| (H6, Sec. III A)."""
        rb, rab = self.impurity_ratios()[:2]
        return abs(rb) / abs(rab)

    def rho1(self):
        """One-site RDM (H8), trace one."""
        ratios = self.impurity_ratios()[len(self.imps) - len(self.rdm_places):]
        d = 1 + max(max(pl) for pl in self.rdm_places)
        rho = np.zeros((d, d))
        for (s1, s2), r in zip(self.rdm_places, ratios):
            rho[s1, s2] = r
            if self.form == "z2":
                rho[s2, s1] = r
        return rho / np.trace(rho)
