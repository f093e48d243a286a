"""Directional CTMRG on a 1x1 unit cell, plain and Z2 forms (paper Sec. II).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper contracts the double-layer network with CTMRG (Sec. II A, Fig. 1d):
four corners C and four edges T of boundary dimension chi, grown by absorbing
rows and columns and truncated back to chi with an SVD.  In the Z2 form every
joined bra-ket leg is expressed in the eigenbasis of the swap S (Sec. II B);
then every tensor is block sparse in the parity of its legs, the matrices that
are decomposed are block diagonal and the SVD and truncation run per parity
sector (Sec. II B, advantages (1)-(3)).

Readings where the paper is silent (it simplifies to C4v and gives no move):
  * directional moves in the order left, right, top, bottom, each applied to
    the current environment; one iteration = four moves;
  * half-system projectors: with quadrants Q1..Q4 around the 4x4 patch,
    H_u = Q1 Q2, H_d = Q3 Q4, M = H_d H_u = W S V^T (truncated),
    P_a = H_u V S^-1/2 (attached below a cut), P_b = S^-1/2 W^T H_d (above);
  * kept states: k = min(chi, #{s_i > tau * s_max}), tau = 1e-12, over the
    merged spectrum of both sectors in the Z2 form, ties broken by
    (value descending, even sector first, index ascending);
  * every new C and T is divided by its Frobenius norm;
  * the initial environment traces the boundary legs with a vector b
    (b = sum_k |k k> for a double layer, i.e. the open boundary).

Pins (tests/test_oracle_pins.py, tests/test_oracle_cylinder.py): exact
finite patches, the Ising model's closed forms, product states, one
truncated cut against a dense SVD (Eckart-Young), and converged fixed points
of short-ranged correlated states against infinite cylinders.  Parity
unpinned: the finite-chi fixed point on i.i.d. tensors, for which neither a
closed form nor a fast-converging cylinder exists (at D = 2 a cylinder
bounds it only to 2e-4); it rests on the agreement of the plain and Z2
forms and on the pins above.

Tensor legs (counter-clockwise, sites at (x, y) with y downwards):
  a[u,l,d,r]; C1[d,r] T1[l,d,r] C2[l,d] T2[u,l,d] C3[u,l] T3[r,u,l]
  C4[r,u] T4[d,r,u].  Bond parities (Z2 form) are kept per side of the
  patch in the order [top, right, bottom, left].
"""
import numpy as np

from . import basis

EINSUM = dict(optimize=True)


def rot_a(a, r):
    """Rotate the 4-leg tensor so that the old right leg becomes the up leg, r times."""
    for _ in range(r % 4):
        a = a.transpose(3, 0, 1, 2)
    return a


def rot_A(A, r):
    """Same rotation on the virtual legs of a single-layer tensor [s,u,l,d,r]."""
    for _ in range(r % 4):
        A = A.transpose(0, 4, 1, 2, 3)
    return A


class Env:
    """Eight environment tensors and (Z2 form) the parity of every bond."""

    def __init__(self, tensors, par=None):
        self.t = list(tensors)          # [C1, T1, C2, T2, C3, T3, C4, T4]
        self.par = None if par is None else [np.asarray(p) for p in par]  # [top, right, bottom, left]

    def copy(self):
        return Env([x.copy() for x in self.t], None if self.par is None else [p.copy() for p in self.par])

    def rotated(self, r):
        """View of the same environment in a frame rotated r quarter turns."""
        t = [self.t[(i + 2 * r) % 8] for i in range(8)]
        par = None if self.par is None else [self.par[(j + r) % 4] for j in range(4)]
        return Env(t, par)

    def store_rotated(self, env_r, r):
        for i in range(8):
            self.t[(i + 2 * r) % 8] = env_r.t[i]
        if self.par is not None:
            for j in range(4):
                self.par[(j + r) % 4] = env_r.par[j]


def _fro_normalise(x):
    n = np.linalg.norm(x)
    return x / n


def _mask(x, pars):
    return np.where(basis.parity_mask(pars), x, 0.0)


def initial_environment(a, b, par_q=None):
    """Open-boundary environment: boundary legs of the 3x3 patch traced with b."""
    C1 = np.einsum("u,l,uldr->dr", b, b, a, **EINSUM)
    T1 = np.einsum("u,uldr->ldr", b, a, **EINSUM)
    C2 = np.einsum("u,r,uldr->ld", b, b, a, **EINSUM)
    T2 = np.einsum("r,uldr->uld", b, a, **EINSUM)
    C3 = np.einsum("d,r,uldr->ul", b, b, a, **EINSUM)
    T3 = np.einsum("d,uldr->rul", b, a, **EINSUM)
    C4 = np.einsum("l,d,uldr->ru", b, b, a, **EINSUM)
    T4 = np.einsum("l,uldr->dru", b, a, **EINSUM)
    ts = [_fro_normalise(x) for x in (C1, T1, C2, T2, C3, T3, C4, T4)]
    par = None if par_q is None else [par_q.copy() for _ in range(4)]
    env = Env(ts, par)
    if par is not None:
        _mask_env(env, par_q)
    return env


def _mask_env(env, pq):
    top, right, bottom, left = env.par
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    env.t = [
        _mask(C1, [left, top]), _mask(T1, [top, pq, top]),
        _mask(C2, [top, right]), _mask(T2, [right, pq, right]),
        _mask(C3, [right, bottom]), _mask(T3, [bottom, pq, bottom]),
        _mask(C4, [bottom, left]), _mask(T4, [left, pq, left]),
    ]


def quadrants(env, a):
    """Enlarged corners of the 4x4 patch as 4-leg tensors.

    Q1[W, N], Q2[N, E], Q3[E, S], Q4[S, W]; every cut is (chi leg, q leg) with
    the environment leg first, so that the norm is Tr(Q1 Q2 Q3 Q4).
    """
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    td = np.tensordot
    # Q1[w,d,t,r] = C1[c,x] T1[x,u,t] T4[w,l,c] a[u,l,d,r]
    y = td(T4, td(C1, T1, ([1], [0])), ([2], [0]))            # [w,l,u,t]
    Q1 = td(y, a, ([2, 1], [0, 1])).transpose(0, 2, 1, 3)       # [w,t,d,r] -> [w,d,t,r]
    # Q2[t,l,e,d] = T1[t,u,x] C2[x,y] T2[y,r,e] a[u,l,d,r]
    y = td(td(T1, C2, ([2], [0])), T2, ([2], [0]))             # [t,u,r,e]
    Q2 = td(y, a, ([1, 2], [0, 3])).transpose(0, 2, 1, 3)       # [t,e,l,d] -> [t,l,e,d]
    # Q3[e,u,m,l] = T2[e,r,y] C3[y,x] T3[x,d,m] a[u,l,d,r]
    y = td(td(T2, C3, ([2], [0])), T3, ([2], [0]))             # [e,r,d,m]
    Q3 = td(y, a, ([1, 2], [3, 2])).transpose(0, 2, 1, 3)       # [e,m,u,l] -> [e,u,m,l]
    # Q4[m,r,w,u] = T3[m,d,x] C4[x,y] T4[y,l,w] a[u,l,d,r]
    y = td(td(T3, C4, ([2], [0])), T4, ([2], [0]))             # [m,d,l,w]
    Q4 = td(y, a, ([1, 2], [2, 1])).transpose(0, 3, 1, 2)       # [m,w,u,r] -> [m,r,w,u]
    return Q1, Q2, Q3, Q4


def _as_matrix(Q):
    s = Q.shape
    return Q.reshape(s[0] * s[1], s[2] * s[3])


def _select(svals, sec, chi, tau):
    """Indices (into the merged list) of the kept states, in merge order."""
    order = np.lexsort((np.arange(len(svals)), sec, -svals))
    smax = svals[order[0]]
    nkeep = int(np.sum(svals > tau * smax))
    k = max(1, min(chi, nkeep))
    return order[:k]


def _cut_parities(legpar_w, legpar_n, legpar_e, legpar_s, par_q):
    """Parity of every index of the four cuts (chi leg major, q leg minor)."""
    return [((p[:, None] + par_q[None, :]) % 2).reshape(-1) for p in (legpar_w, legpar_n, legpar_e, legpar_s)]


def cut_projectors(Q1, Q2, Q3, Q4, chi, tau, pars=None):
    """Projector pair for the cut between Q1 (above) and Q4 (below).

    Q1..Q4 are the four enlarged corners around the cut (see `quadrants`);
    pars = [pW, pN, pE, pS] gives the parity of every index of the west,
    north, east and south cuts in the Z2 form (None: one sector).
    Per sector: H_u = Q1 Q2, H_d = Q3 Q4, M = H_d H_u = W S V^T, and over the
    merged spectrum the kept states give P_a = H_u V S^-1/2 (cut x k, taken
    by objects below the cut) and P_b = S^-1/2 W^T H_d (k x cut, above).
    Returns (Pa[chiW, q, k], Pb[k, chiW, q], (k_even, k_odd), record).
    """
    z2 = pars is not None
    chiW, q = Q1.shape[0], Q1.shape[1]
    m1, m2, m3, m4 = (_as_matrix(Q) for Q in (Q1, Q2, Q3, Q4))
    nW = chiW * q
    if z2:
        pW, pN, pE, pS = pars
        sectors = [0, 1]
    else:
        pW = np.zeros(nW, dtype=np.int64)
        pN = np.zeros(m1.shape[1], dtype=np.int64)
        pE = np.zeros(m2.shape[1], dtype=np.int64)
        pS = np.zeros(m3.shape[1], dtype=np.int64)
        sectors = [0]

    # per sector: H_u = Q1 Q2, H_d = Q3 Q4, M = H_d H_u and its SVD
    parts = []
    for P in sectors:
        iW, iN, iE, iS = (np.nonzero(p == P)[0] for p in (pW, pN, pE, pS))
        if len(iW) == 0 or len(iE) == 0:
            continue
        Hu = m1[np.ix_(iW, iN)] @ m2[np.ix_(iN, iE)]
        Hd = m3[np.ix_(iE, iS)] @ m4[np.ix_(iS, iW)]
        M = Hd @ Hu
        Wm, s, Vt = np.linalg.svd(M)
        parts.append((P, iW, Hu, Hd, Wm, s, Vt))

    svals = np.concatenate([p[5] for p in parts])
    sec = np.concatenate([np.full(len(p[5]), p[0]) for p in parts])
    loc = np.concatenate([np.arange(len(p[5])) for p in parts])
    kept = _select(svals, sec, chi, tau)
    # new bond basis: even sector first, each sector by descending value
    kept = kept[np.lexsort((loc[kept], sec[kept]))]
    knew = len(kept)
    Pa = np.zeros((nW, knew), dtype=m1.dtype)
    Pb = np.zeros((knew, nW), dtype=m1.dtype)
    kcount = [0, 0]
    col = 0
    for (P, iW, Hu, Hd, Wm, s, Vt) in parts:
        idx = loc[kept[sec[kept] == P]]
        kP = len(idx)
        kcount[P] = kP
        if kP == 0:
            continue
        isq = 1.0 / np.sqrt(s[idx])
        # M = W S V^dagger: P_a = H_u V S^-1/2, P_b = S^-1/2 W^dagger H_d
        # (for real blocks the conjugates are the blocks themselves)
        Pa[np.ix_(iW, np.arange(col, col + kP))] = (Hu @ np.conj(Vt[idx]).T) * isq[None, :]
        Pb[np.ix_(np.arange(col, col + kP), iW)] = (np.conj(Wm[:, idx]).T @ Hd) * isq[:, None]
        col += kP
    order = np.argsort(-svals)
    spec = svals[order] / svals[order[0]]
    rec = {"spectrum": spec, "kept": (kcount[0], kcount[1]) if z2 else (knew, 0)}
    return Pa.reshape(chiW, q, knew), Pb.reshape(knew, chiW, q), kcount, rec


def absorb_c1(Pb3, C1, T1):
    """C1'[k,r] = Pb[k,(c,u)] C1[c,x] T1[x,u,r]."""
    return np.tensordot(Pb3, np.tensordot(C1, T1, ([1], [0])), ([1, 2], [0, 1]))


def absorb_t4(Pa3, T4, a, Pb3):
    """T4'[i,r,j] = Pa[(c,u),j] T4[w,l,c] a[u,l,e,r] Pb[i,(w,e)]."""
    td = np.tensordot
    z = td(td(T4, Pa3, ([2], [0])), a, ([1, 2], [1, 0]))       # [w,j,e,r]
    return td(Pb3, z, ([1, 2], [0, 2])).transpose(0, 2, 1)      # [i,j,r] -> [i,r,j]


def absorb_c4(T3, C4, Pa3):
    """C4'[r,j] = T3[r,u,x] C4[x,c] Pa[(c,u),j]."""
    return np.tensordot(np.tensordot(T3, C4, ([2], [0])), Pa3, ([2, 1], [0, 1]))


def left_move(env, a, chi, tau=1e-12, par_q=None):
    """One left move on a 1x1 cell (updates C1, T4, C4 in place).

    Returns a record with the merged spectrum of M (descending, divided by its
    largest value) and the kept sector sizes (k_even, k_odd).
    """
    z2 = env.par is not None
    Q1, Q2, Q3, Q4 = quadrants(env, a)
    pars = None
    if z2:
        top, right, bottom, left = env.par
        pars = _cut_parities(left, top, right, bottom, par_q)
    Pa3, Pb3, kcount, rec = cut_projectors(Q1, Q2, Q3, Q4, chi, tau, pars)
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    env.t[0] = _fro_normalise(absorb_c1(Pb3, C1, T1))
    env.t[7] = _fro_normalise(absorb_t4(Pa3, T4, a, Pb3))
    env.t[6] = _fro_normalise(absorb_c4(T3, C4, Pa3))
    if z2:
        newpar = np.array([0] * kcount[0] + [1] * kcount[1], dtype=np.int64)
        env.par[3] = newpar
        env.t[0] = _mask(env.t[0], [newpar, top])
        env.t[7] = _mask(env.t[7], [newpar, par_q, newpar])
        env.t[6] = _mask(env.t[6], [bottom, newpar])
    return rec


# move order of one iteration: left, right, top, bottom as rotations of the frame
MOVE_ROTATIONS = (("L", 0), ("R", 2), ("T", 1), ("B", 3))


def move(env, a, direction, chi, tau=1e-12, par_q=None):
    r = dict(MOVE_ROTATIONS)[direction]
    env_r = env.rotated(r)
    rec = left_move(env_r, rot_a(a, r), chi, tau, par_q)
    env.store_rotated(env_r, r)
    return rec


def corner_spectra(env, chi):
    """Singular values of the four corners, divided by their sum, padded to chi."""
    out = []
    for i in (0, 2, 4, 6):
        s = np.linalg.svd(env.t[i], compute_uv=False)
        s = s / np.sum(s)
        pad = np.zeros(max(chi, len(s)))
        pad[: len(s)] = s
        out.append(pad)
    return out


def spectra_delta(old, new):
    n = max(len(old[0]), len(new[0]))
    d = 0.0
    for so, sn in zip(old, new):
        a = np.zeros(n)
        b = np.zeros(n)
        a[: len(so)] = so
        b[: len(sn)] = sn
        d = max(d, float(np.linalg.norm(a - b)))
    return d


class Run:
    """State of one CTMRG solve on a 1x1 cell (plain or Z2 form)."""

    def __init__(self, chi, form="dense", A=None, a=None, boundary=None, tau=1e-12, env=None):
        if form not in ("dense", "z2"):
            raise ValueError(form)
        self.form = form
        self.chi = chi
        self.tau = tau
        self.A = A
        if a is None:
            a = basis.double_layer(A)
        self.a_plain = a
        q = a.shape[0]
        if form == "z2" and np.iscomplexobj(a):
            raise ValueError("the masked Z2 form holds real tensors only; complex ones: oracle.complex_z2")
        if form == "z2":
            D = int(round(np.sqrt(q)))
            self.U = basis.hermitian_basis(D)
            self.par_q = basis.leg_parity(D)
            at = basis.rotate(a, self.U)
            self.a = _mask(at, [self.par_q] * 4)
        else:
            self.U = None
            self.par_q = None
            self.a = a
        if env is not None:
            self.env = env
        else:
            if boundary is None:
                D = int(round(np.sqrt(q)))
                boundary = np.eye(D).reshape(-1)
            b = np.asarray(boundary, dtype=np.float64)
            if form == "z2":
                b = self.U @ b
            self.env = initial_environment(self.a, b, self.par_q)
        self.records = []
        self.deltas = []
        self.iterations = 0
        self._spec = corner_spectra(self.env, chi)

    def step(self, n=1):
        for _ in range(n):
            for dname, _r in MOVE_ROTATIONS:
                rec = move(self.env, self.a, dname, self.chi, self.tau, self.par_q)
                rec["move"] = dname
                rec["iteration"] = self.iterations
                self.records.append(rec)
            self.iterations += 1
            new = corner_spectra(self.env, self.chi)
            self.deltas.append(spectra_delta(self._spec, new))
            self._spec = new
        return self

    def run(self, max_iter, tol=None):
        for _ in range(max_iter):
            self.step(1)
            if tol is not None and self.deltas[-1] < tol:
                break
        return self

    # ---------------- observables in the plain basis ----------------
    def plain_env(self):
        """Environment with every q leg in the plain (unrotated) basis."""
        if self.form == "dense":
            return self.env
        U = self.U
        t = list(self.env.t)
        t[1] = np.einsum("lar,ab->lbr", t[1], U)
        t[3] = np.einsum("uad,ab->ubd", t[3], U)
        t[5] = np.einsum("rau,ab->rbu", t[5], U)
        t[7] = np.einsum("dau,ab->dbu", t[7], U)
        return Env(t)

    def epsilon(self):
        """One-site environment eps[U,L,Dn,R] in the plain basis, <eps, a> = 1."""
        eps = epsilon_of(self.env)
        if self.form == "z2":
            eps = basis.unrotate(eps, self.U)
        return eps / np.sum(eps * self.a_plain)

    def rho1(self):
        rho = rho1_of(self.epsilon(), self.A)
        if self.form == "z2":
            rho = 0.5 * (rho + np.conj(rho).T)
        return rho

    def rho2(self, direction="h"):
        r = 0 if direction == "h" else 1
        env = self.plain_env().rotated(r)
        rho = rho2_h_of(env, rot_A(self.A, r))
        if self.form == "z2":
            rho = 0.5 * (rho + np.conj(rho).T)
        return rho

    def energy(self, h=None):
        """Tr(rho_h h) + Tr(rho_v h); its real part (the RDMs of a complex
        tensor in the plain form are Hermitian only up to the truncation)."""
        if h is None:
            h = heisenberg_bond()
        return float(np.real(np.trace(self.rho2("h") @ h) + np.trace(self.rho2("v") @ h)))

    def s_err(self):
        return s_err_of(self.epsilon())

    def log_kappa(self):
        return log_kappa_of(self.env, self.a)


def epsilon_of(env):
    """Contract the 3x3 environment with the centre left open (Sec. III A)."""
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    top, bot = _top_bottom(env)
    td = np.tensordot
    left = td(top, T4, ([0], [2]))                 # [u,b,c,l]
    right = td(bot, T2, ([2], [2]))                # [c,d,b,r]
    return td(left, right, ([1, 2], [2, 0]))       # [u,l,d,r]


def _top_bottom(env):
    """top[a,U,b] = C1 T1 C2 (a: C1 down, b: C2 down); bottom[c,D,e] = C4 T3 C3."""
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    td = np.tensordot
    top = td(td(C1, T1, ([1], [0])), C2, ([2], [0]))                     # [a,U,b]
    bot = td(td(C4, T3, ([0], [2])), C3, ([1], [1])).transpose(0, 1, 2)   # [c,D,e]
    return top, bot


def rho1_of(eps, A):
    """rho1[s,s'] = <eps, A[s] (x) conj(A[s'])>, trace one."""
    D = A.shape[1]
    e8 = eps.reshape((D,) * 8)
    rho = np.einsum("aebfcgdh,sabcd,tefgh->st", e8, A, np.conj(A), **EINSUM)
    return rho / np.trace(rho)


def rho2_h_of(env, A, env_r=None, A_r=None):
    """Two-site RDM of a horizontal bond, rho[(s1 s2), (s1' s2')], trace one.

    The left site is A with environment env; the right site is A_r with
    environment env_r (both default to the left ones, the 1x1 cell).
    """
    env_r = env if env_r is None else env_r
    A_r = A if A_r is None else A_r
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    _, R1, R2, U2, R3, U3, _, _ = env_r.t
    d, D = A.shape[0], A.shape[1]

    def split(T, leg):
        sh = list(T.shape)
        sh[leg:leg + 1] = [D, D]
        return T.reshape(sh)

    T1s, T3s, T4s = split(T1, 1), split(T3, 1), split(T4, 1)
    R1s, U2s, U3s = split(R1, 1), split(U2, 1), split(U3, 1)
    # left half: C1 T1 / T4 [site 1] / C4 T3, open towards site 2.
    # ket legs u,l,e,g and bra legs v,m,f,h of site 1; y, z the top and
    # bottom environment bonds that continue to the right half.
    tl = np.einsum("cx,xuvy->cuvy", C1, T1s, **EINSUM)
    lft = np.einsum("plmc,cuvy->plmuvy", T4s, tl, **EINSUM)
    # ket layer A, bra layer conj(A)
    k1 = np.einsum("plmuvy,suleg->pmvyseg", lft, A, **EINSUM)
    k2 = np.einsum("pmvyseg,tvmfh->pysegtfh", k1, np.conj(A), **EINSUM)
    bl = np.einsum("zefx,xp->zefp", T3s, C4, **EINSUM)
    left = np.einsum("pysegtfh,zefp->ysgthz", k2, bl, **EINSUM)
    # right half: T1 C2 / [site 2] T2 / T3 C3; g, h are the ket and bra
    # legs shared by the two sites.
    tr = np.einsum("yuvx,xc->yuvc", R1s, R2, **EINSUM)
    rgt = np.einsum("yuvc,crwp->yuvrwp", tr, U2s, **EINSUM)
    k1 = np.einsum("yuvrwp,suger->yvwpsge", rgt, A_r, **EINSUM)
    k2 = np.einsum("yvwpsge,tvhfw->ypsgethf", k1, np.conj(A_r), **EINSUM)
    br = np.einsum("px,xefz->pefz", R3, U3s, **EINSUM)
    right = np.einsum("ypsgethf,pefz->ysgthz", k2, br, **EINSUM)
    rho = np.einsum("yagbhz,ycgdhz->acbd", left, right, **EINSUM)
    rho = rho.reshape(d * d, d * d)
    return rho / np.trace(rho)


def heisenberg_bond():
    """S.S for two spins 1/2 as a real 4x4 matrix (sigma^y x sigma^y is real)."""
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    sz = np.array([[1.0, 0.0], [0.0, -1.0]])
    syy = np.array([[0, 0, 0, -1.0], [0, 0, 1.0, 0], [0, 1.0, 0, 0], [-1.0, 0, 0, 0]])
    return 0.25 * (np.kron(sx, sx) + syy + np.kron(sz, sz))


def s_err_of(eps):
    """Hermitian symmetry error ||e - e^dag|| / ||e + e^dag|| (Sec. III A).

    e^dag is e with bra and ket swapped on every leg, complex conjugated
    (for real tensors the conjugate is the tensor itself).
    """
    D = int(round(np.sqrt(eps.shape[0])))
    S = basis.swap_matrix(D)
    ed = np.conj(basis.apply_on_all_legs(S, eps))
    return float(np.linalg.norm(eps - ed) / np.linalg.norm(eps + ed))


def log_kappa_of(env, a):
    """ln of the partition function per site, kappa = Z11 Z00 / (Z10 Z01)."""
    C1, T1, C2, T2, C3, T3, C4, T4 = env.t
    z11 = np.sum(epsilon_of(env) * a)
    z00 = np.trace(C1 @ C2 @ C3 @ C4)
    top, bot = _top_bottom(env)
    z10 = np.sum(top * bot)
    # Z01: C1 C2 / T4 T2 / C4 C3 with T4's right leg joined to T2's left leg
    rgt = np.tensordot(np.tensordot(C1 @ C2, T2, ([1], [0])), C3, ([2], [0]))   # [a,R,y]
    lft = np.tensordot(C4, T4, ([1], [0]))                                      # [y,R,a]
    z01 = np.tensordot(rgt, lft, ([0, 1, 2], [2, 1, 0]))
    return float(np.log(abs(z11)) + np.log(abs(z00)) - np.log(abs(z10)) - np.log(abs(z01)))
