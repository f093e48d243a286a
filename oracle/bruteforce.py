"""Exact contraction of small finite open networks by row transfer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A rows x cols patch of 4-leg site tensors t[u,l,d,r] (Fig. 1c) with the
vector b on every outer leg is contracted exactly, one site at a time.  The
transfer state holds one index per column (the bonds between two rows) and
one horizontal bond; its size is q^(cols+1), so this is only for D = 2 and
widths up to about 8.  A site may be left open ("hole"): its four legs then
stay as free indices of the result, which gives the one-site environment of
Sec. III A exactly.
"""
import numpy as np

from . import basis


def contract(rows, cols, site, b, hole=None):
    """Contract the patch.

    site(i, j) -> 4-leg tensor for row i, column j (ignored at the hole).
    hole: (i, j) or None.  Returns a scalar, or the q^4 tensor [u,l,d,r] of
    the open legs at the hole.
    """
    q = len(b)
    state = np.ones(())
    for _ in range(cols):
        state = np.multiply.outer(state, b)
    nopen = 0  # open legs are kept at the front of the state

    for i in range(rows):
        state = np.multiply.outer(state, b)          # left boundary: axis h at the end
        for j in range(cols):
            pos_b = nopen + j
            pos_h = state.ndim - 1
            if hole is not None and (i, j) == hole:
                # u and l become open legs; new down and right legs are fresh
                state = np.moveaxis(state, [pos_b, pos_h], [0, 1])
                nopen += 2
                eye = np.eye(q)
                state = np.multiply.outer(state, eye)  # (... , D_open, b_j)
                state = np.multiply.outer(state, eye)  # (..., D_open, b_j, R_open, h)
                nd = state.ndim
                # move D_open and R_open to the front (after U, L)
                state = np.moveaxis(state, [nd - 4, nd - 2], [2, 3])
                nopen += 2
                # the fresh b_j sits at nd-3 -> after the moves it is at nd-2
                state = np.moveaxis(state, state.ndim - 2, nopen + j)
                continue
            t = site(i, j)
            state = np.tensordot(state, t, axes=([pos_b, pos_h], [0, 1]))
            # result axes: (others..., d, r): put d back at column j, r stays last
            state = np.moveaxis(state, state.ndim - 2, nopen + j)
        state = np.tensordot(state, b, axes=([state.ndim - 1], [0]))  # right boundary
    for j in range(cols):
        state = np.tensordot(state, b, axes=([nopen], [0]))            # bottom boundary
    if hole is not None:
        # open legs were stored as (U, L, D, R)
        return state
    return state[()]  # a scalar (complex for a complex network)


def epsilon(a, b, L):
    """Normalised one-site environment of the centre of an L x L patch."""
    c = L // 2
    eps = contract(L, L, lambda i, j: a, b, hole=(c, c))
    return eps / np.sum(eps * a)


def rdm1(a, A, b, L):
    """rho1[s,s'] of the centre site of an L x L patch, trace one."""
    c = L // 2
    d = A.shape[0]
    imp = lambda s, sp: basis.impurity(A, s, sp)
    rho = np.zeros((d, d), dtype=np.result_type(a, A))
    for s in range(d):
        for sp in range(d):
            t = imp(s, sp)
            rho[s, sp] = contract(L, L, lambda i, j: t if (i, j) == (c, c) else a, b)
    return rho / np.trace(rho)


def rdm2_h(a, A, b, rows, cols):
    """rho2 of the horizontal pair at the centre row, columns c and c+1."""
    ci = rows // 2
    cj = (cols - 1) // 2
    d = A.shape[0]
    imp = lambda s, sp: basis.impurity(A, s, sp)
    rho = np.zeros((d, d, d, d), dtype=np.result_type(a, A))
    for s1 in range(d):
        for s2 in range(d):
            for t1 in range(d):
                for t2 in range(d):
                    x1, x2 = imp(s1, t1), imp(s2, t2)

                    def site(i, j):
                        if (i, j) == (ci, cj):
                            return x1
                        if (i, j) == (ci, cj + 1):
                            return x2
                        return a

                    rho[s1, s2, t1, t2] = contract(rows, cols, site, b)
    rho = rho.reshape(d * d, d * d)
    return rho / np.trace(rho)
