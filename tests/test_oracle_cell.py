"""Pins of the unit-cell oracle (oracle/cell.py).

  * Lx = Ly = 1 reduces to the one-site oracle, which has its own pins;
  * with chi above the bond growth, the initial environment and the first
    column of a sweep in each of the four directions represent finite
    patches of different tensors exactly (brute-force contraction);
  * orthogonal gauge matrices on the bonds of a 2x2 or 3x2 cell change the
    tensors of every site but not the network, so every gauge-invariant
    output must be unchanged -- a neighbour taken from the wrong site breaks
    this at O(1);
  * the plain and Z2 forms agree;
  * four copies of the Ising PEPS reproduce Onsager's and Yang's values on
    every bond and site.
"""
import numpy as np
import pytest

from oracle import basis, bruteforce, ctmrg
from oracle.cell import CellRun, to_cell
from paper_2410_11596_amd import inputs

from test_oracle_pins import ising_nn_corr, yang_m

SEEDS_2x2 = {(0, 0): 10, (1, 0): 11, (0, 1): 12, (1, 1): 13}
# a 3 x 2 cell as well: with an odd width a mirrored frame is not the same
# set of sites, so the frame maps are pinned in full
CELLS = [(2, 2), (3, 2)]


def cell_seeds(Lx, Ly):
    return {(x, y): 10 + x + Lx * y for y in range(Ly) for x in range(Lx)}


def iid_cell(D, seeds=SEEDS_2x2, d=2):
    return {s: inputs.iid_tensor(d, D, k) for s, k in seeds.items()}


# ------------------------------------------------------------ 1 x 1 ----
@pytest.mark.parametrize("form", ["dense", "z2"])
@pytest.mark.parametrize("D,chi,iters", [(2, 16, 6), (3, 20, 2)])
def test_one_site_cell_is_the_one_site_oracle(form, D, chi, iters):
    A = inputs.iid_tensor(2, D, 0)
    run = ctmrg.Run(chi, form, A=A).step(iters)
    cell = CellRun(chi, form, {(0, 0): A}, 1, 1).step(iters)
    assert len(run.records) == len(cell.records)
    for r1, r2 in zip(run.records, cell.records):
        assert r1["kept"] == r2["kept"]
        assert np.abs(r1["spectrum"] - r2["spectrum"]).max() <= 1e-14
    assert np.abs(run.rho1() - cell.rho1(0, 0)).max() <= 1e-14
    for dr in ("h", "v"):
        assert np.abs(run.rho2(dr) - cell.rho2(0, 0, dr)).max() <= 1e-14
    assert abs(run.energy() - cell.energy()) <= 1e-14
    assert np.allclose(run.deltas, cell.deltas, rtol=1e-12, atol=1e-15)


# ------------------------------------------------------- brute force ----
def _patch(cell, frame_cells, site_frame):
    """A rectangular patch given by frame coordinates, in cell orientation.

    frame_cells: iterable of frame-r positions mapped to unwrapped cell
    coordinates; returns (rows, cols, site(i, j), hole (i, j))."""
    xs = [c[0] for c in frame_cells]
    ys = [c[1] for c in frame_cells]
    x0, y0 = min(xs), min(ys)
    rows, cols = max(ys) - y0 + 1, max(xs) - x0 + 1
    assert rows * cols == len(set(frame_cells))
    site = lambda i, j: cell.a_plain[cell.wrap(x0 + j, y0 + i)]
    return rows, cols, site, (site_frame[1] - y0, site_frame[0] - x0)


def _eps_bf(cell, rows, cols, site, hole):
    b = np.eye(int(round(np.sqrt(cell.a_plain[(0, 0)].shape[0])))).reshape(-1)
    eps = bruteforce.contract(rows, cols, site, b, hole=hole)
    return eps / np.sum(eps * site(*hole))


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_initial_cell_environment_is_each_sites_3x3_patch(form):
    cell = CellRun(64, form, iid_cell(2), 2, 2)
    b = np.eye(2).reshape(-1)
    for (x, y) in cell.sites:
        pos = [(x + i, y + j) for i in (-1, 0, 1) for j in (-1, 0, 1)]
        rows, cols, site, hole = _patch(cell, pos, (x, y))
        eps = _eps_bf(cell, rows, cols, site, hole)
        assert np.abs(cell.epsilon(x, y) - eps).max() <= 1e-12 * np.abs(eps).max()
        # two-site RDMs: the halves of two different environments join into
        # a 3 x 4 (or 4 x 3) patch
        for dr, (dx, dy) in (("h", (1, 0)), ("v", (0, 1))):
            pos2 = sorted(set(pos) | {(px + dx, py + dy) for (px, py) in pos})
            rows, cols, site, h1 = _patch(cell, pos2, (x, y))
            h2 = (h1[0] + dy, h1[1] + dx)
            A1, A2 = cell.A[(x, y)], cell.A[cell.wrap(x + dx, y + dy)]
            rho = np.zeros((2, 2, 2, 2))
            for s1 in range(2):
                for s2 in range(2):
                    for t1 in range(2):
                        for t2 in range(2):
                            i1, i2 = basis.impurity(A1, s1, t1), basis.impurity(A2, s2, t2)
                            f = lambda i, j: i1 if (i, j) == h1 else (i2 if (i, j) == h2 else site(i, j))
                            rho[s1, s2, t1, t2] = bruteforce.contract(rows, cols, f, b)
            rho = rho.reshape(4, 4) / np.trace(rho.reshape(4, 4))
            assert np.abs(cell.rho2(x, y, dr) - rho).max() < 1e-12


@pytest.mark.parametrize("form", ["dense", "z2"])
@pytest.mark.parametrize("r", [0, 1, 2, 3])
@pytest.mark.parametrize("Lx,Ly", CELLS)
def test_one_sweep_is_exact(form, r, Lx, Ly):
    """The first column of a sweep of frame r from the start is exact: after
    it, the sites of frame column 1 see frame columns -1 .. 2 and frame rows
    Y-1 .. Y+1 exactly (the cut keeps all 16 states at D = 2).  The second
    column is not a pin: the half-system projectors cannot keep more states
    than the east cut of the 2x2 block carries (16 < 64), so from there on
    the sweep truncates, as it does at any fixed point."""
    cell = CellRun(64, form, iid_cell(2, cell_seeds(Lx, Ly)), Lx, Ly)
    cell.move(r)
    LY = Ly if r % 2 == 0 else Lx
    assert [sum(rec["kept"]) for rec in cell.records[:LY]] == [16] * LY
    for Y in range(LY):
        pos = [to_cell(r, X, Yr) for X in range(-1, 3) for Yr in (Y - 1, Y, Y + 1)]
        xs, ys = to_cell(r, 1, Y)
        rows, cols, site, hole = _patch(cell, pos, (xs, ys))
        eps = _eps_bf(cell, rows, cols, site, hole)
        got = cell.epsilon(xs, ys)
        assert np.abs(got - eps).max() <= 1e-9 * np.abs(eps).max(), Y


# ------------------------------------------------------------- gauge ----
def _orth(rng, D):
    q, r = np.linalg.qr(rng.standard_normal((D, D)))
    return q * np.sign(np.diag(r))[None, :]


def gauged_cell(tensors, rng, Lx=2, Ly=2):
    """The same network with an orthogonal matrix on each bond of the cell."""
    D = tensors[(0, 0)].shape[1]
    gh = {s: _orth(rng, D) for s in tensors}   # bond (x,y)-(x+1,y)
    gv = {s: _orth(rng, D) for s in tensors}   # bond (x,y)-(x,y+1)
    out = {}
    for (x, y), A in tensors.items():
        A = np.einsum("suldr,rk->suldk", A, gh[(x, y)])
        A = np.einsum("suldr,lk->sukdr", A, gh[((x - 1) % Lx, y)])
        A = np.einsum("suldr,dk->sulkr", A, gv[(x, y)])
        A = np.einsum("suldr,uk->skldr", A, gv[(x, (y - 1) % Ly)])
        out[(x, y)] = A
    return out


@pytest.mark.parametrize("form", ["dense", "z2"])
@pytest.mark.parametrize("Lx,Ly", CELLS)
def test_gauge_covariance_of_the_cell(form, Lx, Ly):
    T = iid_cell(2, cell_seeds(Lx, Ly))
    G = gauged_cell(T, np.random.default_rng(7), Lx, Ly)
    assert all(np.abs(G[s] - T[s]).max() > 0.1 for s in T)
    ref = CellRun(12, form, T, Lx, Ly).step(3)
    gau = CellRun(12, form, G, Lx, Ly).step(3)
    for r1, r2 in zip(ref.records, gau.records):
        assert r1["kept"] == r2["kept"]
        assert np.allclose(r1["spectrum"], r2["spectrum"], rtol=1e-8, atol=1e-13)
    for (x, y) in ref.sites:
        assert np.abs(ref.rho1(x, y) - gau.rho1(x, y)).max() < 1e-9
        for dr in ("h", "v"):
            assert np.abs(ref.rho2(x, y, dr) - gau.rho2(x, y, dr)).max() < 1e-9
    # a tensor placed at the wrong site changes the network
    W = dict(G)
    W[(0, 0)], W[(1, 0)] = G[(1, 0)], G[(0, 0)]
    bad = CellRun(12, form, W, Lx, Ly).step(3)
    assert np.abs(ref.rho1(0, 0) - bad.rho1(0, 0)).max() > 1e-3


# ------------------------------------------------------ dense vs Z2 ----
@pytest.mark.parametrize("D,chi,iters", [(2, 16, 8), (3, 20, 2)])
def test_cell_dense_and_z2_agree(D, chi, iters):
    T = iid_cell(D)
    dense = CellRun(chi, "dense", T, 2, 2).step(iters)
    z2 = CellRun(chi, "z2", T, 2, 2).step(iters)
    for rd, rz in zip(dense.records, z2.records):
        k = sum(rz["kept"])
        assert rd["kept"][0] == k
        assert np.allclose(rd["spectrum"][:k], rz["spectrum"][:k], rtol=1e-6, atol=1e-13)
    for (x, y) in dense.sites:
        assert np.abs(dense.rho1(x, y) - z2.rho1(x, y)).max() < 1e-11
        assert np.abs(dense.rho2(x, y, "v") - z2.rho2(x, y, "v")).max() < 1e-11
        assert np.array_equal(z2.rho2(x, y, "h"), z2.rho2(x, y, "h").T)
    assert abs(dense.energy() - z2.energy()) < 1e-11
    assert z2.s_err() <= 1e-15


# ----------------------------------------------------------- Onsager ----
def test_uniform_ising_cell_against_onsager_and_yang():
    beta = 0.45
    A = inputs.ising_peps(beta)
    cell = CellRun(16, "z2", {s: A for s in SEEDS_2x2}, 2, 2, boundary=inputs.ising_up_boundary(beta))
    for _ in range(300):
        cell.step(1)
        if cell.deltas[-1] < 1e-12:
            break
    zz = np.kron(np.diag([1.0, -1.0]), np.diag([1.0, -1.0]))
    for (x, y) in cell.sites:
        for dr in ("h", "v"):
            assert abs(np.trace(cell.rho2(x, y, dr) @ zz) - ising_nn_corr(beta)) < 1e-8
        r1 = cell.rho1(x, y)
        assert abs((r1[0, 0] - r1[1, 1]) - yang_m(beta)) < 1e-6
