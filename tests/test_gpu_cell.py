"""GPU parity on unit cells: the HIP CTMRG on Lx x Ly cells of different
tensors against the unit-cell oracle (same seeds, same iteration count).

Compared per site: the one- and two-site RDMs (both bond directions), the
one-site environment in the plain basis, the energy, and for every cut the
kept spectrum, its sector sizes and where it sits (frame, column, row).
Tolerance: 1e-10 on RDM entries and energies, as for the 1x1 cell.
"""
import numpy as np
import pytest

from oracle import ctmrg
from oracle.cell import CellRun
from paper_2410_11596_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


def cell(D, Lx, Ly, d=2):
    return {(x, y): inputs.iid_tensor(d, D, 10 + x + Lx * y) for y in range(Ly) for x in range(Lx)}


def _compare(g, o, tol=TOL, spectra_rtol=1e-6):
    for (x, y) in o.sites:
        assert np.abs(g.rdm1(x, y) - o.rho1(x, y)).max() < tol, (x, y)
        for dr in ("h", "v"):
            assert np.abs(g.rdm2(dr, x, y) - o.rho2(x, y, dr)).max() < tol, (x, y, dr)
        eo = o.epsilon(x, y)
        assert np.abs(g.epsilon(x, y) - eo).max() < 1e3 * tol * np.abs(eo).max()
    h = ctmrg.heisenberg_bond()
    assert abs(g.energy(h) - o.energy(h)) < tol * max(1.0, abs(o.energy(h)))
    recs = g.records()
    assert len(recs) == len(o.records)
    for rg, ro in zip(recs, o.records):
        assert (rg["frame"], rg["column"], rg["row"]) == (ro["frame"], ro["column"], ro["row"])
        assert tuple(rg["kept"]) == tuple(ro["kept"])
        k = sum(rg["kept"])
        assert np.allclose(rg["spectrum"][:k], ro["spectrum"][:k], rtol=spectra_rtol, atol=1e-13)


def _run(T, chi, form, iters, Lx, Ly, **kw):
    from paper_2410_11596_amd import CTMRG

    g = CTMRG(T, chi, form=form, **kw).step(iters)
    assert (g.Lx, g.Ly) == (Lx, Ly)
    o = CellRun(chi, form, T, Lx, Ly, boundary=kw.get("boundary")).step(iters)
    return g, o


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_cell_2x2_d2_chi16(form):
    T = cell(2, 2, 2)
    g, o = _run(T, 16, form, 10, 2, 2)
    _compare(g, o)
    if form == "z2":
        assert g.s_err() <= 1e-15
        for (x, y) in o.sites:
            r2 = g.rdm2("v", x, y)
            assert np.array_equal(r2, r2.T)


@pytest.mark.parametrize("Lx,Ly", [(1, 2), (2, 1), (3, 2)])
def test_cell_shapes_d2(Lx, Ly):
    """A column of one site (sources are the targets), one row, an odd width."""
    T = cell(2, Lx, Ly)
    g, o = _run(T, 12, "z2", 4, Lx, Ly)
    _compare(g, o)


@pytest.mark.parametrize("form", ["z2", "dense"])
def test_config2_cell_2x2_d4_chi64(form):
    """D = 4 (10+6), chi = 64, 2x2 cell of different tensors."""
    T = cell(4, 2, 2)
    g, o = _run(T, 64, form, 3, 2, 2)
    _compare(g, o)


def test_uniform_ising_cell_up_boundary():
    beta = 0.45
    A = inputs.ising_peps(beta)
    T = {(x, y): A for x in range(2) for y in range(2)}
    g, o = _run(T, 16, "z2", 30, 2, 2, boundary=inputs.ising_up_boundary(beta))
    for (x, y) in o.sites:
        assert np.abs(g.rdm1(x, y) - o.rho1(x, y)).max() < TOL
    assert all(r["kept"][1] == 0 for r in g.records())


def test_cell_sites_are_checked():
    from paper_2410_11596_amd import CTMRG
    from paper_2410_11596_amd.binding import HctmError

    g = CTMRG(cell(2, 2, 2), 8, form="z2")
    with pytest.raises(HctmError):
        g.rdm1(2, 0)
    with pytest.raises(HctmError):
        g.log_kappa()
    g.close()
