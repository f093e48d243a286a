"""GPU parity on correlated states, against the oracle and an independent
reference.

The HIP path runs on perturbed product states: CTMRG on a 1x1 cell in both
forms, on a 3x2 cell of six different tensors, on a complex tensor in the
real representation of Sec. II C and on a C4v-symmetric tensor in the C4v
scheme, and HOTRG for the free energy.  Each is compared with the oracle
after the same iterations (1e-10 on RDM entries, energies, ln kappa and
ln Z) and with the infinite cylinder of the oracle's pins (the leading
eigenvectors of its row transfer matrix), which shares nothing with either.
The cylinder bounds are the oracle pins' own, since the GPU adds at most
1e-10 to them.
"""
import numpy as np
import pytest

from oracle import c4v, cell, complex_z2, ctmrg, hotrg
from paper_2410_11596_amd import inputs
from test_oracle_cylinder import _cylinder_cell, _cylinder_of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


def _gpu(A, chi, **kw):
    from paper_2410_11596_amd import CTMRG

    return CTMRG(A, chi, **kw)


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_perturbed_product_state(form):
    A = inputs.perturbed_product(2, 2, 0, eps=0.1)
    print(f"perturbed product D=2 chi=8 form={form}", flush=True)
    g = _gpu(A, 8, form=form).step(30)
    o = ctmrg.Run(8, form, A=A).step(30)
    h = ctmrg.heisenberg_bond()
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < TOL
    assert np.abs(g.rdm2("v") - o.rho2("v")).max() < TOL
    assert abs(g.energy(h) - o.energy(h)) < TOL
    assert abs(g.log_kappa() - o.log_kappa()) < TOL
    f, r1, rh, rv = _cylinder_of(A, 7)
    assert abs(g.log_kappa() - f) < 5e-11 + TOL
    assert np.abs(g.rdm1() - r1).max() < 1e-9
    assert np.abs(g.rdm2("h") - rh).max() < 3e-9
    assert np.abs(g.rdm2("v") - rv).max() < 3e-9
    assert abs(g.energy(h) - (np.trace(rh @ h) + np.trace(rv @ h))) < 2e-10


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_cell_of_perturbed_product_states(form):
    Lx, Ly = 3, 2
    As = {(x, y): inputs.perturbed_product(2, 2, 10 * y + x, eps=0.05) for y in range(Ly) for x in range(Lx)}
    print(f"3x2 cell of perturbed product states chi=8 form={form}", flush=True)
    g = _gpu(As, 8, form=form).step(30)
    assert (g.Lx, g.Ly) == (Lx, Ly)
    o = cell.CellRun(8, form, As, Lx, Ly).step(30)
    _, r1, rh, rv = _cylinder_cell(As, Lx, Ly, 6)
    h = ctmrg.heisenberg_bond()
    for (x, y) in r1:
        assert np.abs(g.rdm1(x, y) - o.rho1(x, y)).max() < TOL, (x, y)
        assert np.abs(g.rdm1(x, y) - r1[(x, y)]).max() < 1e-8, (x, y)
        for dr, ref in (("h", rh), ("v", rv)):
            assert np.abs(g.rdm2(dr, x, y) - o.rho2(x, y, dr)).max() < TOL, (x, y, dr)
            assert np.abs(g.rdm2(dr, x, y) - ref[(x, y)]).max() < 1e-8, (x, y, dr)
    assert abs(g.energy(h) - o.energy(h)) < TOL
    e_cyl = np.mean([np.trace(rh[s] @ h) + np.trace(rv[s] @ h) for s in r1])
    assert abs(g.energy(h) - e_cyl) < 5e-10 + TOL


def test_complex_perturbed_product_state():
    A = inputs.product_state([1.0, 0.0], 2) + 0.1 * inputs.complex_iid_tensor(2, 2, 3)
    print("complex perturbed product D=2 chi=8", flush=True)
    g = _gpu(A, 8).step(30)
    o = complex_z2.Run(8, A).step(30)
    h = ctmrg.heisenberg_bond()
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < TOL
    assert np.abs(g.rdm2("v") - o.rho2("v")).max() < TOL
    assert abs(g.energy(h) - o.energy(h)) < TOL
    _, r1, rh, rv = _cylinder_of(A, 7)
    assert np.abs(g.rdm1() - r1).max() < 2e-10
    assert np.abs(g.rdm2("h") - rh).max() < 2e-10
    assert np.abs(g.rdm2("v") - rv).max() < 2e-10


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_c4v_perturbed_product_state(form):
    A = inputs.product_state([1.0, 0.0], 2) + 0.2 * inputs.c4v_iid_tensor(2, 2, 5)
    print(f"C4v perturbed product D=2 chi=8 form={form}", flush=True)
    g = _gpu(A, 8, form=form, c4v=True).step(20)
    o = c4v.C4vRun(8, form, A=A).step(20)
    h = ctmrg.heisenberg_bond()
    assert np.abs(g.rdm1() - o.rho1()).max() < TOL
    assert np.abs(g.rdm2("h") - o.rho2("h")).max() < TOL
    assert abs(g.energy(h) - o.energy(h)) < TOL
    assert abs(g.log_kappa() - o.log_kappa()) < TOL
    f, r1, rh, rv = _cylinder_of(A, 7)
    assert abs(g.log_kappa() - f) < 5e-11 + TOL
    assert np.abs(g.rdm1() - r1).max() < 2e-10 + TOL
    assert np.abs(g.rdm2("h") - rh).max() < 5e-10 + TOL
    assert np.abs(g.rdm2("v") - rv).max() < 5e-10 + TOL


@pytest.mark.parametrize("form", ["dense", "z2"])
def test_hotrg_perturbed_product_state(form):
    from paper_2410_11596_amd import HOTRG

    A = inputs.perturbed_product(2, 2, 0, eps=0.05)
    print(f"HOTRG perturbed product D=2 chi=12 form={form}", flush=True)
    g = HOTRG(A, 12, form=form)
    g.step(30)
    o = hotrg.Run(12, form, A=A).step(30)
    assert abs(g.log_z() - o.log_z()) < TOL
    f = _cylinder_of(A, 7)[0]
    assert abs(g.log_z() - f) < 2e-7 + TOL
