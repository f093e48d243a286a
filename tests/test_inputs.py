"""The seeded input generators (shared by the oracle tests and the GPU
path; they hold none of the method's arithmetic)."""
import numpy as np

from oracle import ctmrg
from paper_2410_11596_amd import inputs


def test_heisenberg_bond_matrix():
    h = inputs.heisenberg_bond_matrix()
    # the same operator as the oracle's (built there from Pauli matrices)
    assert np.array_equal(h, ctmrg.heisenberg_bond())
    # singlet -3/4, triplet 1/4 (three times)
    assert np.allclose(np.linalg.eigvalsh(h), [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


def test_iid_tensor_is_seeded_and_normalised():
    a = inputs.iid_tensor(2, 3, 7)
    assert np.array_equal(a, inputs.iid_tensor(2, 3, 7))
    assert not np.array_equal(a, inputs.iid_tensor(2, 3, 8))
    assert a.shape == (2, 3, 3, 3, 3) and np.abs(a).max() == 1.0


def test_c4v_iid_tensor_has_the_eight_symmetries():
    from oracle import c4v

    A = inputs.c4v_iid_tensor(2, 3, 7)
    assert c4v.is_c4v(A)
    assert np.abs(A - inputs.c4v_iid_tensor(2, 3, 7)).max() == 0.0
    assert np.abs(A - c4v.c4v_symmetrize(inputs.iid_tensor(2, 3, 7))).max() < 1e-15
