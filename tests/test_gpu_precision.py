"""Block products of the moves in FP32 (CTM_PREC_FP32) or BF16x3
(CTM_PREC_BF16X3) for the enlarged corners, halves, projectors and
renormalisation; the truncated SVD, normalisations and observables in FP64.

Measured against the FP64 form of the same library (itself checked against
the oracle in test_gpu_ctmrg.py): after the same iterations the RDMs agree
to about 1e-7 with FP32 products (bound 1e-6 here) and 2e-6 with BF16x3
(bound 1e-5), and FP64 iterations started from that environment reach the
converged FP64 environment (RDMs and energy within 1e-10) once the corner
spectra change by less than 1e-10."""
import numpy as np
import pytest

from paper_2410_11596_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()


H = inputs.heisenberg_bond_matrix()


def _obs(g):
    return np.concatenate([g.rdm1().ravel(), g.rdm2("h").ravel(), g.rdm2("v").ravel()]), g.energy(H)


def _ctm(A, chi, **kw):
    from paper_2410_11596_amd import CTMRG

    return CTMRG(A, chi, **kw)


BOUND = {"fp32": 1e-6, "bf16x3": 1e-5}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("form", ["z2", "dense"])
def test_low_precision_block_products_track_fp64_d4(form, prec):
    A = inputs.iid_tensor(2, 4, 0)
    g64 = _ctm(A, 64, form=form).step(8)
    g32 = _ctm(A, 64, form=form, precision=prec).step(8)
    o64, e64 = _obs(g64)
    o32, e32 = _obs(g32)
    err = np.abs(o32 - o64).max()
    assert 1e-12 < err < BOUND[prec]  # the rounding shows, within its accuracy
    assert abs(e32 - e64) < BOUND[prec]
    if form == "z2":
        assert g32.s_err() <= 1e-15  # Hermitian by construction in any precision
        r2 = g32.rdm2("h")
        assert np.array_equal(r2, r2.T)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fp64_refinement_reaches_the_fp64_fixed_point(prec):
    A = inputs.iid_tensor(2, 4, 0)
    g64 = _ctm(A, 64)
    for _ in range(60):
        g64.step(1)
        if g64.converged(1e-10)[0]:
            break
    assert g64.converged(1e-10)[0]
    o64, e64 = _obs(g64)
    g32 = _ctm(A, 64, precision=prec).step(20)
    o, e = _obs(g32)
    assert np.abs(o - o64).max() < BOUND[prec]
    g32.set_precision("fp64")
    for r in range(1, 41):
        g32.step(1)
        if r == 3:
            o, e = _obs(g32)
            assert np.abs(o - o64).max() < 100 * BOUND[prec] ** 2 + 1e-8
        if g32.converged(1e-10)[0]:
            break
    assert g32.converged(1e-10)[0]
    o, e = _obs(g32)
    assert np.abs(o - o64).max() < 1e-10
    assert abs(e - e64) < 1e-10


def test_precision_is_checked():
    from paper_2410_11596_amd.binding import HctmError

    g = _ctm(inputs.iid_tensor(2, 2, 0), 8)
    with pytest.raises(ValueError):
        g.set_precision("bf16")
    from paper_2410_11596_amd import binding

    with pytest.raises(HctmError):
        binding._check(binding.lib().ctm_set_precision(g._ctx, 7), g._ctx)
    g.close()
