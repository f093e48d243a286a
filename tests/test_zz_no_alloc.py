"""The no-allocation Jacobi entry point (hctm_dev_jacobi_noalloc) against
hctm_dev_jacobi with caller-allocated scratch: the same kernels on the same
input give the same decomposition bit for bit, on two calls in a row (the
second smaller, reusing the static buffer), and a request beyond the static
buffer is refused before any work is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_11596_amd import binding

    binding.lib()
    return binding


def _graded(m, n, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    k = min(m, n)
    return (U[:, :k] * np.logspace(0, -9, k)) @ V[:, :k].T


def _run(hc, X, m, n, pre, noalloc):
    dX = torch.tensor(X, dtype=torch.float64, device="cuda")
    sv = torch.zeros(n, dtype=torch.float64, device="cuda")
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    sw = torch.zeros(4, dtype=torch.int32, device="cuda")
    V = torch.zeros((n, n), dtype=torch.float64, device="cuda") if m == n else None
    if noalloc:
        hc.dev_jacobi_noalloc(dX, m, n, 1.1e-16 * m, 40, sv, perm, sw, V, pre=pre)
    else:
        vlog = torch.zeros(max(1, hc.jacobi_log_doubles(n, 40)), dtype=torch.float64, device="cuda")
        work = torch.zeros(m * n, dtype=torch.float64, device="cuda")
        hc.dev_jacobi(dX, m, n, 1.1e-16 * m, 40, sv, perm, sw, V if m == n else None, vlog if m == n else None,
                      pre=pre, work=work)
    torch.cuda.synchronize()
    out = [dX.cpu().numpy(), sv.cpu().numpy(), perm.cpu().numpy(), sw.cpu().numpy()]
    if V is not None:
        out.append(V.cpu().numpy())
    return out


@pytest.mark.parametrize("first,second", [((150, 150, 0), (40, 40, 16)), ((126, 126, 42), (33, 7, 3))])
def test_noalloc_jacobi_matches_allocating_entry(hc, first, second):
    for m, n, pre in (first, second):
        print(f"jacobi noalloc m={m} n={n} pre={pre}", flush=True)
        X = _graded(m, n, m + 7 * n)
        a = _run(hc, X, m, n, pre, noalloc=False)
        b = _run(hc, X, m, n, pre, noalloc=True)
        assert len(a) == len(b)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert int(b[3][0]) > 0  # converged
        k = min(m, n)
        assert np.abs(b[1][:k] - np.logspace(0, -9, k)).max() < 1e-13


def test_noalloc_jacobi_refuses_more_than_its_buffer(hc):
    n = 512
    X = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    sv = torch.zeros(n, dtype=torch.float64, device="cuda")
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    sw = torch.zeros(4, dtype=torch.int32, device="cuda")
    V = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(hc.HctmError) as e:
        hc.dev_jacobi_noalloc(X, n, n, 1e-14, 40, sv, perm, sw, V)
    assert e.value.code == hc.CTM_E_ARG and "static buffer" in str(e.value)
