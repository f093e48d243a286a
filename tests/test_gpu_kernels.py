"""GPU checks of the building blocks of the move, each against a plain numpy
FP64 computation of the same operation (ragged sizes, every operand layout)."""
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (130, 129, 257), (256, 384, 128), (300, 7, 1000),
                                   (2000, 1990, 70), (1937, 2051, 33)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_matches_numpy(hc, M, N, K, ta, tb):
    """FP64 products; the last two sizes give enough tiles for the large
    128 x 64 tile, with ragged edges in both directions."""
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * ta + 3 * tb)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    cs = rng.standard_normal(N)
    ref = 1.5 * (A.T if ta else A) @ (B.T if tb else B) * cs[None, :] - 0.5 * C0
    dA, dB, dC, dcs = _dev(A), _dev(B), _dev(C0), _dev(cs)
    hc.dev_gemm(dA, dB, dC, M, N, K, A.shape[1], B.shape[1], N, ta, tb, 1.5, -0.5, dcs)
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    scale = np.abs(A).max() * np.abs(B).max() * K * np.abs(cs).max() + np.abs(C0).max()
    assert np.abs(out - ref).max() <= 1e-14 * scale


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (130, 129, 257), (300, 260, 1000), (2600, 100, 2600)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_f32_matches_rounded_operands(hc, M, N, K, ta, tb):
    """FP32 products (CTM_PREC_FP32): equal to the product of the operands
    rounded to FP32, up to FP32 accumulation, K * 2^-24 |A||B| per entry."""
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * ta + 3 * tb)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    cs = rng.standard_normal(N)
    A32, B32 = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    opA, opB = (A32.T if ta else A32), (B32.T if tb else B32)
    ref = 1.5 * (opA @ opB) * cs[None, :] - 0.5 * C0
    bound = 1.5 * K * 2.0 ** -24 * (np.abs(opA) @ np.abs(opB)) * np.abs(cs)[None, :] + 1e-14 * np.abs(C0)
    dA, dB, dC, dcs = _dev(A), _dev(B), _dev(C0), _dev(cs)
    scratch = torch.zeros(16 * M * N, dtype=torch.float64, device="cuda")
    hc.dev_gemm(dA, dB, dC, M, N, K, A.shape[1], B.shape[1], N, ta, tb, 1.5, -0.5, dcs, scratch, f32=True)
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    assert np.all(np.abs(out - ref) <= bound)
    # and it is not the FP64 product: the operand rounding shows at K >= 5
    if K >= 5:
        ref64 = 1.5 * ((A.T if ta else A) @ (B.T if tb else B)) * cs[None, :] - 0.5 * C0
        assert np.abs(out - ref64).max() > 1e-12


def _bf16(x):
    """Round FP32 values to BF16 (nearest, ties to even) in FP64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u << 16).astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (130, 129, 257), (300, 260, 1000)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_gemm_bf16x3_matches_split_operands(hc, M, N, K, ta, tb):
    """BF16x3 products (CTM_PREC_BF16X3): each FP32-rounded operand x = hi +
    lo in BF16, hi*hi + hi*lo + lo*hi accumulated in FP32; equal to that sum
    computed in FP64 up to FP32 accumulation, and within 2^-15 relative of
    the FP64 product."""
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * ta + 3 * tb)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    def parts(X):
        x = X.astype(np.float32).astype(np.float64)
        hi = _bf16(x)
        return hi, _bf16(x - hi)
    ah, al = parts(A)
    bh, bl = parts(B)
    op = lambda X, t: X.T if t else X
    ref3 = op(ah, ta) @ op(bh, tb) + op(ah, ta) @ op(bl, tb) + op(al, ta) @ op(bh, tb)
    absAB = np.abs(op(A, ta)) @ np.abs(op(B, tb))
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    scratch = torch.zeros(16 * M * N, dtype=torch.float64, device="cuda")
    hc.dev_gemm(dA, dB, dC, M, N, K, A.shape[1], B.shape[1], N, ta, tb, 1.0, 0.0, None, scratch, precision="bf16x3")
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    assert np.all(np.abs(out - ref3) <= (K + 2) * 2.0 ** -24 * 3 * absAB + 1e-300)
    ref64 = op(A, ta) @ op(B, tb)
    assert np.all(np.abs(out - ref64) <= 2.0 ** -15 * absAB + 1e-300)


@pytest.mark.parametrize("M,N,K,ta", [(126, 126, 2600, 1), (60, 84, 5000, 0), (7, 300, 3000, 1)])
def test_gemm_split_k(hc, M, N, K, ta):
    """Small outputs with a long reduction are split over K (Gram matrices)."""
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M, N))
    ref = 2.0 * (A.T if ta else A) @ B + 0.25 * C0
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    scratch = torch.zeros(64 * M * N, dtype=torch.float64, device="cuda")
    hc.dev_gemm(dA, dB, dC, M, N, K, A.shape[1], N, N, ta, 0, 2.0, 0.25, None, scratch)
    torch.cuda.synchronize()
    assert np.abs(scratch.cpu().numpy()).max() > 0.0  # the split path was taken
    assert np.abs(dC.cpu().numpy() - ref).max() <= 1e-13 * np.sqrt(K) * 8


def test_gemm_leading_dims_and_zero_k(hc):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((70, 90))
    B = rng.standard_normal((60, 80))
    C = rng.standard_normal((70, 100))
    dA, dB, dC = _dev(A), _dev(B), _dev(C)
    # sub-block product with leading dimensions larger than the sizes
    hc.dev_gemm(dA, dB, dC, 50, 40, 60, 90, 80, 100, 0, 0, 1.0, 0.0)
    torch.cuda.synchronize()
    ref = C.copy()
    ref[:50, :40] = A[:50, :60] @ B[:60, :40]
    assert np.abs(dC.cpu().numpy() - ref).max() < 1e-12
    # K = 0: C = beta C
    hc.dev_gemm(dA, dB, dC, 70, 100, 0, 90, 80, 100, 0, 0, 1.0, 0.5)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), 0.5 * ref)


@pytest.mark.parametrize("shape,perm", [((3, 40, 5, 33), (0, 3, 2, 1)), ((64, 64), (1, 0)), ((7, 1, 9, 2, 5), (4, 2, 0, 1, 3)),
                                         ((50, 3, 70), (0, 1, 2)), ((5, 18, 18, 72), (0, 3, 2, 1)),
                                         ((4, 3, 10, 37), (0, 3, 2, 1)), ((6, 9, 7, 18), (0, 2, 1, 3)),
                                         ((2, 31, 33, 40), (0, 3, 2, 1))])
def test_copy_is_exact_permutation(hc, shape, perm):
    """Exact permutations; (w, l, u, t) -> (w, t, u, l) with a short l joins
    l and u into one destination-fast index of the LDS tile."""
    rng = np.random.default_rng(len(shape))
    X = rng.standard_normal(shape)
    Y = np.ascontiguousarray(X.transpose(perm))
    dX = _dev(X)
    dY = torch.zeros(Y.size, dtype=torch.float64, device="cuda")
    istr = [X.strides[p] // 8 for p in perm]
    ostr = [s // 8 for s in Y.strides]
    hc.dev_copy(dX, dY, list(Y.shape), istr, ostr)
    torch.cuda.synchronize()
    assert np.array_equal(dY.cpu().numpy().reshape(Y.shape), Y)


@pytest.mark.parametrize("n", [1, 12, 16, 17, 33, 64, 65, 100, 126, 142, 160, 192, 200, 224, 250])
def test_cholesky_inverse(hc, n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n + 30, n))
    G = X.T @ X
    dG, dR = _dev(G), torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    hc.dev_chol_inv(dG, dR, n, 0.0, info)
    torch.cuda.synchronize()
    Ri = dR.cpu().numpy()
    assert int(info[0].item()) == 0
    assert np.allclose(np.tril(Ri, -1), 0.0)
    # Q = X R^-1 has orthonormal columns
    Q = X @ Ri
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-11 * np.linalg.cond(X) ** 2


@pytest.mark.parametrize("a0,a1,a2,a3,K,beta", [(5, 7, 3, 9, 11, 0.0), (72, 21, 21, 15, 648, 0.0),
                                                (60, 84, 15, 21, 100, 0.5), (1, 130, 2, 70, 33, 0.0)])
def test_gemm_scatter_is_permuted_product(hc, a0, a1, a2, a3, K, beta):
    """A product whose rows are legs (i0, i1) and columns (i2, i3), written
    straight into the layout [i0 i2 | i1 i3]: the same as forming it and
    permuting (bitwise: the same products, only stored elsewhere); large
    shapes take the 128 x 64 tile, small ones the 64 x 64 one (never split)."""
    rng = np.random.default_rng(a0 + a1 + a2 + a3 + K)
    M, N = a0 * a1, a2 * a3
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C0 = rng.standard_normal((a0, a2, a1, a3))
    dA, dB = _dev(A), _dev(B)
    dC = _dev(C0)
    hc.dev_gemm_scatter(dA, dB, dC, M, N, K, K, N, a1, a3, [a2 * a1 * a3, a3, a1 * a3, 1], alpha=1.5, beta=beta)
    ref_flat = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    hc.dev_gemm(dA, dB, ref_flat, M, N, K, K, N, N, 0, 0, 1.5, 0.0)
    torch.cuda.synchronize()
    ref = ref_flat.cpu().numpy().reshape(a0, a1, a2, a3).transpose(0, 2, 1, 3)
    if beta != 0.0:
        ref = ref + beta * C0
        got = dC.cpu().numpy().reshape(a0, a2, a1, a3)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    else:
        assert np.array_equal(dC.cpu().numpy().reshape(a0, a2, a1, a3), ref)


def test_peak_probes(hc):
    """The chip-ceiling probes: the MFMA probe reports the flops it issues
    and leaves finite positive sums; the stream probe copies exactly
    (odd length: the last element by a plain copy); misaligned buffers are
    an argument error."""
    sink = torch.zeros(8 * 256, dtype=torch.float64, device="cuda")
    assert hc.dev_mfma_probe(sink, 8, 3) == 8 * 4 * 3 * 32 * 8 * 2048
    torch.cuda.synchronize()
    s = sink.cpu().numpy()
    assert np.all(np.isfinite(s)) and np.all(s > 0)
    n = 100001
    src = torch.from_numpy(np.random.default_rng(5).standard_normal(n)).cuda()
    dst = torch.zeros_like(src)
    hc.dev_stream_probe(src, dst, n)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    with pytest.raises(Exception):
        hc.dev_stream_probe(src[1:], dst[1:], 10)


@pytest.mark.parametrize("n,dead", [(20, 3), (100, 57), (128, 127), (128, 64), (96, 0)])
def test_cholesky_inverse_dead_pivot(hc, n, dead):
    """A zero row and column of G (a dead pivot inside or at the edge of an
    eight-column block): it is counted in info, its row and column of R^-1 are
    zero, and the other columns of X R^-1 are orthonormal."""
    rng = np.random.default_rng(n + dead)
    X = rng.standard_normal((n + 30, n))
    X[:, dead] = 0.0
    G = X.T @ X
    dG, dR = _dev(G), torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    hc.dev_chol_inv(dG, dR, n, 0.0, info)
    torch.cuda.synchronize()
    Ri = dR.cpu().numpy()
    assert int(info[0].item()) == 1
    assert np.all(Ri[dead, :] == 0.0) and np.all(Ri[:, dead] == 0.0)
    keep = [j for j in range(n) if j != dead]
    Q = X @ Ri[:, keep]
    assert np.abs(Q.T @ Q - np.eye(n - 1)).max() < 1e-11 * np.linalg.cond(X[:, keep]) ** 2


@pytest.mark.parametrize("m,n,pre,l2", [(1, 1, 0, 0), (8, 5, 0, 0), (8, 5, 2, 0), (40, 40, 0, 0), (40, 40, 16, 0),
                                        (120, 97, 0, 0), (120, 97, 33, 0), (126, 126, 42, 0), (150, 150, 0, 0),
                                        (201, 180, 0, 0), (150, 150, 0, 1), (160, 160, 16, 1), (216, 216, 72, 1),
                                        (201, 180, 0, 1), (256, 256, 0, 1), (33, 7, 3, 1),
                                        (64, 64, 0, 0), (100, 100, 16, 0), (128, 90, 0, 0), (129, 100, 0, 0),
                                        (200, 60, 0, 0), (200, 60, 0, 1), (300, 40, 0, 0)])
def test_jacobi_svd(hc, m, n, pre, l2):
    """Jacobi SVD in LDS (n <= 160, m <= 160; instances of 4, 8 and 10 rows
    per lane), in L2 with a scratch copy (l2 = 1, n, m <= 256) or in global
    memory (no scratch); with and without the first phase over the trailing
    columns; tall blocks with more rows than the LDS kernel takes (200 x 60,
    300 x 40) go to the other kernels."""
    rng = np.random.default_rng(m + n)
    # graded singular values, as in the CTMRG spectra
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    k = min(m, n)
    s = np.logspace(0, -9, k)
    X = (U[:, :k] * s) @ V[:, :k].T
    dX = _dev(X)
    sv = torch.zeros(n, dtype=torch.float64, device="cuda")
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    sw = torch.zeros(4, dtype=torch.int32, device="cuda")
    V = torch.zeros((n, n), dtype=torch.float64, device="cuda") if m == n else None
    vlog = torch.zeros(max(1, hc.jacobi_log_doubles(n, 60)), dtype=torch.float64, device="cuda") if m == n else None
    work = torch.zeros(m * n, dtype=torch.float64, device="cuda") if l2 else None
    hc.dev_jacobi(dX, m, n, 1.1e-16 * m, 60, sv, perm, sw, V, vlog, pre=pre, work=work)
    torch.cuda.synchronize()
    if pre:
        assert int(sw[1].item()) >= 1
    if V is not None:
        Vh = V.cpu().numpy()
        # accumulated rotations: orthogonality to a few hundred ulps
        assert np.abs(Vh.T @ Vh - np.eye(n)).max() < 1e-12
        assert np.abs(X @ Vh - dX.cpu().numpy()).max() < 1e-12
    assert int(sw[0].item()) >= 0
    got = sv.cpu().numpy()
    assert np.all(np.diff(got) <= 0)
    assert np.abs(got[:k] - s).max() < 1e-13
    assert np.abs(got[k:]).max(initial=0.0) < 1e-13
    Y = dX.cpu().numpy()[:, perm.cpu().numpy()[:k]]
    Un = Y / got[None, :k]
    # left vectors of the well separated leading values are orthonormal
    top = s > 1e-6
    assert np.abs(Un[:, top].T @ Un[:, top] - np.eye(int(top.sum()))).max() < 1e-9
