"""The C ABI without a GPU: every symbol the headers declare is exported by
libhctm.so, and the calls that do no device work (defaults, workspace sizing,
argument checks) behave as documented in include/hctm.h."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_11596_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("hctm.h", "hctm_testing.h", "hctm_serve.h", "hctm_hotrg.h")]
DECL = re.compile(r"^\s*(?:const\s+)?(?:int|void|char|long long|size_t)\s*\**\s*(\w+)\s*\(", re.M)


def declared():
    names = []
    for h in HEADERS:
        with open(h) as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        names += DECL.findall(text)
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2410_11596_amd import build

        build.build()
    return binding.lib()


def test_headers_declare_the_documented_calls():
    names = declared()
    for must in ("ctm_init", "ctm_step", "ctm_converged", "ctm_rdm_1site", "ctm_rdm_2site", "ctm_free"):
        assert must in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol(L):
    names = declared()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert sorted(binding.EXPORTS) == sorted(names)


def test_opts_default(L):
    o = binding.CtmOpts()
    assert L.ctm_opts_default(ctypes.byref(o)) == binding.CTM_OK
    assert o.form == binding.CTM_FORM_Z2
    assert o.svd_rel_cutoff == 1e-12
    assert o.svd_iters == 12
    assert not o.boundary and not o.stream and not o.workspace
    assert o.Lx == 1 and o.Ly == 1
    assert o.precision == binding.CTM_PREC_FP64
    assert o.c4v == 0
    assert L.ctm_opts_default(None) == binding.CTM_E_ARG


def _ws(L, d, D, chi, **kw):
    o = binding.CtmOpts()
    L.ctm_opts_default(ctypes.byref(o))
    keep = None
    for k, v in kw.items():
        if k == "boundary":
            keep = np.ascontiguousarray(v, dtype=np.float64)
            o.boundary = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            setattr(o, k, v)
    n = ctypes.c_size_t(0)
    rc = L.ctm_workspace_size(d, D, chi, ctypes.byref(o), ctypes.byref(n))
    return rc, n.value


def test_workspace_size_grows_with_chi_and_cell(L):
    rc, a = _ws(L, 2, 4, 32)
    assert rc == 0 and a > 0
    rc, b = _ws(L, 2, 4, 64)
    assert rc == 0 and b > a
    rc, c = _ws(L, 2, 4, 64, Lx=2, Ly=2)
    assert rc == 0 and c > b
    # the D = 6, chi = 144 workload fits comfortably in one GPU's HBM
    rc, big = _ws(L, 2, 6, 144)
    assert rc == 0 and big < 16 * 2**30


def test_workspace_size_at_the_limits(L):
    """The largest accepted sizes give finite sizes that keep growing (no
    overflow of the size arithmetic), one past them is rejected, and the
    smallest problem is accepted."""
    rc, one = _ws(L, 1, 1, 1)
    assert rc == 0 and one > 0
    rc, a = _ws(L, 2, 8, 4096)
    assert rc == 0
    rc, b = _ws(L, 16, 8, 4096)
    assert rc == 0 and b > a
    rc, c = _ws(L, 16, 8, 4096, Lx=4, Ly=4)
    assert rc == 0 and c > b and c < 2**62
    assert _ws(L, 2, 8, 4097)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 8, 4096, Lx=5)[0] == binding.CTM_E_ARG
    # one GPU's 288 GB holds a D = 6 solve up to chi of about 1500
    assert _ws(L, 2, 6, 1500)[1] < 288e9 < _ws(L, 2, 6, 1600)[1]


@pytest.mark.parametrize("d,D,chi", [(0, 2, 8), (17, 2, 8), (2, 0, 8), (2, 9, 8), (2, 2, 0), (2, 2, 5000)])
def test_size_checks(L, d, D, chi):
    rc, _ = _ws(L, d, D, chi)
    assert rc == binding.CTM_E_ARG
    assert b"must be" in L.ctm_last_error(None)


def test_option_checks(L):
    assert _ws(L, 2, 2, 8, form=7)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, svd_rel_cutoff=-1.0)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, svd_iters=0)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, Lx=0)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, Ly=5)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, precision=3)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, precision=binding.CTM_PREC_BF16X3)[0] == 0
    assert _ws(L, 2, 2, 8, precision=binding.CTM_PREC_FP32)[0] == 0
    assert _ws(L, 2, 2, 8, c4v=2)[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, c4v=1)[0] == 0
    assert _ws(L, 2, 2, 8, c4v=1, Lx=2)[0] == binding.CTM_E_ARG
    assert b"1 x 1" in L.ctm_last_error(None)
    # the Z2 form needs a swap-symmetric boundary vector; the plain form does not
    b = np.array([1.0, 0.5, 0.0, 1.0])
    assert _ws(L, 2, 2, 8, boundary=b)[0] == binding.CTM_E_ARG
    assert b"swap symmetric" in L.ctm_last_error(None)
    assert _ws(L, 2, 2, 8, boundary=b, form=binding.CTM_FORM_DENSE)[0] == 0
    assert _ws(L, 2, 2, 8, boundary=np.array([1.0, 0.5, 0.5, 1.0]))[0] == 0
    assert _ws(L, 2, 2, 8, boundary=np.zeros(4))[0] == binding.CTM_E_ARG
    assert _ws(L, 2, 2, 8, boundary=np.array([1.0, np.nan, np.nan, 1.0]))[0] == binding.CTM_E_NUMERIC


def test_init_rejects_bad_arguments_before_touching_a_device(L):
    A = np.ones((2, 2, 2, 2, 2))
    ctx = ctypes.c_void_p(1234)
    dp = A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.ctm_init(ctypes.byref(ctx), dp, 2, 9, 8, None) == binding.CTM_E_ARG
    assert ctx.value is None  # *out is cleared on failure
    assert L.ctm_init(ctypes.byref(ctx), None, 2, 2, 8, None) == binding.CTM_E_ARG
    assert L.ctm_init(None, dp, 2, 2, 8, None) == binding.CTM_E_ARG
    A[0, 0, 0, 0, 0] = np.inf
    assert L.ctm_init(ctypes.byref(ctx), dp, 2, 2, 8, None) == binding.CTM_E_NUMERIC
    assert b"non-finite" in L.ctm_last_error(None)


def test_null_context(L):
    L.ctm_free(None)
    assert L.ctm_step(None, 1) == binding.CTM_E_ARG
    assert L.ctm_set_precision(None, binding.CTM_PREC_FP32) == binding.CTM_E_ARG
    n = ctypes.c_int(0)
    assert L.ctm_num_records(None, ctypes.byref(n)) == binding.CTM_E_ARG
    assert isinstance(L.ctm_last_error(None), bytes)


def test_server_argument_checks(L):
    """The serving calls reject bad arguments before touching a device."""
    s = ctypes.c_void_p()
    assert L.ctm_server_create(None, 1 << 20, 2) == binding.CTM_E_ARG
    assert L.ctm_server_create(ctypes.byref(s), 0, 2) == binding.CTM_E_ARG
    assert L.ctm_server_create(ctypes.byref(s), 1 << 20, 0) == binding.CTM_E_ARG
    assert L.ctm_server_create(ctypes.byref(s), 1 << 20, 65) == binding.CTM_E_ARG
    assert s.value is None
    A = np.ones(2 * 2 ** 4)
    i = ctypes.c_longlong()
    dp = A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.ctm_server_submit(None, dp, 2, 2, 8, 0, 1e-10, 10, ctypes.byref(i)) == binding.CTM_E_ARG
    info = binding.SolveInfo()
    assert L.ctm_server_wait(None, 1, None, None, None, ctypes.byref(info)) == binding.CTM_E_ARG
    assert L.ctm_server_load(None, None, None) == binding.CTM_E_ARG
    L.ctm_server_destroy(None)


def test_c4v_init_rejects_a_tensor_without_the_symmetries_before_touching_a_device(L):
    from oracle import c4v
    from paper_2410_11596_amd import inputs

    o = binding.CtmOpts()
    L.ctm_opts_default(ctypes.byref(o))
    o.c4v = 1
    ctx = ctypes.c_void_p(1234)
    A = np.ascontiguousarray(inputs.iid_tensor(2, 3, 4))
    rc = L.ctm_init(ctypes.byref(ctx), A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, 3, 8, ctypes.byref(o))
    assert rc == binding.CTM_E_ARG and ctx.value is None
    assert b"not invariant" in L.ctm_last_error(None)
    # a tensor with the rotations but not the reflection is refused too
    B = inputs.iid_tensor(2, 3, 5)
    R = sum(np.transpose(B, (0,) + tuple(1 + (np.arange(4) + r) % 4)) for r in range(4)) / 4.0
    assert np.abs(np.transpose(R, (0, 2, 3, 4, 1)) - R).max() < 1e-15
    assert not c4v.is_c4v(R)
    R = np.ascontiguousarray(R)
    rc = L.ctm_init(ctypes.byref(ctx), R.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, 3, 8, ctypes.byref(o))
    assert rc == binding.CTM_E_ARG
    # the symmetrised tensor passes the check (on a machine without a device
    # the call then fails at the device, not at the argument check)
    S = np.ascontiguousarray(c4v.c4v_symmetrize(inputs.iid_tensor(2, 3, 4)))
    rc = L.ctm_init(ctypes.byref(ctx), S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, 3, 8, ctypes.byref(o))
    assert rc != binding.CTM_E_ARG
    if rc == binding.CTM_OK:
        L.ctm_free(ctx)


def test_hotrg_argument_checks_before_touching_a_device(L):
    o = binding.HotrgOpts()
    assert L.hotrg_opts_default(ctypes.byref(o)) == binding.CTM_OK
    assert o.form == binding.CTM_FORM_Z2 and o.svd_rel_cutoff == 1e-12 and o.probes == 0 and not o.stream
    A = np.ones((2, 2, 2, 2, 2))
    dp = A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ctx = ctypes.c_void_p(99)
    assert L.hotrg_init(ctypes.byref(ctx), dp, 2, 7, 8, ctypes.byref(o)) == binding.CTM_E_ARG
    assert ctx.value is None
    assert L.hotrg_init(ctypes.byref(ctx), dp, 2, 2, 65, ctypes.byref(o)) == binding.CTM_E_ARG
    assert b"at most 64" in L.hotrg_last_error(None)
    o.form = binding.CTM_FORM_DENSE
    assert L.hotrg_init(ctypes.byref(ctx), dp, 2, 2, 65, ctypes.byref(o)) == binding.CTM_E_ARG
    o.form = 5
    assert L.hotrg_init(ctypes.byref(ctx), dp, 2, 2, 8, ctypes.byref(o)) == binding.CTM_E_ARG
    o.form = binding.CTM_FORM_Z2
    o.probes = 2
    assert L.hotrg_init(ctypes.byref(ctx), dp, 2, 2, 8, ctypes.byref(o)) == binding.CTM_E_ARG
    o.probes = 0
    A[1, 0, 0, 0, 0] = np.nan
    assert L.hotrg_init(ctypes.byref(ctx), dp, 2, 2, 8, ctypes.byref(o)) == binding.CTM_E_NUMERIC
    assert L.hotrg_init(ctypes.byref(ctx), None, 2, 2, 8, ctypes.byref(o)) == binding.CTM_E_ARG
    assert L.hotrg_step(None, 1) == binding.CTM_E_ARG
    assert L.hotrg_log_z(None, None) == binding.CTM_E_ARG
    L.hotrg_free(None)


def test_hook_extents():
    """The extents the binding checks before a raw-pointer test hook runs."""
    assert binding._span(50, 60, 90) == 49 * 90 + 60
    assert binding._span(0, 60, 90) == 0 and binding._span(70, 0, 90) == 0
    assert binding._box(0, [2, 3], [3, 1]) == (0, 6)
    assert binding._box(5, [4], [-1]) == (2, 6)
    assert binding._box(0, [3, 0], [1, 1]) == (0, 0)
    # the scattered product's box: [M/T, T, N/R, R] over a permuted (a0, a2, a1, a3) array
    a0, a1, a2, a3 = 3, 4, 5, 6
    assert binding._box(0, [a0, a1, a2, a3], [a2 * a1 * a3, a3, a1 * a3, 1]) == (0, a0 * a1 * a2 * a3)
