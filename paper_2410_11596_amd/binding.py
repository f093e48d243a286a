"""ctypes binding of libhctm.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; this module
only converts arguments, takes device memory and the stream from PyTorch, and
raises on error codes.  If the library is missing the import of `lib()` fails
loudly; there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhctm.so")

CTM_OK, CTM_E_ARG, CTM_E_NOMEM, CTM_E_HIP, CTM_E_NUMERIC, CTM_E_STATE = range(6)
CTM_FORM_Z2, CTM_FORM_DENSE = 0, 1
CTM_PREC_FP64, CTM_PREC_FP32, CTM_PREC_BF16X3 = 0, 1, 2
ERROR_NAMES = {1: "CTM_E_ARG", 2: "CTM_E_NOMEM", 3: "CTM_E_HIP", 4: "CTM_E_NUMERIC", 5: "CTM_E_STATE"}

# every C symbol that the headers under include/ declare
EXPORTS = [
    "ctm_opts_default", "ctm_workspace_size", "ctm_init", "ctm_step", "ctm_converged",
    "ctm_rdm_1site", "ctm_rdm_2site", "ctm_energy", "ctm_free", "ctm_last_error",
    "ctm_env_epsilon", "ctm_s_err", "ctm_log_kappa", "ctm_num_records", "ctm_record",
    "ctm_sector_dims", "ctm_timing", "ctm_gemm_stats", "ctm_gemm_reduce_stats", "ctm_set_precision",
    "ctm_corner_spectrum", "ctm_svd_health", "ctm_record_status",
    "ctm_workspace_size_complex", "ctm_init_complex", "ctm_rdm_1site_complex", "ctm_rdm_2site_complex",
    "ctm_server_create", "ctm_server_submit", "ctm_server_wait", "ctm_server_load", "ctm_server_destroy",
    "ctm_server_submit_complex", "ctm_server_wait_complex",
    "hotrg_opts_default", "hotrg_init", "hotrg_step", "hotrg_log_z", "hotrg_sym_error", "hotrg_set_bond",
    "hotrg_energy", "hotrg_track_rdm1", "hotrg_rdm1", "hotrg_num_records",
    "hotrg_record", "hotrg_last_error", "hotrg_free",
    "hctm_dev_gemm", "hctm_dev_gemm_f32", "hctm_dev_gemm_bf16x3", "hctm_dev_copy", "hctm_dev_chol_inv", "hctm_dev_jacobi", "hctm_dev_jacobi_log_doubles",
    "hctm_dev_jacobi_noalloc", "hctm_dev_mfma_probe", "hctm_dev_stream_probe", "hctm_dev_gemm_scatter",
]


class CtmOpts(ctypes.Structure):
    _fields_ = [
        ("form", ctypes.c_int),
        ("Lx", ctypes.c_int),
        ("Ly", ctypes.c_int),
        ("boundary", ctypes.POINTER(ctypes.c_double)),
        ("svd_rel_cutoff", ctypes.c_double),
        ("svd_iters", ctypes.c_int),
        ("form_m", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("c4v", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("profile", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class HotrgOpts(ctypes.Structure):
    _fields_ = [
        ("form", ctypes.c_int),
        ("svd_rel_cutoff", ctypes.c_double),
        ("probes", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("iterations", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("delta", ctypes.c_double),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_end", ctypes.c_double),
        ("message", ctypes.c_char * 160),
    ]


class HctmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_LIB = None


def lib():
    """Load libhctm.so (built in place by __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_11596_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    dp, ip, vp = P(ctypes.c_double), P(ctypes.c_int), ctypes.c_void_p
    ctx = vp
    sig = {
        "ctm_opts_default": ([P(CtmOpts)], ctypes.c_int),
        "ctm_workspace_size": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, P(CtmOpts), P(ctypes.c_size_t)], ctypes.c_int),
        "ctm_init": ([P(vp), dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(CtmOpts)], ctypes.c_int),
        "ctm_step": ([ctx, ctypes.c_int], ctypes.c_int),
        "ctm_converged": ([ctx, ctypes.c_double, ip, dp], ctypes.c_int),
        "ctm_rdm_1site": ([ctx, ctypes.c_int, ctypes.c_int, dp], ctypes.c_int),
        "ctm_rdm_2site": ([ctx, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp], ctypes.c_int),
        "ctm_energy": ([ctx, dp, dp], ctypes.c_int),
        "ctm_free": ([ctx], None),
        "ctm_last_error": ([ctx], ctypes.c_char_p),
        "ctm_env_epsilon": ([ctx, ctypes.c_int, ctypes.c_int, dp], ctypes.c_int),
        "ctm_s_err": ([ctx, dp], ctypes.c_int),
        "ctm_log_kappa": ([ctx, dp], ctypes.c_int),
        "ctm_num_records": ([ctx, ip], ctypes.c_int),
        "ctm_record": ([ctx, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, ip], ctypes.c_int),
        "ctm_sector_dims": ([ctx, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip], ctypes.c_int),
        "ctm_corner_spectrum": ([ctx, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip], ctypes.c_int),
        "ctm_svd_health": ([ctx, ip, ip], ctypes.c_int),
        "ctm_workspace_size_complex": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, P(CtmOpts), P(ctypes.c_size_t)],
                                       ctypes.c_int),
        "ctm_init_complex": ([P(vp), dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(CtmOpts)], ctypes.c_int),
        "ctm_rdm_1site_complex": ([ctx, ctypes.c_int, ctypes.c_int, dp, dp], ctypes.c_int),
        "ctm_rdm_2site_complex": ([ctx, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp], ctypes.c_int),
        "ctm_record_status": ([ctx, ctypes.c_int, ip], ctypes.c_int),
        "ctm_timing": ([ctx, dp, ctypes.c_int, ip], ctypes.c_int),
        "ctm_gemm_stats": ([ctx, dp, dp, P(ctypes.c_longlong), ctypes.c_int], ctypes.c_int),
        "ctm_gemm_reduce_stats": ([ctx, dp, P(ctypes.c_longlong)], ctypes.c_int),
        "hctm_dev_gemm": ([vp, vp, vp] + [ctypes.c_int] * 8 + [ctypes.c_double, ctypes.c_double, vp, vp,
                                                               ctypes.c_longlong, vp], ctypes.c_int),
        "hctm_dev_gemm_f32": ([vp, vp, vp] + [ctypes.c_int] * 8 + [ctypes.c_double, ctypes.c_double, vp, vp,
                                                                   ctypes.c_longlong, vp], ctypes.c_int),
        "hctm_dev_gemm_bf16x3": ([vp, vp, vp] + [ctypes.c_int] * 8 + [ctypes.c_double, ctypes.c_double, vp, vp,
                                                                      ctypes.c_longlong, vp], ctypes.c_int),
        "hctm_dev_mfma_probe": ([vp, ctypes.c_int, ctypes.c_int, dp, vp], ctypes.c_int),
        "hctm_dev_gemm_scatter": ([vp, vp, vp] + [ctypes.c_int] * 7 + [ctypes.c_double, ctypes.c_double,
                                                                      ctypes.c_int, ctypes.c_int,
                                                                      P(ctypes.c_longlong), vp], ctypes.c_int),
        "hctm_dev_stream_probe": ([vp, vp, ctypes.c_longlong, vp], ctypes.c_int),
        "ctm_set_precision": ([ctx, ctypes.c_int], ctypes.c_int),
        "ctm_server_create": ([P(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_int], ctypes.c_int),
        "ctm_server_submit": ([ctypes.c_void_p, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_double, ctypes.c_int, P(ctypes.c_longlong)], ctypes.c_int),
        "ctm_server_wait": ([ctypes.c_void_p, ctypes.c_longlong, dp, dp, dp, P(SolveInfo)], ctypes.c_int),
        "ctm_server_load": ([ctypes.c_void_p, ip, ip], ctypes.c_int),
        "ctm_server_submit_complex": ([ctypes.c_void_p, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_int, P(ctypes.c_longlong)], ctypes.c_int),
        "ctm_server_wait_complex": ([ctypes.c_void_p, ctypes.c_longlong, dp, dp, dp, dp, dp, dp, P(SolveInfo)],
                                    ctypes.c_int),
        "ctm_server_destroy": ([ctypes.c_void_p], None),
        "hctm_dev_copy": ([vp, vp, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_longlong), P(ctypes.c_longlong), vp],
                          ctypes.c_int),
        "hctm_dev_chol_inv": ([vp, vp, ctypes.c_int, ctypes.c_double, vp, vp], ctypes.c_int),
        "hctm_dev_jacobi": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp,
                             vp, vp, vp],
                            ctypes.c_int),
        "hctm_dev_jacobi_log_doubles": ([ctypes.c_int, ctypes.c_int], ctypes.c_longlong),
        "hctm_dev_jacobi_noalloc": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp,
                                     vp, vp, vp, vp], ctypes.c_int),
        "hotrg_opts_default": ([P(HotrgOpts)], ctypes.c_int),
        "hotrg_init": ([P(vp), dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(HotrgOpts)], ctypes.c_int),
        "hotrg_step": ([vp, ctypes.c_int], ctypes.c_int),
        "hotrg_log_z": ([vp, dp], ctypes.c_int),
        "hotrg_sym_error": ([vp, dp, dp, dp], ctypes.c_int),
        "hotrg_set_bond": ([vp, dp], ctypes.c_int),
        "hotrg_energy": ([vp, dp], ctypes.c_int),
        "hotrg_track_rdm1": ([vp], ctypes.c_int),
        "hotrg_rdm1": ([vp, dp], ctypes.c_int),
        "hotrg_num_records": ([vp, ip], ctypes.c_int),
        "hotrg_record": ([vp, ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, ip, dp], ctypes.c_int),
        "hotrg_last_error": ([vp], ctypes.c_char_p),
        "hotrg_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _LIB = L
    return L


def _check(code, ctx=None):
    if code != CTM_OK:
        msg = lib().ctm_last_error(ctx).decode(errors="replace")
        raise HctmError(code, msg)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _torch():
    import torch  # noqa: PLC0415 (device memory and streams only)

    if not torch.cuda.is_available():
        raise RuntimeError("libhctm needs a HIP GPU (torch.cuda.is_available() is False)")
    return torch


def workspace_size(d, D, chi, form="z2", Lx=1, Ly=1):
    o = CtmOpts()
    _check(lib().ctm_opts_default(ctypes.byref(o)))
    o.form = CTM_FORM_Z2 if form == "z2" else CTM_FORM_DENSE
    o.Lx, o.Ly = Lx, Ly
    n = ctypes.c_size_t()
    _check(lib().ctm_workspace_size(d, D, chi, ctypes.byref(o), ctypes.byref(n)))
    return n.value


def _cell_array(A):
    """(Ly, Lx, d, D, D, D, D) array from one tensor, a dict {(x, y): A} or such an array."""
    if isinstance(A, dict):
        Lx = 1 + max(x for x, _ in A)
        Ly = 1 + max(y for _, y in A)
        if len(A) != Lx * Ly:
            raise ValueError("the dict must hold every site (x, y) of the cell")
        A = np.stack([np.stack([np.asarray(A[(x, y)], dtype=np.float64) for x in range(Lx)]) for y in range(Ly)])
    A = np.asarray(A, dtype=np.float64)
    if A.ndim == 5:
        A = A[None, None]
    if A.ndim != 7 or len(set(A.shape[3:])) != 1 or A.shape[4] != A.shape[3]:
        raise ValueError("A must have shape (d, D, D, D, D) or (Ly, Lx, d, D, D, D, D)")
    return np.ascontiguousarray(A)


def _precision_code(p):
    codes = {"fp64": CTM_PREC_FP64, "fp32": CTM_PREC_FP32, "bf16x3": CTM_PREC_BF16X3}
    if p not in codes:
        raise ValueError(f"precision must be one of {sorted(codes)}")
    return codes[p]


class CTMRG:
    """One CTMRG solve on the GPU (Z2 or plain form).

    A: one real tensor (d, D, D, D, D), legs [s, u, l, d, r], for the 1x1
    cell, or the tensors of an Lx x Ly cell as an array (Ly, Lx, d, D, D, D,
    D) or a dict {(x, y): tensor}.  Device memory is a torch uint8 tensor
    handed to the library as its workspace; work runs on torch's current HIP
    stream.  c4v=True selects the C4v-symmetric scheme (one corner, one edge)
    for a tensor invariant under the symmetries of the square.
    """

    def __init__(self, A, chi, form="z2", boundary=None, svd_rel_cutoff=1e-12, svd_iters=12, seed=0x5EED,
                 stream=None, torch_workspace=True, profile=False, form_m=False, precision="fp64", c4v=False):
        torch = _torch()
        self.complex = bool(np.iscomplexobj(A))
        if self.complex:
            Ac = np.ascontiguousarray(A, dtype=np.complex128)
            if Ac.ndim != 5:
                raise ValueError("a complex tensor must have shape (d, D, D, D, D) (1 x 1 cell)")
            A_re, A_im = np.ascontiguousarray(Ac.real), np.ascontiguousarray(Ac.imag)
            A = A_re
        A = _cell_array(A)
        self.Ly, self.Lx = A.shape[0], A.shape[1]
        self.d, self.D, self.chi = A.shape[2], A.shape[3], int(chi)
        self.form = form
        o = CtmOpts()
        _check(lib().ctm_opts_default(ctypes.byref(o)))
        o.form = CTM_FORM_Z2 if form == "z2" else CTM_FORM_DENSE
        o.Lx, o.Ly = self.Lx, self.Ly
        o.svd_rel_cutoff = svd_rel_cutoff
        o.svd_iters = svd_iters
        o.form_m = 1 if form_m else 0
        o.precision = _precision_code(precision)
        o.c4v = 1 if c4v else 0
        o.seed = seed
        o.profile = 1 if profile else 0
        self._b = None
        if boundary is not None:
            self._b = np.ascontiguousarray(boundary, dtype=np.float64).reshape(-1)
            o.boundary = _dptr(self._b)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        self._ws = None
        size_fn = lib().ctm_workspace_size_complex if self.complex else lib().ctm_workspace_size
        if torch_workspace:
            nbytes = ctypes.c_size_t()
            _check(size_fn(self.d, self.D, self.chi, ctypes.byref(o), ctypes.byref(nbytes)))
            self._ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
            o.workspace = ctypes.c_void_p(self._ws.data_ptr())
            o.workspace_bytes = nbytes.value
        ctx = ctypes.c_void_p()
        if self.complex:
            _check(lib().ctm_init_complex(ctypes.byref(ctx), _dptr(A_re), _dptr(A_im), self.d, self.D, self.chi,
                                          ctypes.byref(o)))
        else:
            _check(lib().ctm_init(ctypes.byref(ctx), _dptr(A), self.d, self.D, self.chi, ctypes.byref(o)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            lib().ctm_free(self._ctx)
            self._ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_precision(self, precision):
        """'fp64', 'fp32' or 'bf16x3' for the block products of the following steps."""
        _check(lib().ctm_set_precision(self._ctx, _precision_code(precision)), self._ctx)
        return self

    def step(self, n=1):
        _check(lib().ctm_step(self._ctx, int(n)), self._ctx)
        return self

    def converged(self, tol):
        c = ctypes.c_int()
        dl = ctypes.c_double()
        _check(lib().ctm_converged(self._ctx, tol, ctypes.byref(c), ctypes.byref(dl)), self._ctx)
        return bool(c.value), dl.value

    def run(self, max_iter, tol=None):
        for _ in range(max_iter):
            self.step(1)
            if tol is not None and self.converged(tol)[0]:
                break
        return self

    def rdm1(self, x=0, y=0):
        """One-site RDM (complex128 for a complex tensor)."""
        if self.complex:
            re, im = np.zeros((self.d, self.d)), np.zeros((self.d, self.d))
            _check(lib().ctm_rdm_1site_complex(self._ctx, x, y, _dptr(re), _dptr(im)), self._ctx)
            return re + 1j * im
        rho = np.zeros((self.d, self.d))
        _check(lib().ctm_rdm_1site(self._ctx, x, y, _dptr(rho)), self._ctx)
        return rho

    def rdm2(self, direction="h", x=0, y=0):
        """Two-site RDM [(s1 s2), (s1' s2')] (complex128 for a complex tensor)."""
        n = self.d * self.d
        dr = 0 if direction == "h" else 1
        if self.complex:
            re, im = np.zeros((n, n)), np.zeros((n, n))
            _check(lib().ctm_rdm_2site_complex(self._ctx, x, y, dr, _dptr(re), _dptr(im)), self._ctx)
            return re + 1j * im
        rho = np.zeros((n, n))
        _check(lib().ctm_rdm_2site(self._ctx, x, y, dr, _dptr(rho)), self._ctx)
        return rho

    def energy(self, h):
        h = np.ascontiguousarray(h, dtype=np.float64)
        e = ctypes.c_double()
        _check(lib().ctm_energy(self._ctx, _dptr(h), ctypes.byref(e)), self._ctx)
        return e.value

    def epsilon(self, x=0, y=0):
        q = self.D * self.D
        eps = np.zeros((q, q, q, q))
        _check(lib().ctm_env_epsilon(self._ctx, x, y, _dptr(eps)), self._ctx)
        return eps

    def s_err(self):
        s = ctypes.c_double()
        _check(lib().ctm_s_err(self._ctx, ctypes.byref(s)), self._ctx)
        return s.value

    def log_kappa(self):
        s = ctypes.c_double()
        _check(lib().ctm_log_kappa(self._ctx, ctypes.byref(s)), self._ctx)
        return s.value

    def num_records(self):
        n = ctypes.c_int()
        _check(lib().ctm_num_records(self._ctx, ctypes.byref(n)), self._ctx)
        return n.value

    def record(self, m):
        cap = 8192
        s = np.zeros(cap)
        n, ke, ko = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        info = (ctypes.c_int * 8)()
        _check(lib().ctm_record(self._ctx, m, _dptr(s), cap, ctypes.byref(n), ctypes.byref(ke), ctypes.byref(ko),
                                info), self._ctx)
        st = ctypes.c_int()
        _check(lib().ctm_record_status(self._ctx, m, ctypes.byref(st)), self._ctx)
        return {"spectrum": s[: n.value].copy(), "kept": (ke.value, ko.value), "frame": info[0],
                "column": info[1], "row": info[2], "iters": (info[3], info[4]), "sweeps": (info[5], info[6]),
                "implicit": bool(info[7]), "unconverged": (bool(st.value & 1), bool(st.value & 2)),
                "multiplet_split": bool(st.value & 4)}

    def records(self):
        return [self.record(m) for m in range(self.num_records())]

    def corner_spectrum(self, corner, x=0, y=0):
        """Merged, sum-normalised, zero-padded spectrum of corner 0..3 (C1..C4)."""
        n = ctypes.c_int()
        _check(lib().ctm_corner_spectrum(self._ctx, x, y, corner, None, 0, ctypes.byref(n)), self._ctx)
        s = np.zeros(n.value)
        _check(lib().ctm_corner_spectrum(self._ctx, x, y, corner, _dptr(s), n.value, ctypes.byref(n)), self._ctx)
        return s

    def svd_health(self):
        """(truncations with a sector stopped at the iteration cap, truncations
        whose chi cut split a near-degenerate multiplet)."""
        u, m = ctypes.c_int(), ctypes.c_int()
        _check(lib().ctm_svd_health(self._ctx, ctypes.byref(u), ctypes.byref(m)), self._ctx)
        return u.value, m.value

    def sector_dims(self, side, x=0, y=0):
        e, o = ctypes.c_int(), ctypes.c_int()
        _check(lib().ctm_sector_dims(self._ctx, x, y, side, ctypes.byref(e), ctypes.byref(o)), self._ctx)
        return e.value, o.value

    def gemm_stats(self, reset=False):
        """Profile mode: GEMM kernel flops, seconds and launches, and the
        split-K reductions' seconds and launches (read before a reset)."""
        f, t, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        rt, rn = ctypes.c_double(), ctypes.c_longlong()
        _check(lib().ctm_gemm_reduce_stats(self._ctx, ctypes.byref(rt), ctypes.byref(rn)), self._ctx)
        _check(lib().ctm_gemm_stats(self._ctx, ctypes.byref(f), ctypes.byref(t), ctypes.byref(n), 1 if reset else 0),
               self._ctx)
        return {"flops": f.value, "seconds": t.value, "launches": n.value, "reduce_seconds": rt.value,
                "reduce_launches": rn.value}

    def timing(self):
        t = np.zeros(16)
        n = ctypes.c_int()
        _check(lib().ctm_timing(self._ctx, _dptr(t), 16, ctypes.byref(n)), self._ctx)
        return t[: n.value].copy()


# ------------------------------------------------------------ test hooks ----
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, lo, hi, name, dtype="float64"):
    """t must be a device tensor of dtype whose elements cover [lo, hi): the
    kernels behind these hooks take raw pointers and cannot check."""
    torch = _torch()
    if t.dtype != getattr(torch, dtype) or not t.is_cuda:
        raise ValueError(f"{name}: a {dtype} device tensor")
    if hi > lo and (lo < 0 or hi > t.numel()):
        raise ValueError(f"{name}: the call reaches elements [{lo}, {hi}) of a tensor of {t.numel()}")


def _span(rows, cols, ld):
    """Elements spanned by a row-major rows x cols operand with leading dimension ld."""
    return 0 if rows <= 0 or cols <= 0 else (rows - 1) * ld + cols


def _box(offset, dims, strides):
    """[lowest, highest + 1) of the offsets offset + sum x_j strides_j, 0 <= x_j < dims_j."""
    if any(d <= 0 for d in dims):
        return 0, 0
    lo = offset + sum((d - 1) * s for d, s in zip(dims, strides) if s < 0)
    hi = offset + sum((d - 1) * s for d, s in zip(dims, strides) if s > 0)
    return lo, hi + 1


def dev_gemm(A, B, C, M, N, K, lda, ldb, ldc, ta=0, tb=0, alpha=1.0, beta=0.0, cscale=None, scratch=None,
             f32=False, precision=None):
    """precision: 'fp64' (default), 'fp32' or 'bf16x3' (f32=True is 'fp32')."""
    torch = _torch()
    cs = _ptr(cscale) if cscale is not None else None
    sp = _ptr(scratch) if scratch is not None else None
    sn = scratch.numel() if scratch is not None else 0
    p = precision or ("fp32" if f32 else "fp64")
    f = {"fp64": lib().hctm_dev_gemm, "fp32": lib().hctm_dev_gemm_f32, "bf16x3": lib().hctm_dev_gemm_bf16x3}[p]
    _need(A, 0, _span(K, M, lda) if ta else _span(M, K, lda), "A")
    _need(B, 0, _span(N, K, ldb) if tb else _span(K, N, ldb), "B")
    _need(C, 0, _span(M, N, ldc), "C")
    if cscale is not None:
        _need(cscale, 0, max(N, 0), "cscale")
    if scratch is not None:
        _need(scratch, 0, 0, "scratch")
    _check(f(_ptr(A), _ptr(B), _ptr(C), M, N, K, lda, ldb, ldc, ta, tb, alpha, beta, cs, sp, sn, _stream_ptr(torch)))


def dev_gemm_scatter(A, B, C, M, N, K, lda, ldb, T, R, strides, ta=0, tb=0, alpha=1.0, beta=0.0):
    """alpha op(A) op(B) + beta C with element (i0 T + i1, i2 R + i3) stored at
    C + sum_q i_q strides[q]."""
    torch = _torch()
    _need(A, 0, _span(K, M, lda) if ta else _span(M, K, lda), "A")
    _need(B, 0, _span(N, K, ldb) if tb else _span(K, N, ldb), "B")
    if T >= 1 and R >= 1 and M % T == 0 and N % R == 0:  # else the library refuses the call
        _need(C, *_box(0, [M // T, T, N // R, R], [int(x) for x in strides]), "C")
    s = (ctypes.c_longlong * 4)(*[int(x) for x in strides])
    _check(lib().hctm_dev_gemm_scatter(_ptr(A), _ptr(B), _ptr(C), M, N, K, lda, ldb, ta, tb, alpha, beta, T, R, s,
                                       _stream_ptr(torch)))


def dev_mfma_probe(sink, blocks, iters):
    """Enqueue the FP64 matrix-core issue probe on torch's current stream;
    returns the flops it executes (time it with events on that stream)."""
    torch = _torch()
    if sink.dtype != torch.float64 or not sink.is_cuda or sink.numel() < blocks * 256:
        raise ValueError("sink: a float64 device tensor of at least blocks * 256 elements")
    f = ctypes.c_double(0.0)
    _check(lib().hctm_dev_mfma_probe(_ptr(sink), blocks, iters, ctypes.byref(f), _stream_ptr(torch)))
    return f.value


def dev_stream_probe(src, dst, n):
    """Enqueue dst[:n] = src[:n] (16-byte accesses) on torch's current stream."""
    torch = _torch()
    for x in (src, dst):
        if x.dtype != torch.float64 or not x.is_cuda or x.numel() < n:
            raise ValueError("src, dst: float64 device tensors of at least n elements")
    _check(lib().hctm_dev_stream_probe(_ptr(src), _ptr(dst), n, _stream_ptr(torch)))


def dev_copy(src, dst, dims, istr, ostr, in_offset=0, out_offset=0):
    torch = _torch()
    r = len(dims)
    d = (ctypes.c_int * r)(*dims)
    i = (ctypes.c_longlong * r)(*istr)
    o = (ctypes.c_longlong * r)(*ostr)
    _need(src, *_box(in_offset, dims, istr), "src")
    _need(dst, *_box(out_offset, dims, ostr), "dst")
    ip = ctypes.c_void_p(src.data_ptr() + 8 * in_offset)
    op = ctypes.c_void_p(dst.data_ptr() + 8 * out_offset)
    _check(lib().hctm_dev_copy(ip, op, r, d, i, o, _stream_ptr(torch)))


def dev_chol_inv(G, Rinv, n, rel, info):
    torch = _torch()
    _need(G, 0, max(n, 0) ** 2, "G")
    _need(Rinv, 0, max(n, 0) ** 2, "Rinv")
    _need(info, 0, 1, "info", "int32")
    _check(lib().hctm_dev_chol_inv(_ptr(G), _ptr(Rinv), n, rel, _ptr(info), _stream_ptr(torch)))


def _jacobi_need(X, m, n, max_sweeps, sv, perm, sweeps, V, pre):
    mn = max(m, 0) * max(n, 0)
    _need(X, 0, mn, "X")
    _need(sv, 0, max(n, 0), "sv")
    _need(perm, 0, max(n, 0), "perm", "int32")
    _need(sweeps, 0, 2 if 2 <= pre < n else 1, "sweeps", "int32")
    if V is not None:
        _need(V, 0, max(n, 0) ** 2, "V")


def dev_jacobi(X, m, n, tol, max_sweeps, sv, perm, sweeps, V=None, vlog=None, pre=0, work=None):
    torch = _torch()
    _jacobi_need(X, m, n, max_sweeps, sv, perm, sweeps, V, pre)
    if vlog is not None:
        _need(vlog, 0, jacobi_log_doubles(n, max_sweeps), "vlog")
    if work is not None:
        _need(work, 0, max(m, 0) * max(n, 0), "work")
    vp = _ptr(V) if V is not None else None
    lp = _ptr(vlog) if vlog is not None else None
    wp = _ptr(work) if work is not None else None
    _check(lib().hctm_dev_jacobi(_ptr(X), m, n, tol, max_sweeps, pre, _ptr(sv), _ptr(perm), _ptr(sweeps), vp, lp,
                                 wp, _stream_ptr(torch)))


def dev_jacobi_noalloc(X, m, n, tol, max_sweeps, sv, perm, sweeps, V=None, pre=0):
    """hctm_dev_jacobi_noalloc: the Jacobi SVD with its scratch in the
    library's static device buffer (no allocation)."""
    torch = _torch()
    _jacobi_need(X, m, n, max_sweeps, sv, perm, sweeps, V, pre)
    vp = _ptr(V) if V is not None else None
    _check(lib().hctm_dev_jacobi_noalloc(_ptr(X), m, n, tol, max_sweeps, pre, _ptr(sv), _ptr(perm), _ptr(sweeps), vp,
                                         _stream_ptr(torch)))


def jacobi_log_doubles(n, max_sweeps):
    return int(lib().hctm_dev_jacobi_log_doubles(n, max_sweeps))


def _hcheck(code, ctx=None):
    if code != CTM_OK:
        msg = lib().hotrg_last_error(ctx).decode(errors="replace")
        raise HctmError(code, msg)


class HOTRG:
    """HOTRG on the double layer of A (d, D, D, D, D) on the GPU, Z2 or
    plain form; probes=True carries the symmetry probes b and |b|; bond=h
    (d^2 x d^2) the impurities of the bond energy; rdm1=True those of the
    one-site RDM.  Work runs
    on torch's current HIP stream; the context allocates its own device
    memory."""

    def __init__(self, A, chi, form="z2", svd_rel_cutoff=1e-12, probes=False, bond=None, rdm1=False,
                 stream=None):
        torch = _torch()
        A = np.ascontiguousarray(A, dtype=np.float64)
        if A.ndim != 5:
            raise ValueError("A must have shape (d, D, D, D, D)")
        self.d, self.D, self.chi, self.form = A.shape[0], A.shape[1], int(chi), form
        o = HotrgOpts()
        _hcheck(lib().hotrg_opts_default(ctypes.byref(o)))
        o.form = CTM_FORM_Z2 if form == "z2" else CTM_FORM_DENSE
        o.svd_rel_cutoff = svd_rel_cutoff
        o.probes = 1 if probes else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        ctx = ctypes.c_void_p()
        _hcheck(lib().hotrg_init(ctypes.byref(ctx), _dptr(A), self.d, self.D, self.chi, ctypes.byref(o)))
        self._ctx = ctx
        if bond is not None:
            h = np.ascontiguousarray(bond, dtype=np.float64).reshape(self.d ** 2, self.d ** 2)
            _hcheck(lib().hotrg_set_bond(self._ctx, _dptr(h)), self._ctx)
        if rdm1:
            _hcheck(lib().hotrg_track_rdm1(self._ctx), self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            lib().hotrg_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, n=1):
        _hcheck(lib().hotrg_step(self._ctx, int(n)), self._ctx)
        return self

    def log_z(self):
        v = ctypes.c_double()
        _hcheck(lib().hotrg_log_z(self._ctx, ctypes.byref(v)), self._ctx)
        return v.value

    def rho1(self):
        """One-site RDM (needs rdm1=True), trace one."""
        rho = np.zeros((self.d, self.d))
        _hcheck(lib().hotrg_rdm1(self._ctx, _dptr(rho)), self._ctx)
        return rho

    def energy(self):
        """<h> on a vertical bond (the operator given as bond=)."""
        v = ctypes.c_double()
        _hcheck(lib().hotrg_energy(self._ctx, ctypes.byref(v)), self._ctx)
        return v.value

    def impurity_ratios(self):
        e, zb, za = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _hcheck(lib().hotrg_sym_error(self._ctx, ctypes.byref(e), ctypes.byref(zb), ctypes.byref(za)), self._ctx)
        return zb.value, za.value

    def sym_error(self):
        zb, za = self.impurity_ratios()
        return abs(zb) / abs(za)

    def records(self):
        n = ctypes.c_int()
        _hcheck(lib().hotrg_num_records(self._ctx, ctypes.byref(n)), self._ctx)
        out = []
        for i in range(n.value):
            cap = 4096
            s = np.zeros(cap)
            m, ke, ko, side = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            disc = np.zeros(2)
            _hcheck(lib().hotrg_record(self._ctx, i, _dptr(s), cap, ctypes.byref(m), ctypes.byref(ke),
                                       ctypes.byref(ko), ctypes.byref(side), _dptr(disc)), self._ctx)
            out.append({"spectrum": s[: m.value].copy(), "kept": (ke.value, ko.value), "side": side.value,
                        "discarded": tuple(disc)})
        return out


class Server:
    """Concurrent CTMRG solves on one GPU (include/hctm_serve.h): solves are
    admitted first come, first served, by their workspace in a device pool
    of pool_bytes, at most max_active at a time, each on its own stream and
    host worker thread inside the library."""

    def __init__(self, pool_bytes, max_active=8):
        s = ctypes.c_void_p()
        _check(lib().ctm_server_create(ctypes.byref(s), int(pool_bytes), int(max_active)))
        self._s = s
        self._d = {}

    def submit(self, A, chi, form="z2", tol=1e-10, max_iter=100):
        """Queue a solve; a complex A runs the complex path (Z2 form)."""
        i = ctypes.c_longlong()
        if np.iscomplexobj(A):
            Ac = np.ascontiguousarray(A, dtype=np.complex128)
            re, im = np.ascontiguousarray(Ac.real), np.ascontiguousarray(Ac.imag)
            d, D = re.shape[0], re.shape[1]
            if form != "z2":
                raise ValueError("complex tensors are solved in the Z2 form")
            _check(lib().ctm_server_submit_complex(self._s, _dptr(re), _dptr(im), d, D, int(chi), float(tol),
                                                   int(max_iter), ctypes.byref(i)))
            self._d[i.value] = (d, True)
            return i.value
        A = np.ascontiguousarray(A, dtype=np.float64)
        d, D = A.shape[0], A.shape[1]
        code = CTM_FORM_Z2 if form == "z2" else CTM_FORM_DENSE
        _check(lib().ctm_server_submit(self._s, _dptr(A), d, D, int(chi), code, float(tol), int(max_iter),
                                       ctypes.byref(i)))
        self._d[i.value] = (d, False)
        return i.value

    def wait(self, sid):
        """Results of solve sid (complex128 RDMs for a complex tensor)."""
        d, cplx = self._d.pop(sid)
        r1, rh, rv = np.zeros((d * d,)), np.zeros((d ** 4,)), np.zeros((d ** 4,))
        info = SolveInfo()
        if cplx:
            i1, ih, iv = np.zeros((d * d,)), np.zeros((d ** 4,)), np.zeros((d ** 4,))
            _check(lib().ctm_server_wait_complex(self._s, sid, _dptr(r1), _dptr(i1), _dptr(rh), _dptr(ih), _dptr(rv),
                                                 _dptr(iv), ctypes.byref(info)))
            r1, rh, rv = r1 + 1j * i1, rh + 1j * ih, rv + 1j * iv
        else:
            _check(lib().ctm_server_wait(self._s, sid, _dptr(r1), _dptr(rh), _dptr(rv), ctypes.byref(info)))
        return {"status": info.status, "message": info.message.decode(errors="replace"),
                "iterations": info.iterations, "converged": bool(info.converged), "delta": info.delta,
                "t_submit": info.t_submit, "t_start": info.t_start, "t_end": info.t_end,
                "rho1": r1.reshape(d, d), "rho2_h": rh.reshape(d * d, d * d), "rho2_v": rv.reshape(d * d, d * d)}

    def load(self):
        w, r = ctypes.c_int(), ctypes.c_int()
        _check(lib().ctm_server_load(self._s, ctypes.byref(w), ctypes.byref(r)))
        return w.value, r.value

    def close(self):
        if getattr(self, "_s", None):
            lib().ctm_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
