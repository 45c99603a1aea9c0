"""Thin ctypes binding of libgdr.so (include/gdr.h): same names, argument
marshalling only. Device vectors are torch tensors (complex128, on the GPU)
passed by data pointer; torch supplies device memory and the stream.

Every numerical step runs in the HIP library; if the library is missing the
import fails loudly.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdr.so")

GDR_OK = 0
GDR_NOT_CONVERGED = 1
GDR_ERR_ARG = -1
GDR_ERR_HIP = -2
GDR_ERR_OOM = -3
GDR_ERR_BREAKDOWN = -4
GDR_ERR_STATE = -5
GDR_PREC_F64 = 0
GDR_PREC_MIXED = 1
GDR_PREC_F32 = 1
GDR_LINKS_F64 = 0
GDR_LINKS_F32 = 1
GDR_LINKS_F16 = 2
K_CLASSES = ["dslash", "gs_project", "gs_update", "gs_close", "small", "combine",
             "recombine", "other"]

SYMBOLS = [
    "gdr_ctx_create", "gdr_ctx_destroy", "gdr_last_error", "gdr_wilson_create",
    "gdr_op_destroy", "gdr_bidiag_create", "gdr_op_size", "gdr_op_link_bytes", "gdr_op_apply",
    "gdr_op_apply_noalloc",
    "gdr_op_tables", "gdr_op_dslash_bench",
    "gdr_params_default",
    "gdr_solve_dr_sh", "gdr_solve_proj_sh", "gdr_solve", "gdr_defl_k", "gdr_defl_export",
    "gdr_defl_import", "gdr_defl_destroy", "gdr_tune_load", "gdr_tune_report",
    "gdr_solve_many",
]


class gdr_c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class gdr_params(ctypes.Structure):
    _fields_ = [("m_dr", ctypes.c_int), ("k", ctypes.c_int), ("m_proj", ctypes.c_int),
                ("tol", ctypes.c_double), ("tol_extra", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int),
                ("batch", ctypes.c_int), ("related_rhs", ctypes.c_int),
                ("max_refine", ctypes.c_int), ("profile", ctypes.c_int),
                ("m_clean", ctypes.c_int), ("proj_k", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("galerkin", ctypes.c_int),
                ("sstep", ctypes.c_int), ("sstep_reorth", ctypes.c_double),
                ("refine_floor", ctypes.c_double), ("persistent", ctypes.c_int)]


class gdr_stats(ctypes.Structure):
    _fields_ = [("cycles_dr", ctypes.c_int), ("cycles_extra", ctypes.c_int),
                ("cycles_proj", ctypes.c_int), ("cycles_cleanup", ctypes.c_int),
                ("mvp_dr", ctypes.c_int64), ("mvp_extra", ctypes.c_int64),
                ("mvp_proj", ctypes.c_int64), ("mvp_fp64", ctypes.c_int64),
                ("mvp_cleanup", ctypes.c_int64), ("t_total", ctypes.c_double),
                ("t_phase", ctypes.c_double * 8), ("resid", ctypes.POINTER(ctypes.c_double)),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int),
                ("hist_len", ctypes.c_int), ("theta", ctypes.POINTER(gdr_c64)),
                ("theta_cap", ctypes.c_int), ("theta_len", ctypes.c_int),
                ("k_ms", ctypes.c_double * 8), ("k_bytes", ctypes.c_double * 8),
                ("k_flops", ctypes.c_double * 8), ("k_launches", ctypes.c_int64 * 8),
                ("resid_main", ctypes.c_double)]


class GdrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gdr error %d: %s" % (code, msg))
        self.code = code


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libgdr.so not built: run paper_0707_0502_amd.build (%s)" % path)
    lib = ctypes.CDLL(path)
    vp, ip, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.gdr_ctx_create.argtypes = [ip, vp, ctypes.POINTER(vp)]
    lib.gdr_ctx_destroy.argtypes = [vp]
    lib.gdr_ctx_destroy.restype = None
    lib.gdr_last_error.argtypes = [vp]
    lib.gdr_last_error.restype = ctypes.c_char_p
    lib.gdr_wilson_create.argtypes = [vp, ctypes.POINTER(ip), ctypes.POINTER(ip), ctypes.c_double,
                                      vp, ip, ip, ctypes.POINTER(vp)]
    lib.gdr_op_destroy.argtypes = [vp]
    lib.gdr_op_destroy.restype = None
    lib.gdr_bidiag_create.argtypes = [vp, i64, vp, vp, ctypes.POINTER(vp)]
    lib.gdr_op_size.argtypes = [vp]
    lib.gdr_op_size.restype = i64
    lib.gdr_op_link_bytes.argtypes = [vp, ip]
    lib.gdr_op_apply.argtypes = [vp, gdr_c64, vp, vp, ip, ip]
    lib.gdr_op_apply_noalloc.argtypes = [vp, gdr_c64, vp, vp, ip, ip]
    lib.gdr_op_tables.argtypes = [vp, vp, vp, vp]
    lib.gdr_op_dslash_bench.argtypes = [vp, ip, ip, ip, ip, vp]
    lib.gdr_params_default.argtypes = [ctypes.POINTER(gdr_params)]
    lib.gdr_params_default.restype = None
    lib.gdr_solve_dr_sh.argtypes = [vp, ip, ctypes.POINTER(gdr_c64), vp, vp,
                                    ctypes.POINTER(gdr_params), ctypes.POINTER(gdr_stats),
                                    ctypes.POINTER(vp)]
    lib.gdr_solve_proj_sh.argtypes = [vp, vp, ip, ctypes.POINTER(gdr_c64), ip, vp, vp,
                                      ctypes.POINTER(gdr_params), ctypes.POINTER(gdr_stats)]
    lib.gdr_solve.argtypes = [vp, ip, ctypes.POINTER(gdr_c64), ip, vp, vp,
                              ctypes.POINTER(gdr_params), ctypes.POINTER(gdr_stats)]
    lib.gdr_defl_k.argtypes = [vp]
    lib.gdr_defl_export.argtypes = [vp, vp, vp]
    lib.gdr_defl_import.argtypes = [vp, ip, vp, vp, ip, ctypes.POINTER(vp)]
    lib.gdr_defl_destroy.argtypes = [vp]
    lib.gdr_defl_destroy.restype = None
    lib.gdr_solve_many.argtypes = [ip, ctypes.POINTER(vp), ip, ctypes.POINTER(gdr_c64), ip,
                                   ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(gdr_params), ctypes.POINTER(gdr_stats)]
    lib.gdr_tune_load.argtypes = [ctypes.c_char_p]
    lib.gdr_tune_report.argtypes = [ctypes.c_char_p, i64]
    lib.gdr_tune_report.restype = i64
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _ptr(t):
    """Device or host address of a torch tensor / numpy array (contiguous)."""
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        if not t.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return ctypes.c_void_p(t.ctypes.data)
    raise TypeError(type(t))


def _dev(t, name, numel):
    """Address of a device vector argument, after the checks the C-ABI relies
    on: a contiguous CUDA complex128 tensor of exactly `numel` entries (the
    library reads and writes that many; a host buffer would fault the GPU)."""
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError("%s must be a CUDA tensor (device memory), got %s" % (name, type(t).__name__))
    if str(t.dtype) != "torch.complex128":
        raise TypeError("%s must be complex128, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d entries, expected %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _host(a, name, numel):
    """Address of a host complex128 array argument of exactly `numel` entries."""
    if not isinstance(a, np.ndarray):
        raise TypeError("%s must be a numpy array (host memory), got %s" % (name, type(a).__name__))
    if a.dtype != np.complex128:
        raise TypeError("%s must be complex128, got %s" % (name, a.dtype))
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("%s must be C-contiguous" % name)
    if a.size != numel:
        raise ValueError("%s has %d entries, expected %d" % (name, a.size, numel))
    return ctypes.c_void_p(a.ctypes.data)


def _nrhs(B, n):
    """Number of right-hand sides in the device tensor B (a positive multiple of n entries)."""
    if not (hasattr(B, "is_cuda") and B.is_cuda):
        raise TypeError("B must be a CUDA tensor (device memory), got %s" % type(B).__name__)
    if B.numel() == 0 or B.numel() % n:
        raise ValueError("B has %d entries, not a positive multiple of n = %d" % (B.numel(), n))
    return B.numel() // n


def _stats(stats, nrhs, ns):
    """The gdr_stats pointer of a Stats object sized for nrhs x ns residuals."""
    if stats is None:
        return None
    if ns > 0 and stats.resid.shape != (nrhs, ns):
        raise ValueError("Stats holds %s residuals, the solve writes (%d, %d)"
                         % (stats.resid.shape, nrhs, ns))
    return ctypes.byref(stats.s)


def _sig(sigmas):
    arr = (gdr_c64 * len(sigmas))()
    for i, s in enumerate(sigmas):
        s = complex(s)
        arr[i] = gdr_c64(s.real, s.imag)
    return arr


class Ctx:
    def __init__(self, handle):
        self.h = handle

    def error(self):
        return lib().gdr_last_error(self.h).decode()

    def check(self, rc):
        if rc < 0:
            raise GdrError(rc, self.error())
        return rc


class Op:
    def __init__(self, ctx, handle, dims=None, n=None):
        self.ctx, self.h = ctx, handle
        self.dims = tuple(dims) if dims is not None else None
        self.n = 12 * int(np.prod(dims)) if dims is not None else int(n)


class Defl:
    def __init__(self, op, handle):
        self.op, self.h = op, handle


class Stats:
    """Caller-owned buffers for gdr_stats (resid, per-cycle history, theta)."""

    def __init__(self, nrhs=1, ns=1, hist_cap=20000, theta_cap=20000):
        self.resid = np.zeros((nrhs, ns))
        self.hist_buf = np.zeros((hist_cap, 5))
        self.theta_buf = np.zeros(theta_cap, dtype=np.complex128)
        self.s = gdr_stats()
        self.s.resid = self.resid.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s.hist = self.hist_buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s.hist_cap = hist_cap
        self.s.theta = ctypes.cast(self.theta_buf.ctypes.data, ctypes.POINTER(gdr_c64))
        self.s.theta_cap = theta_cap

    @property
    def hist(self):
        return self.hist_buf[:self.s.hist_len]

    @property
    def theta(self):
        return self.theta_buf[:self.s.theta_len]

    def as_dict(self):
        s = self.s
        return dict(cycles_dr=s.cycles_dr, cycles_extra=s.cycles_extra,
                    cycles_proj=s.cycles_proj, cycles_cleanup=s.cycles_cleanup,
                    mvp_dr=s.mvp_dr, mvp_extra=s.mvp_extra, mvp_proj=s.mvp_proj,
                    mvp_fp64=s.mvp_fp64, mvp_cleanup=s.mvp_cleanup, t_total=s.t_total,
                    t_phase=list(s.t_phase), resid_main=s.resid_main)

    def kernels(self):
        s = self.s
        return {K_CLASSES[i]: dict(ms=s.k_ms[i], bytes=s.k_bytes[i], flops=s.k_flops[i],
                                   launches=s.k_launches[i]) for i in range(8)}


def gdr_params_default(**kw):
    p = gdr_params()
    lib().gdr_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def gdr_ctx_create(device=0, stream=None):
    h = ctypes.c_void_p()
    rc = lib().gdr_ctx_create(device, ctypes.c_void_p(stream or 0), ctypes.byref(h))
    if rc != GDR_OK:
        raise GdrError(rc, "gdr_ctx_create failed")
    return Ctx(h)


def gdr_ctx_destroy(ctx):
    lib().gdr_ctx_destroy(ctx.h)


def gdr_last_error(ctx):
    return ctx.error()


def gdr_wilson_create(ctx, dims, bc, kappa, links, link_storage=GDR_LINKS_F32):
    """links: numpy (host) or torch (device) complex128 [4][Lt][Lz][Ly][Lx][3][3]."""
    if len(dims) != 4 or len(bc) != 4:
        raise ValueError("dims and bc need 4 entries")
    d = (ctypes.c_int * 4)(*dims)
    b = (ctypes.c_int * 4)(*bc)
    on_dev = int(hasattr(links, "is_cuda") and links.is_cuda)
    nl = 36 * int(np.prod(dims))
    ptr = _dev(links, "links", nl) if on_dev else _host(links, "links", nl)
    h = ctypes.c_void_p()
    ctx.check(lib().gdr_wilson_create(ctx.h, d, b, float(kappa), ptr, on_dev,
                                      link_storage, ctypes.byref(h)))
    return Op(ctx, h, dims)


def gdr_bidiag_create(ctx, diag, super_):
    """Bidiagonal operator from host sequences of n and n-1 complex entries."""
    d = np.ascontiguousarray(diag, dtype=np.complex128)
    e = np.ascontiguousarray(super_, dtype=np.complex128)
    h = ctypes.c_void_p()
    ctx.check(lib().gdr_bidiag_create(ctx.h, len(d), _ptr(d), _ptr(e) if len(e) else None,
                                      ctypes.byref(h)))
    return Op(ctx, h, n=len(d))


def gdr_op_destroy(op):
    lib().gdr_op_destroy(op.h)


def gdr_op_size(op):
    return lib().gdr_op_size(op.h)


def gdr_op_link_bytes(op, precision):
    return lib().gdr_op_link_bytes(op.h, precision)


def gdr_op_apply(op, sigma, x, y, nvec=1, precision=GDR_PREC_F64):
    s = complex(sigma)
    want = nvec * op.n if nvec > 0 else None   # nvec = 0 touches nothing
    px, py = _dev(x, "x", want), _dev(y, "y", want)
    return op.ctx.check(lib().gdr_op_apply(op.h, gdr_c64(s.real, s.imag), px, py, nvec, precision))


def gdr_op_apply_noalloc(op, sigma, x, y, nvec=1, precision=GDR_PREC_F64):
    s = complex(sigma)
    want = nvec * op.n if nvec > 0 else None
    px, py = _dev(x, "x", want), _dev(y, "y", want)
    return op.ctx.check(lib().gdr_op_apply_noalloc(op.h, gdr_c64(s.real, s.imag), px, py, nvec,
                                                   precision))


def gdr_op_tables(op):
    vol = op.n // 12
    eo = np.zeros(vol, np.int32)
    nbr = np.zeros((vol, 8), np.int32)
    sign = np.zeros((vol, 8), np.int8)
    op.ctx.check(lib().gdr_op_tables(op.h, _ptr(eo), _ptr(nbr), _ptr(sign)))
    return eo, nbr, sign


def gdr_op_dslash_bench(op, precision, nvec, nsets, reps):
    """Per-launch milliseconds of `reps` operator launches on nvec vectors in the
    internal layout, rotating over nsets buffer sets."""
    ms = np.zeros(reps, np.float64)
    op.ctx.check(lib().gdr_op_dslash_bench(op.h, precision, nvec, nsets, reps, _ptr(ms)))
    return ms


def gdr_solve_dr_sh(op, sigmas, b, x, params, stats=None, want_defl=True):
    ns = len(sigmas)
    # ns < 1 is the library's to reject (GDR_ERR_ARG); no size to check then
    pb, px = _dev(b, "b", op.n), _dev(x, "x", ns * op.n if ns > 0 else None)
    pst = _stats(stats, 1, ns)
    h = ctypes.c_void_p()
    rc = op.ctx.check(lib().gdr_solve_dr_sh(
        op.h, ns, _sig(sigmas), pb, px, ctypes.byref(params), pst,
        ctypes.byref(h) if want_defl else None))
    return rc, (Defl(op, h) if want_defl and h.value else None)


def gdr_solve_proj_sh(op, defl, sigmas, B, X, params, stats=None):
    ns = len(sigmas)
    nrhs = _nrhs(B, op.n)
    pB, pX = _dev(B, "B", nrhs * op.n), _dev(X, "X", nrhs * ns * op.n if ns > 0 else None)
    pst = _stats(stats, nrhs, ns)
    return op.ctx.check(lib().gdr_solve_proj_sh(
        op.h, defl.h, ns, _sig(sigmas), nrhs, pB, pX, ctypes.byref(params), pst))


def gdr_solve(op, sigmas, B, X, params, stats=None):
    ns = len(sigmas)
    nrhs = _nrhs(B, op.n)
    pB, pX = _dev(B, "B", nrhs * op.n), _dev(X, "X", nrhs * ns * op.n if ns > 0 else None)
    pst = _stats(stats, nrhs, ns)
    return op.ctx.check(lib().gdr_solve(
        op.h, ns, _sig(sigmas), nrhs, pB, pX, ctypes.byref(params), pst))


def gdr_solve_many(ops, sigmas, Bs, Xs, params, stats=None):
    """Independent problems on several lattices: ops[l] with right-hand sides
    Bs[l] (nrhs x n_l) into Xs[l] (nrhs x ns x n_l); stats: None or one Stats
    per lattice. params.persistent selects the batched first phase."""
    nops = len(ops)
    if nops < 1 or len(Bs) != nops or len(Xs) != nops:
        raise ValueError("one right-hand side and one solution buffer per operator")
    ns = len(sigmas)
    nrhs = _nrhs(Bs[0], ops[0].n)
    hv = (ctypes.c_void_p * nops)(*[o.h for o in ops])
    pb = (ctypes.c_void_p * nops)()
    px = (ctypes.c_void_p * nops)()
    for l, o in enumerate(ops):
        pb[l] = _dev(Bs[l], "B[%d]" % l, nrhs * o.n).value
        px[l] = _dev(Xs[l], "X[%d]" % l, nrhs * ns * o.n if ns > 0 else None).value
    sa = None
    if stats is not None:
        if len(stats) != nops:
            raise ValueError("one Stats per operator")
        sa = (gdr_stats * nops)()
        for l, s_ in enumerate(stats):
            _stats(s_, nrhs, ns)
            sa[l] = s_.s
    rc = lib().gdr_solve_many(nops, hv, ns, _sig(sigmas), nrhs, pb, px, ctypes.byref(params),
                              sa)
    if sa is not None:
        for l, s_ in enumerate(stats):
            ctypes.memmove(ctypes.byref(s_.s), ctypes.byref(sa[l]), ctypes.sizeof(gdr_stats))
    return ops[0].ctx.check(rc)


def gdr_defl_k(defl):
    return lib().gdr_defl_k(defl.h)


def gdr_defl_export(defl, V=None, Hbar=None):
    """V: device tensor of (k+1)*n entries; Hbar: host array of (k+1)*k entries
    (column-major); either may be None."""
    k = gdr_defl_k(defl)
    pV = _dev(V, "V", (k + 1) * defl.op.n) if V is not None else None
    pH = _host(Hbar, "Hbar", (k + 1) * k) if Hbar is not None else None
    return defl.op.ctx.check(lib().gdr_defl_export(defl.h, pV, pH))


def gdr_defl_import(op, k, V, Hbar, precision=GDR_PREC_F64):
    pV = _dev(V, "V", (k + 1) * op.n)
    pH = _host(Hbar, "Hbar", (k + 1) * k)
    h = ctypes.c_void_p()
    op.ctx.check(lib().gdr_defl_import(op.h, k, pV, pH, precision, ctypes.byref(h)))
    return Defl(op, h)


def gdr_defl_destroy(defl):
    lib().gdr_defl_destroy(defl.h)


def gdr_tune_load(path):
    """Read launch-tuning decisions from a cache file; returns the lines taken
    (GDR_ERR_ARG if the file cannot be opened)."""
    return lib().gdr_tune_load(os.fsencode(path))


def gdr_tune_report():
    """The launch-tuning decisions so far, one line each."""
    n = lib().gdr_tune_report(None, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    lib().gdr_tune_report(buf, n + 1)
    return buf.value.decode()
