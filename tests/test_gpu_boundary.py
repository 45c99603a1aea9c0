"""The C-ABI's status contract and error paths on the GPU, through the
library:

* non-finite right-hand sides and shifts are rejected (GDR_ERR_ARG) by all
  three solve calls before any iteration;
* a host pointer where the header asks for device memory is rejected by the
  library itself (GDR_ERR_ARG), below the binding's own checks;
* a shifted system that is exactly singular gives GDR_ERR_BREAKDOWN: the
  bidiagonal matrix of Example 1 with n = 8 < m, so the Krylov space fills in
  one cycle, and a shift equal to a diagonal entry (an eigenvalue of the
  upper bidiagonal matrix; Sec. 2.1's shifted least-squares problems then
  have a singular square part);
* max_cycles = 1 returns GDR_NOT_CONVERGED with every true residual filled;
* a deflation pair exported and imported again (the resume path of the
  deflation handle, Sec. 4: GMRES-Proj-Sh reuses V_{k+1} and H_bar_k) gives
  the same products and solutions as the original handle, bit for bit.
"""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import config_data, ctx, dev, empty, host, make_op, say

pytestmark = pytest.mark.gpu


def _p(cfg, prec, **kw):
    from paper_0707_0502_amd import gdr
    p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"], tol=cfg["tol"],
                               tol_extra=cfg["tol_extra"], precision=prec)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.fixture(scope="module")
def c1():
    cfg, links, kappa, B = config_data("C1")
    return cfg, links, kappa, B


def test_nonfinite_rhs_rejected(c1):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = c1
    op = make_op(links, kappa)
    n, sig = op.n, cfg["sigmas"]
    ns = len(sig)
    p = _p(cfg, gdr.GDR_PREC_F64, max_cycles=3)
    _, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), empty(ns * n), p)
    assert defl is not None
    for bad in (np.nan, np.inf, complex(0, np.nan)):
        b = B[0].copy()
        b[n // 3] = bad
        say("non-finite entry", bad)
        with pytest.raises(gdr.GdrError) as e:
            gdr.gdr_solve_dr_sh(op, sig, dev(b), empty(ns * n), p)
        assert e.value.code == gdr.GDR_ERR_ARG
        B2 = np.stack([B[0], b])
        for prec in (gdr.GDR_PREC_F64, gdr.GDR_PREC_MIXED):
            with pytest.raises(gdr.GdrError) as e:
                gdr.gdr_solve(op, sig, dev(B2.ravel()), empty(2 * ns * n), _p(cfg, prec, max_cycles=3))
            assert e.value.code == gdr.GDR_ERR_ARG
            with pytest.raises(gdr.GdrError) as e:
                gdr.gdr_solve_proj_sh(op, defl, sig, dev(B2.ravel()), empty(2 * ns * n),
                                      _p(cfg, prec, max_cycles=3))
            assert e.value.code == gdr.GDR_ERR_ARG
    for bad in (np.nan, np.inf):
        with pytest.raises(gdr.GdrError) as e:
            gdr.gdr_solve_dr_sh(op, [0.0, complex(bad, 0)], dev(B[0]), empty(2 * n), p)
        assert e.value.code == gdr.GDR_ERR_ARG
    # the context still works after the rejections
    st = gdr.Stats(1, ns)
    rc, d2 = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), empty(ns * n), p, st, want_defl=False)
    assert rc in (gdr.GDR_OK, gdr.GDR_NOT_CONVERGED) and np.isfinite(st.resid).all()
    gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)


class _HipAttr(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int), ("device", ctypes.c_int),
                ("devicePointer", ctypes.c_void_p), ("hostPointer", ctypes.c_void_p),
                ("isManaged", ctypes.c_int), ("allocationFlags", ctypes.c_uint)]


def _runtime_sees_host(addr):
    """The HIP runtime's own classification of an address: True when it is not
    device (2) or managed (3) memory."""
    hip = ctypes.CDLL("libamdhip64.so")
    a = _HipAttr()
    rc = hip.hipPointerGetAttributes(ctypes.byref(a), ctypes.c_void_p(addr))
    if rc != 0:
        hip.hipGetLastError()
        return True
    return a.type not in (2, 3)


def test_host_pointer_rejected_by_the_library(c1):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = c1
    op = make_op(links, kappa)
    n = op.n
    xh = np.ascontiguousarray(B[0])
    yd = empty(n)
    if not _runtime_sees_host(xh.ctypes.data):
        pytest.skip("the runtime reports this host buffer as device memory")
    lib = gdr.lib()
    rc = lib.gdr_op_apply(op.h, gdr.gdr_c64(0, 0), ctypes.c_void_p(xh.ctypes.data),
                          ctypes.c_void_p(yd.data_ptr()), 1, gdr.GDR_PREC_F64)
    say("host x:", rc, gdr.gdr_last_error(op.ctx))
    assert rc == gdr.GDR_ERR_ARG
    p = _p(cfg, gdr.GDR_PREC_F64, max_cycles=2)
    sig = (gdr.gdr_c64 * 2)(gdr.gdr_c64(0, 0), gdr.gdr_c64(-0.1, 0))
    xd = empty(2 * n)
    rc = lib.gdr_solve_dr_sh(op.h, 2, sig, ctypes.c_void_p(xh.ctypes.data),
                             ctypes.c_void_p(xd.data_ptr()), ctypes.byref(p), None, None)
    assert rc == gdr.GDR_ERR_ARG
    gdr.gdr_op_destroy(op)


def test_singular_shift_is_a_breakdown():
    from paper_0707_0502_amd import gdr
    n = 8
    d = np.arange(1, n + 1).astype(complex)
    e = np.ones(n - 1, complex)
    op = gdr.gdr_bidiag_create(ctx(), d, e)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    p = gdr.gdr_params_default(m_dr=10, k=3, m_proj=10, tol=1e-10, precision=gdr.GDR_PREC_F64)
    # regular shifts: solved exactly in one cycle (lucky breakdown at n)
    st = gdr.Stats(1, 2)
    rc, defl = gdr.gdr_solve_dr_sh(op, [0.0, -0.5], dev(b), empty(2 * n), p, st)
    say("regular shifts rc", rc, "resid", st.resid)
    assert rc == gdr.GDR_OK and st.resid.max() <= 1e-12
    # sigma_2 = 3, a diagonal entry: M - 3 I is singular
    with pytest.raises(gdr.GdrError) as err:
        gdr.gdr_solve_dr_sh(op, [0.0, 3.0], dev(b), empty(2 * n), p, gdr.Stats(1, 2))
    say("singular shift:", err.value)
    assert err.value.code == gdr.GDR_ERR_BREAKDOWN
    gdr.gdr_op_destroy(op)


def test_max_cycles_one_not_converged(c1):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = c1
    op = make_op(links, kappa)
    n, sig = op.n, cfg["sigmas"]
    ns = len(sig)
    st = gdr.Stats(1, ns)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), empty(ns * n),
                                   _p(cfg, gdr.GDR_PREC_F64, max_cycles=1), st)
    say("FP64 one cycle: rc", rc, "resid", st.resid)
    assert rc == gdr.GDR_NOT_CONVERGED
    assert st.s.cycles_dr == 1 and st.s.mvp_dr == cfg["m_dr"]
    assert np.isfinite(st.resid).all() and (st.resid > 0).all() and st.resid.max() > cfg["tol"]
    gdr.gdr_defl_destroy(defl)
    # mixed precision with no refinement round
    B2 = np.stack([B[0], B[0][::-1].copy()])
    st = gdr.Stats(2, ns)
    rc = gdr.gdr_solve(op, sig, dev(B2.ravel()), empty(2 * ns * n),
                       _p(cfg, gdr.GDR_PREC_MIXED, max_cycles=1, max_refine=0), st)
    say("mixed one cycle: rc", rc, "resid", st.resid)
    assert rc == gdr.GDR_NOT_CONVERGED
    assert np.isfinite(st.resid).all() and (st.resid > 0).all() and st.resid.max() > cfg["tol"]
    gdr.gdr_op_destroy(op)


@pytest.mark.parametrize("prec", [0, 1])
def test_defl_export_import_roundtrip(prec):
    """GMRES-Proj-Sh on two later right-hand sides with the handle from the
    first solve and with a handle rebuilt from its export: identical counts
    and solutions (the export and import are exact: FP64 stays FP64, the FP32
    basis widens to FP64 and rounds back to the same values)."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = config_data("C2")
    op = make_op(links, kappa)
    n, sig = op.n, cfg["sigmas"]
    ns = len(sig)
    p = _p(cfg, prec)
    if prec == gdr.GDR_PREC_MIXED:
        p.tol, p.tol_extra = 1e-8, 1e-4
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), empty(ns * n), p)
    k = gdr.gdr_defl_k(defl)
    assert k == cfg["k"]
    V = empty((k + 1) * n)
    Hb = np.zeros((k, k + 1), complex)
    gdr.gdr_defl_export(defl, V, Hb)
    d2 = gdr.gdr_defl_import(op, k, V, Hb, prec)
    Bl = dev(B[1:3].ravel())
    out = []
    for d in (defl, d2):
        X = empty(2 * ns * n)
        st = gdr.Stats(2, ns)
        rc = gdr.gdr_solve_proj_sh(op, d, sig, Bl, X, p, st)
        out.append((rc, st.as_dict(), host(X), st.resid.copy()))
        say("prec", prec, "rc", rc, {k_: v for k_, v in st.as_dict().items() if k_.startswith("mvp")})
    (rc1, s1, X1, r1), (rc2, s2, X2, r2) = out
    assert rc1 == rc2
    for key in ("mvp_extra", "mvp_proj", "mvp_fp64", "mvp_cleanup", "cycles_proj", "cycles_extra"):
        assert s1[key] == s2[key], key
    assert s1["mvp_extra"] > 0
    assert np.array_equal(X1, X2)
    assert np.array_equal(r1, r2)
    gdr.gdr_defl_destroy(d2)
    gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)
