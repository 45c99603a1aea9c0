"""The largest parameters the C-ABI accepts, on the 4^4 lattice (n = 3072):
Krylov subspaces of m = 64 for GMRES-DR-Sh and GMRES-Proj-Sh, 16 shifts, and
k up to m - 1. Plain FP64 runs the same algorithm as the oracle (equal cycle
and product counts, solutions to 1e-10); mixed precision reaches the
tolerance for every (shift, RHS) pair; one past each limit is rejected."""
import numpy as np
import pytest

import synth
from oracle import gmres, wilson
from tests.gpu_common import config_data, dev, empty, host, make_op, rel, say

pytestmark = pytest.mark.gpu

SIG16 = list(np.linspace(0.0, -0.3, 16))


@pytest.fixture(scope="module")
def c1_two_rhs():
    cfg, links, kappa, B = config_data("C1")
    b2 = synth.rhs_z4(cfg["dims"], 4242).ravel()
    B2 = np.stack([B[0], b2])
    return cfg, links, kappa, B2, wilson.WilsonOperator(links, kappa)


def _params(precision, m_dr, k, m_proj, tol, tol_extra):
    from paper_0707_0502_amd import gdr
    return gdr.gdr_params_default(m_dr=m_dr, k=k, m_proj=m_proj, tol=tol, tol_extra=tol_extra,
                                  precision=precision)


def test_m64_16_shifts_fp64_parity(c1_two_rhs):
    """GMRES-DR(64,30)-Sh on RHS 1, extra RHS, GMRES(64)-Proj(30)-Sh on RHS 2,
    16 shifts, FP64: the same products as the oracle, the same solutions and
    the same true residuals."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A = c1_two_rhs
    sig = np.array(SIG16, complex)
    tol, tol_extra = 1e-10, 1e-5
    say("oracle m = 64, 16 shifts, 2 RHS ...")
    ref = gmres.solve_all(A, B, sig, 64, 30, 64, tol, tol_extra)
    op = make_op(links, kappa)
    n = op.n
    X = empty(2 * len(sig) * n)
    st = gdr.Stats(2, len(sig))
    rc = gdr.gdr_solve(op, SIG16, dev(B.ravel()), X, _params(gdr.GDR_PREC_F64, 64, 30, 64, tol,
                                                              tol_extra), st)
    d = st.as_dict()
    say("gpu rc", rc, d)
    # the corrected residuals of the non-base shifts are as accurate as the
    # extra right-hand side (1e-5), so the FP64 path can end above tol: the
    # status follows the oracle's true residuals
    expect = gdr.GDR_OK if ref["resid"].max() <= tol else gdr.GDR_NOT_CONVERGED
    assert rc == expect
    Xh = host(X).reshape(2, len(sig), n)
    say("gpu resid", np.array2string(st.resid, precision=2))
    say("oracle resid", np.array2string(ref["resid"], precision=2))
    worst = 0.0
    for j in range(2):
        for i in range(len(sig)):
            worst = max(worst, rel(Xh[j, i], ref["X"][j, i]))
            # residuals far below tol carry the rounding of the last cycle
            assert abs(st.resid[j, i] - ref["resid"][j, i]) <= 1e-3 * ref["resid"][j, i] + 0.2 * tol
    say("max relative difference to the oracle %.2e" % worst)
    assert worst <= 1e-10
    assert d["mvp_dr"] == ref["runs"][0]["mvps"]
    assert d["mvp_extra"] == ref["extra"]["mvps"]
    assert d["mvp_proj"] == ref["runs"][1]["mvps"]
    gdr.gdr_op_destroy(op)


@pytest.mark.parametrize("k", [30, 63])
def test_m64_16_shifts_mixed(c1_two_rhs, k):
    """The same limits in mixed precision (s-step blocks of 8 across the
    whole 64-column basis), k = 30 and k = m - 1 = 63: every true FP64
    residual at most 1e-8."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A = c1_two_rhs
    op = make_op(links, kappa)
    n = op.n
    X = empty(2 * len(SIG16) * n)
    st = gdr.Stats(2, len(SIG16))
    rc = gdr.gdr_solve(op, SIG16, dev(B.ravel()), X,
                       _params(gdr.GDR_PREC_MIXED, 64, k, 64, 1e-8, 1e-4), st)
    say("k", k, "rc", rc, "max resid %.2e" % st.resid.max(), st.as_dict())
    assert rc == gdr.GDR_OK
    assert st.resid.max() <= 1e-8
    Xh = host(X).reshape(2, len(SIG16), n)
    for j, i in ((0, 0), (1, 15)):
        r = np.linalg.norm(gmres.true_residual(A, B[j], Xh[j, i], SIG16[i])) / np.linalg.norm(B[j])
        assert r <= 1e-8 * 1.01
    gdr.gdr_op_destroy(op)


def test_one_past_the_limits(c1_two_rhs):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A = c1_two_rhs
    op = make_op(links, kappa)
    n = op.n
    for sig, p in ((SIG16, _params(gdr.GDR_PREC_F64, 65, 30, 64, 1e-8, 1e-4)),
                   (SIG16, _params(gdr.GDR_PREC_F64, 64, 30, 65, 1e-8, 1e-4)),
                   (SIG16, _params(gdr.GDR_PREC_F64, 64, 64, 64, 1e-8, 1e-4)),
                   (SIG16 + [-0.31], _params(gdr.GDR_PREC_F64, 64, 30, 64, 1e-8, 1e-4))):
        X = empty(2 * len(sig) * n)
        with pytest.raises(gdr.GdrError) as e:
            gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, gdr.Stats(2, len(sig)))
        assert e.value.code == gdr.GDR_ERR_ARG
    gdr.gdr_op_destroy(op)
