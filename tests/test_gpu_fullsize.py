"""The 24^3x48 workload at full size, in the configuration bench.py times:
12 Z4 right-hand sides x 6 shifts, GMRES-DR(60,20)-Sh on the first, the
extra right-hand side, then GMRES(40)-Proj(20)-Sh batched over the other 11
with the correction, mixed precision (FP32 operator, Gram-Schmidt and basis;
FP64 small problems, accumulation and refinement), tol 1e-8.

Checked by properties that hold at any size, since the oracle cannot solve
this system in reasonable time: every FP64 true residual the library reports
is at most the tolerance, and for sampled (right-hand side, shift) pairs the
oracle's own operator recomputes the true residual from the returned
solution. The FP32 operator itself, launched over 12 vectors at once as in
the solve, is compared with the oracle's operator on sampled vectors. The
16^3x32 workload (one right-hand side) is solved in mixed precision and in
plain FP64, and the two solutions are compared."""
import numpy as np
import pytest

from oracle import gmres, wilson
from tests.gpu_common import config_data, ctx, dev, empty, host, make_op, say, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4():
    say("C4 inputs ...")
    cfg, links, kappa, B = config_data("C4")
    say("C4 inputs ready")
    return cfg, links, kappa, B


@pytest.mark.timeout(900)
def test_c4_operator_batch_of_12_against_oracle(c4):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = c4
    op = make_op(links, kappa)
    n = op.n
    sigma = -0.05
    X = B[:12]
    y = empty(12 * n)
    gdr.gdr_op_apply(op, sigma, dev(X.ravel()), y, 12, gdr.GDR_PREC_F32)
    got = host(y).reshape(12, n)
    dims = cfg["dims"]
    for v in (0, 11):
        say("oracle operator on vector", v)
        ref = wilson.apply_A(links, kappa, X[v].reshape(tuple(dims[::-1]) + (4, 3)), sigma).ravel()
        err = np.abs(got[v] - ref).max() / np.abs(ref).max()
        say("vector", v, "max error / max |ref| = %.2e" % err)
        assert err <= 1e-6
    gdr.gdr_op_destroy(op)


@pytest.mark.timeout(900)
def test_c4_mixed_batched_solve(c4):
    from paper_0707_0502_amd import gdr
    torch = torch_mod()
    cfg, links, kappa, B = c4
    op = make_op(links, kappa)
    n = op.n
    sig = list(cfg["sigmas"])
    nrhs, ns = B.shape[0], len(sig)
    Bd = dev(B.ravel())
    X = torch.zeros(nrhs * ns * n, dtype=torch.complex128, device="cuda")
    p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"],
                               tol=cfg["tol"], tol_extra=cfg["tol_extra"],
                               precision=gdr.GDR_PREC_MIXED, batch=1)
    st = gdr.Stats(nrhs, ns)
    say("C4 mixed solve ...")
    rc = gdr.gdr_solve(op, sig, Bd, X, p, st)
    say("C4 rc", rc, "max resid %.2e" % st.resid.max(), st.as_dict())
    assert rc == gdr.GDR_OK
    assert st.resid.shape == (nrhs, ns)
    assert st.resid.max() <= cfg["tol"]
    # the first right-hand side by GMRES-DR-Sh, the rest batched by Proj-Sh
    d = st.as_dict()
    assert d["mvp_dr"] > 0 and d["mvp_proj"] > 0 and d["mvp_extra"] > 0
    A = wilson.WilsonOperator(links, kappa)
    for j, i in ((0, 0), (nrhs - 1, ns - 1), (5, 2)):
        x = X[(j * ns + i) * n:(j * ns + i + 1) * n].cpu().numpy()
        res = np.linalg.norm(gmres.true_residual(A, B[j], x, sig[i])) / np.linalg.norm(B[j])
        say("oracle true residual rhs %d shift %d: %.3e (library %.3e)" % (j, i, res, st.resid[j, i]))
        assert res <= cfg["tol"] * 1.01
        assert abs(res - st.resid[j, i]) <= 1e-3 * cfg["tol"]
    gdr.gdr_op_destroy(op)


@pytest.mark.timeout(900)
def test_c3_mixed_against_fp64():
    """16^3x32, one Gaussian right-hand side x 6 shifts, GMRES-DR(60,20)-Sh:
    the mixed-precision solve and the plain FP64 solve both reach the
    tolerance for every shift (library FP64 residuals, and the oracle's
    operator for two shifts), and their solutions agree to the accuracy the
    tolerance allows."""
    from paper_0707_0502_amd import gdr
    torch = torch_mod()
    cfg, links, kappa, B = config_data("C3")
    op = make_op(links, kappa)
    n = op.n
    sig = list(cfg["sigmas"])
    ns = len(sig)
    Bd = dev(B[0])
    out = {}
    for prec in (gdr.GDR_PREC_F64, gdr.GDR_PREC_MIXED):
        X = torch.zeros(ns * n, dtype=torch.complex128, device="cuda")
        p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"],
                                   tol=cfg["tol"], tol_extra=cfg["tol_extra"], precision=prec)
        st = gdr.Stats(1, ns)
        rc = gdr.gdr_solve(op, sig, Bd, X, p, st)
        say("C3 precision", prec, "rc", rc, "max resid %.2e" % st.resid.max(), st.as_dict())
        assert rc == gdr.GDR_OK
        assert st.resid.max() <= cfg["tol"]
        out[prec] = X.cpu().numpy().reshape(ns, n)
    A = wilson.WilsonOperator(links, kappa)
    xm = out[gdr.GDR_PREC_MIXED]
    for i in (0, ns - 1):
        res = np.linalg.norm(gmres.true_residual(A, B[0], xm[i], sig[i])) / np.linalg.norm(B[0])
        say("oracle true residual of the mixed solution, shift %d: %.3e" % (i, res))
        assert res <= cfg["tol"] * 1.01
    x64 = out[gdr.GDR_PREC_F64]
    for i in range(ns):
        d = np.linalg.norm(xm[i] - x64[i]) / np.linalg.norm(x64[i])
        say("shift %d: |x_mixed - x_fp64| / |x_fp64| = %.2e" % (i, d))
        # both solve to a 1e-8 residual; the error bound is the residual
        # times the conditioning (smallest |eigenvalue| of A - sigma ~ 0.02)
        assert d <= 100 * cfg["tol"]
    gdr.gdr_op_destroy(op)
