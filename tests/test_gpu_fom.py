"""GPU parity of the Galerkin variant (gdr_params.galerkin = 1): FOM-DR-Sh and
FOM(m)-Sh (Sec. 3, Examples 2 and 3) on the same C-ABI solvers, against the
oracle's FOM runs.

FP64 with deflation: the GPU and the oracle run the same algorithm on the same
inputs, so product counts are equal, per-cycle residual norms agree to 1e-8
relative, kept Ritz values to 1e-8 and solutions to 1e-10 (as for GMRES-DR-Sh).
Example 2 without deflation (FOM(40)-Sh, shifts 0.4, 0, -1) is erratic for the
base shift: some of its Galerkin systems are nearly singular (the residual
jumps by 30x within a cycle), which multiplies rounding differences between
the device's Householder solves and the oracle's LU solves by their condition
number. Its per-cycle residual norms are therefore compared to 1e-6 relative
(room for a condition number of 1e9 at FP64 rounding) and the converged
shift's solution to 1e-8, besides what the paper states: the sigma = -1 system
below 1e-8 in 400 products, checked with the FP64 true residual."""
import numpy as np
import pytest

from oracle import gmres, wilson
from tests.gpu_common import config_data, ctx, dev, empty, host, make_op, rel, say

pytestmark = pytest.mark.gpu


def example1():
    d = np.concatenate([[0.1], np.arange(1, 1000)]).astype(np.complex128)
    e = np.ones(999, np.complex128)

    def mv(v):
        w = d * v
        w[:-1] += e * v[1:]
        return w
    return d, e, mv


@pytest.fixture(scope="module")
def bop():
    from paper_0707_0502_amd import gdr
    d, e, mv = example1()
    op = gdr.gdr_bidiag_create(ctx(), d, e)
    yield op, mv
    gdr.gdr_op_destroy(op)


def test_fomdr_bidiag_fp64_parity(bop):
    """FOM-DR(25,10)-Sh, shifts 0, -0.4, -2, tolerance 1e-10, three seeds."""
    from paper_0707_0502_amd import gdr
    op, mv = bop
    sig = [0, -0.4, -2]
    for seed in range(3):
        b = np.random.default_rng(seed).standard_normal(1000) + 0j
        ref = gmres.gmres_dr_sh(mv, b, sig, 25, 10, 1e-10, fom=True)
        x = empty(3 * 1000)
        st = gdr.Stats(1, 3)
        p = gdr.gdr_params_default(m_dr=25, k=10, tol=1e-10, precision=gdr.GDR_PREC_F64,
                                   galerkin=1)
        rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(b), x, p, st)
        say("seed", seed, "rc", rc, "gpu mvps", st.s.mvp_dr, "oracle", ref["mvps"])
        assert rc == gdr.GDR_OK
        assert st.s.mvp_dr == ref["mvps"]
        for h, e in zip(st.hist, ref["history"]):
            assert abs(h[3] - e["r1"]) <= 1e-8 * e["r1"], (h, e["r1"])
        th = st.theta.reshape(-1, 10)
        for t, e in zip(th, ref["history"]):
            assert np.abs(t - e["theta"]).max() <= 1e-8 * np.abs(e["theta"]).max()
        xh = host(x).reshape(3, 1000)
        errs = [rel(xh[i], ref["x"][i]) for i in range(3)]
        say("  rel err", errs, "resid", st.resid[0])
        assert max(errs) <= 1e-10
        if defl is not None:
            gdr.gdr_defl_destroy(defl)


def test_example2_fom_sh(bop):
    """FOM(40)-Sh (k = 0), shifts 0.4, 0, -1, 400 products: sigma = -1 reaches
    a true relative residual below 1e-8, the base shift does not converge."""
    from paper_0707_0502_amd import gdr
    op, mv = bop
    sig = [0.4, 0, -1]
    b = np.random.default_rng(0).standard_normal(1000) + 0j
    ref = gmres.gmres_dr_sh(mv, b, sig, 40, 0, 1e-8, max_cycles=10, fom=True)
    x = empty(3 * 1000)
    st = gdr.Stats(1, 3)
    p = gdr.gdr_params_default(m_dr=40, k=0, tol=1e-8, max_cycles=10,
                               precision=gdr.GDR_PREC_F64, galerkin=1)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(b), x, p, st)
    say("rc", rc, "mvps", st.s.mvp_dr, "resid", st.resid[0])
    say("  gpu r1", st.hist[:, 3], "\n  oracle r1", [e["r1"] for e in ref["history"]])
    assert rc == gdr.GDR_NOT_CONVERGED
    assert st.s.mvp_dr == 400 == ref["mvps"]
    assert st.resid[0, 2] <= 1e-8
    assert st.resid[0, 0] > 1e-2
    xh = host(x).reshape(3, 1000)
    r = np.linalg.norm(gmres.true_residual(mv, b, xh[2], -1)) / np.linalg.norm(b)
    assert r <= 1e-8
    err = rel(xh[2], ref["x"][2])
    say("  sigma=-1 rel err vs oracle", err)
    assert err <= 1e-8
    assert len(st.hist) == len(ref["history"]) == 10
    for h, e in zip(st.hist, ref["history"]):
        assert abs(h[3] - e["r1"]) <= 1e-6 * e["r1"], (h, e["r1"])
    if defl is not None:
        gdr.gdr_defl_destroy(defl)


def test_fomdr_two_rhs_proj(bop):
    """RHS 1 by FOM-DR(25,10)-Sh, then the extra right-hand side and RHS 2 by
    GMRES(15)-Proj(10)-Sh with the correction over FOM-DR's deflation pair,
    FP64: same products and solutions as the oracle's driver."""
    from paper_0707_0502_amd import gdr
    op, mv = bop
    sig = [0, -0.4, -2]
    B = np.random.default_rng(11).standard_normal((2, 1000)) + 0j
    ref = gmres.solve_all(mv, B, sig, 25, 10, 15, 1e-8, 1e-6, fom=True)
    X = empty(2 * 3 * 1000)
    st = gdr.Stats(2, 3)
    p = gdr.gdr_params_default(m_dr=25, k=10, m_proj=15, tol=1e-8, tol_extra=1e-6,
                               precision=gdr.GDR_PREC_F64, galerkin=1)
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, st)
    dd = st.as_dict()
    say("rc", rc, dd)
    assert rc == gdr.GDR_OK
    assert dd["mvp_dr"] == ref["runs"][0]["mvps"]
    assert dd["mvp_extra"] == ref["extra"]["mvps"]
    assert dd["mvp_proj"] == ref["runs"][1]["mvps"]
    Xh = host(X).reshape(2, 3, 1000)
    for j in range(2):
        for i in range(3):
            assert rel(Xh[j, i], ref["X"][j, i]) <= 1e-10
    assert st.resid.max() <= 1e-8


def test_fomdr_wilson_c1(bop):
    """FOM-DR-Sh on the 4^4 Wilson lattice (five shifts): FP64 parity with the
    oracle; mixed precision reaches the tolerance on every shift."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = config_data("C1")
    A = wilson.WilsonOperator(links, kappa)
    sig = np.array(cfg["sigmas"], complex)
    ref = gmres.gmres_dr_sh(A, B[0], sig, cfg["m_dr"], cfg["k"], cfg["tol"], fom=True)
    op = make_op(links, kappa)
    n = op.n
    for prec in (gdr.GDR_PREC_F64, gdr.GDR_PREC_MIXED):
        x = empty(len(sig) * n)
        st = gdr.Stats(1, len(sig))
        p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], tol=cfg["tol"],
                                   precision=prec, galerkin=1)
        rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), x, p, st)
        say("prec", prec, "rc", rc, "mvps", st.s.mvp_dr, "oracle", ref["mvps"],
            "resid", st.resid[0])
        assert rc == gdr.GDR_OK
        X = host(x).reshape(len(sig), n)
        if prec == gdr.GDR_PREC_F64:
            assert st.s.mvp_dr == ref["mvps"]
            for i in range(len(sig)):
                assert rel(X[i], ref["x"][i]) <= 1e-10
        for i in range(len(sig)):
            r = np.linalg.norm(gmres.true_residual(A, B[0], X[i], sig[i])) / np.linalg.norm(B[0])
            assert r <= cfg["tol"] * 1.01
        if defl is not None:
            gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)
