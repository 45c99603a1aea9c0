"""The paper's bidiagonal test matrix (Example 1: n = 1000, diagonal 0.1, 1,
2, ..., 999, superdiagonal 1) as a second operator behind the same C-ABI
solvers: the operator against its definition, Example 4's GMRES-DR(25,10)-Sh
against the oracle (equal products, solutions to 1e-10) and the paper's
printed count (250 products to 1e-10), and the multiple right-hand side path
(extra right-hand side, GMRES-Proj-Sh, correction) against the oracle."""
import json
import os

import numpy as np
import pytest

from oracle import gmres
from tests.gpu_common import ctx, dev, empty, host, rel, say

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


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
    yield op, d, e, mv
    gdr.gdr_op_destroy(op)


def test_apply_matches_definition(bop):
    from paper_0707_0502_amd import gdr
    op, d, e, mv = bop
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 1000)) + 1j * rng.standard_normal((3, 1000))
    sigma = -0.4 + 0.1j
    want = np.stack([mv(v) - sigma * v for v in x])
    y = empty(3 * 1000)
    gdr.gdr_op_apply(op, sigma, dev(x.ravel()), y, 3, gdr.GDR_PREC_F64)
    got = host(y).reshape(3, 1000)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    gdr.gdr_op_apply(op, sigma, dev(x.ravel()), y, 3, gdr.GDR_PREC_F32)
    got = host(y).reshape(3, 1000)
    assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()
    assert gdr.gdr_op_size(op) == 1000


def test_tables_rejected_for_bidiagonal(bop):
    from paper_0707_0502_amd import gdr
    op = bop[0]
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_op_tables(op)
    assert e.value.code == gdr.GDR_ERR_ARG


def test_example4_dr_sh(bop):
    """GMRES-DR(25,10)-Sh, sigma = 0, -0.4, -2, relative residual 1e-10, five
    random right-hand sides: per seed the GPU takes the oracle's products and
    matches its solutions; the median is the paper's 250."""
    from paper_0707_0502_amd import gdr
    op, d, e, mv = bop
    sig = [0, -0.4, -2]
    counts = []
    for seed in range(5):
        b = np.random.default_rng(seed).standard_normal(1000) + 0j
        ref = gmres.gmres_dr_sh(mv, b, sig, 25, 10, 1e-10)
        x = empty(3 * 1000)
        st = gdr.Stats(1, 3)
        p = gdr.gdr_params_default(m_dr=25, k=10, tol=1e-10, precision=gdr.GDR_PREC_F64)
        rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(b), x, p, st)
        say("seed", seed, "rc", rc, "gpu mvps", st.s.mvp_dr, "oracle", ref["mvps"])
        assert rc == gdr.GDR_OK
        assert st.s.mvp_dr == ref["mvps"]
        xh = host(x).reshape(3, 1000)
        for i in range(3):
            assert rel(xh[i], ref["x"][i]) <= 1e-10
        counts.append(st.s.mvp_dr)
        if defl is not None:
            gdr.gdr_defl_destroy(defl)
    assert np.median(counts) == GOLDEN["example4_mvps_to_1e-10"]["value"]


def test_two_rhs_proj_sh_with_correction(bop):
    """RHS 1 by GMRES-DR(25,10)-Sh, then the extra right-hand side v_{k+1}
    and RHS 2 by GMRES(15)-Proj(10)-Sh with the correction (Sec. 4), FP64:
    same products and solutions as the oracle's driver; mixed precision
    reaches 1e-8 for every (shift, RHS)."""
    from paper_0707_0502_amd import gdr
    op, d, e, mv = bop
    sig = [0, -0.4, -2]
    rng = np.random.default_rng(11)
    B = rng.standard_normal((2, 1000)) + 0j
    ref = gmres.solve_all(mv, B, sig, 25, 10, 15, 1e-8, 1e-6)
    X = empty(2 * 3 * 1000)
    st = gdr.Stats(2, 3)
    p = gdr.gdr_params_default(m_dr=25, k=10, m_proj=15, tol=1e-8, tol_extra=1e-6,
                               precision=gdr.GDR_PREC_F64)
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, st)
    dd = st.as_dict()
    say("rc", rc, dd)
    assert dd["mvp_dr"] == ref["runs"][0]["mvps"]
    assert dd["mvp_extra"] == ref["extra"]["mvps"]
    assert dd["mvp_proj"] == ref["runs"][1]["mvps"]
    Xh = host(X).reshape(2, 3, 1000)
    for j in range(2):
        for i in range(3):
            assert rel(Xh[j, i], ref["X"][j, i]) <= 1e-10
            assert abs(st.resid[j, i] - ref["resid"][j, i]) <= 1e-3 * ref["resid"][j, i] + 1e-13
    # mixed precision with refinement
    X = empty(2 * 3 * 1000)
    st = gdr.Stats(2, 3)
    p.precision = gdr.GDR_PREC_MIXED
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, st)
    say("mixed rc", rc, st.as_dict())
    Xh = host(X).reshape(2, 3, 1000)
    for j in range(2):
        for i in range(3):
            r = np.linalg.norm(B[j] - (mv(Xh[j, i]) - sig[i] * Xh[j, i])) / np.linalg.norm(B[j])
            assert r <= 1e-8
    assert rc == gdr.GDR_OK


def test_table41_accurate_eigenvector_projection(bop):
    """Example 4 / Table 4.1 on the GPU: RHS 1 by GMRES-DR(25,10)-Sh to 1e-10,
    RHS 2 by GMRES(15)-Proj-Sh over the leading k' approximate eigenvectors
    only (proj_k = k'): products and solutions equal the oracle's, and the
    products grow as k' shrinks (the printed trend)."""
    from paper_0707_0502_amd import gdr
    op, d, e, mv = bop
    sig = [0, -0.4, -2]
    b1 = np.random.default_rng(0).standard_normal(1000) + 0j
    b2 = np.random.default_rng(100).standard_normal(1000) + 0j
    ref1 = gmres.gmres_dr_sh(mv, b1, sig, 25, 10, 1e-10)
    x1 = empty(3 * 1000)
    p = gdr.gdr_params_default(m_dr=25, k=10, m_proj=15, tol=1e-10, precision=gdr.GDR_PREC_F64)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(b1), x1, p, gdr.Stats(1, 3))
    assert rc == gdr.GDR_OK and defl is not None
    counts = []
    for kp in (10, 6, 2):
        ref = gmres.gmres_proj_sh(mv, b2, sig, ref1["defl"], 15, 1e-10, 200, kp=kp)
        X = empty(3 * 1000)
        st = gdr.Stats(1, 3)
        p.proj_k = kp
        rc = gdr.gdr_solve_proj_sh(op, defl, sig, dev(b2), X, p, st)
        say("k'", kp, "rc", rc, "gpu mvps", st.s.mvp_proj, "oracle", ref["mvps"],
            "extra", st.s.mvp_extra)
        assert st.s.mvp_proj == ref["mvps"]
        assert st.s.mvp_extra == 0
        Xh = host(X).reshape(3, 1000)
        errs = [rel(Xh[i], ref["x"][i]) for i in range(3)]
        say("  rel err per shift", errs, "gpu resid", st.resid[0],
            "oracle resid", [np.linalg.norm(gmres.true_residual(mv, b2, ref["x"][i], sig[i]))
                             / np.linalg.norm(b2) for i in range(3)])
        assert max(errs) <= 1e-10
        counts.append(st.s.mvp_proj)
    assert counts[0] <= counts[1] <= counts[2]
    gdr.gdr_defl_destroy(defl)
