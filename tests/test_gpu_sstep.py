"""The s-step Arnoldi cycle of the FP32 path (gdr_params.sstep = block size):
the deflation pair it hands over satisfies the Arnoldi relation
A V_k = V_{k+1} H_bar_k and V_{k+1} is orthonormal, both to FP32 accuracy,
for block sizes 1 (one vector per step) to 8 (5..8 on the matrix-core
sweeps), on the bidiagonal matrix
and on a Wilson lattice; the mixed solves it drives reach the tolerance."""
import numpy as np
import pytest

from oracle import gmres, wilson
from tests.gpu_common import config_data, ctx, dev, empty, host, make_op, say

pytestmark = pytest.mark.gpu


def bidiag_op(n=1000):
    from paper_0707_0502_amd import gdr
    d = np.concatenate([[0.1], np.arange(1, n)]).astype(np.complex128)
    e = np.ones(n - 1, np.complex128)

    def mv(v):
        w = d * v
        w[:-1] += e * v[1:]
        return w
    return gdr.gdr_bidiag_create(ctx(), d, e), mv


def relation(gdr, op, defl, mv_host, n):
    k = gdr.gdr_defl_k(defl)
    V = empty((k + 1) * n)
    Hb = np.zeros((k, k + 1), complex)
    gdr.gdr_defl_export(defl, V, Hb)
    Vh = host(V).reshape(k + 1, n).T
    Hbar = Hb.T
    AV = np.stack([mv_host(Vh[:, i]) for i in range(k)], axis=1)
    rel = np.linalg.norm(AV - Vh @ Hbar) / np.linalg.norm(Hbar)
    orth = np.abs(Vh.conj().T @ Vh - np.eye(k + 1)).max()
    return rel, orth


@pytest.mark.parametrize("reorth", [20.0, 0.0])
@pytest.mark.parametrize("sstep", [1, 2, 3, 4, 5, 6, 7, 8])
def test_arnoldi_relation_bidiagonal(sstep, reorth):
    from paper_0707_0502_amd import gdr
    # blocks of more than 4 run on the matrix-core sweeps, which take n % 16 == 0
    n = 1000 if sstep <= 4 else 1024
    op, mv = bidiag_op(n)
    b = np.random.default_rng(5).standard_normal(n) + 0j
    sig = [0, -0.4, -2]
    x = empty(3 * n)
    st = gdr.Stats(1, 3)
    p = gdr.gdr_params_default(m_dr=25, k=10, tol=1e-6, max_cycles=2, precision=gdr.GDR_PREC_MIXED,
                               sstep=sstep, sstep_reorth=reorth)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(b), x, p, st)
    say("sstep", sstep, "reorth", reorth, "rc", rc, "hist", st.hist[:, 3])
    assert defl is not None
    rel, orth = relation(gdr, op, defl, mv, n)
    say("  A V_k - V_{k+1} H_k rel %.3e, orthonormality %.3e" % (rel, orth))
    assert rel <= 1e-5 and orth <= 1e-5
    gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)


@pytest.mark.parametrize("reorth", [20.0, 0.0])
@pytest.mark.parametrize("sstep", [1, 4, 6, 8])
def test_arnoldi_relation_wilson(sstep, reorth):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B = config_data("C1")
    A = wilson.WilsonOperator(links, kappa)
    op = make_op(links, kappa)
    n = op.n
    sig = np.array(cfg["sigmas"], complex)
    x = empty(len(sig) * n)
    st = gdr.Stats(1, len(sig))
    p = gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], tol=1e-6, max_cycles=2,
                               precision=gdr.GDR_PREC_MIXED, sstep=sstep, sstep_reorth=reorth)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), x, p, st)
    say("sstep", sstep, "reorth", reorth, "rc", rc, "hist", st.hist[:, 3])
    assert defl is not None
    rel, orth = relation(gdr, op, defl, A, n)
    say("  A V_k - V_{k+1} H_k rel %.3e, orthonormality %.3e" % (rel, orth))
    assert rel <= 1e-5 and orth <= 1e-5
    gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)
