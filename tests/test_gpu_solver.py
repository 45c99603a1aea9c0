"""GPU parity of the solvers (through the C-ABI) against the oracle.

Plain FP64: the GPU and the oracle run the same algorithm on the same
inputs, so cycle counts and matrix-vector product counts are equal, the
per-cycle residual norms and kept harmonic Ritz values agree to 1e-8
relative, and every solution agrees to 1e-10 relative. Mixed precision:
every true FP64 residual is at most the tolerance; the error against the
oracle is reported per shift."""
import numpy as np
import pytest

from oracle import gmres, wilson
from tests.gpu_common import config_data, ctx, dev, empty, host, make_op, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    cfg, links, kappa, B = config_data("C1")
    A = wilson.WilsonOperator(links, kappa)
    sig = np.array(cfg["sigmas"], complex)
    ref = gmres.gmres_dr_sh(A, B[0], sig, cfg["m_dr"], cfg["k"], cfg["tol"])
    return cfg, links, kappa, B, A, sig, ref


@pytest.fixture(scope="module")
def c2():
    cfg, links, kappa, B = config_data("C2")
    A = wilson.WilsonOperator(links, kappa)
    sig = np.array(cfg["sigmas"], complex)
    say("oracle C2 ...")
    ref = gmres.solve_all(A, B, sig, cfg["m_dr"], cfg["k"], cfg["m_proj"], cfg["tol"],
                          cfg["tol_extra"])
    say("oracle C2 done")
    return cfg, links, kappa, B, A, sig, ref


def params(cfg, precision):
    from paper_0707_0502_amd import gdr
    return gdr.gdr_params_default(m_dr=cfg["m_dr"], k=cfg["k"], m_proj=cfg["m_proj"],
                                  tol=cfg["tol"], tol_extra=cfg["tol_extra"],
                                  precision=precision)


def test_c1_dr_sh_fp64_parity(c1):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, ref = c1
    say("C1 FP64 GMRES-DR-Sh")
    op = make_op(links, kappa)
    n = op.n
    x = empty(len(sig) * n)
    st = gdr.Stats(1, len(sig))
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), x, params(cfg, gdr.GDR_PREC_F64), st)
    assert rc == gdr.GDR_OK
    d = st.as_dict()
    say("  gpu cycles", d["cycles_dr"], "mvps", d["mvp_dr"], "oracle", ref["cycles"], ref["mvps"])
    assert d["cycles_dr"] == ref["cycles"] and d["mvp_dr"] == ref["mvps"]
    hist = st.hist
    for h, e in zip(hist, ref["history"]):
        assert abs(h[3] - e["r1"]) <= 1e-8 * e["r1"]
    # kept harmonic Ritz values per cycle, in selection order
    th = st.theta.reshape(-1, cfg["k"])
    for t, e in zip(th, ref["history"]):
        assert np.abs(t - e["theta"]).max() <= 1e-8 * np.abs(e["theta"]).max()
    X = host(x).reshape(len(sig), n)
    for i in range(len(sig)):
        err = rel(X[i], ref["x"][i])
        say("  shift", sig[i], "rel err", err, "resid", st.resid[0, i])
        assert err <= 1e-10
    # the exported deflation pair satisfies A V_k = V_{k+1} H_bar_k
    k = gdr.gdr_defl_k(defl)
    V = empty((k + 1) * n)
    Hb = np.zeros((k, k + 1), complex)   # column-major (k+1) x k
    gdr.gdr_defl_export(defl, V, Hb)
    Vh = host(V).reshape(k + 1, n)
    Hbar = Hb.T
    AV = empty(k * n)
    gdr.gdr_op_apply(op, 0.0, V[:k * n], AV, k)
    AVh = host(AV).reshape(k, n)
    resid = np.linalg.norm(AVh.T - Vh.T @ Hbar) / np.linalg.norm(Hbar)
    say("  ||A V_k - V_{k+1} H_k|| / ||H_k|| =", resid)
    assert resid <= 1e-12
    assert np.abs(Vh.conj() @ Vh.T - np.eye(k + 1)).max() <= 1e-12
    gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)


def test_c1_mixed_reaches_tolerance(c1):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, ref = c1
    say("C1 mixed GMRES-DR-Sh + cleanup")
    op = make_op(links, kappa)
    n = op.n
    x = empty(len(sig) * n)
    st = gdr.Stats(1, len(sig))
    p = params(cfg, gdr.GDR_PREC_MIXED)
    p.tol = 1e-8
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), x, p, st)
    say("  rc", rc, st.as_dict())
    X = host(x).reshape(len(sig), n)
    for i in range(len(sig)):
        r = np.linalg.norm(gmres.true_residual(A, B[0], X[i], sig[i])) / np.linalg.norm(B[0])
        say("  shift", sig[i], "true resid (oracle)", r, "lib", st.resid[0, i],
            "err vs oracle", rel(X[i], ref["x"][i]))
        assert r <= 1e-8
        assert abs(r - st.resid[0, i]) <= 1e-3 * r + 1e-15
    assert rc == gdr.GDR_OK
    gdr.gdr_defl_destroy(defl)
    gdr.gdr_op_destroy(op)


def test_c2_full_fp64_parity(c2):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, ref = c2
    say("C2 FP64 gdr_solve (DR-Sh, extra RHS, Proj-Sh batch, correction)")
    op = make_op(links, kappa)
    n = op.n
    nrhs, ns = B.shape[0], len(sig)
    X = empty(nrhs * ns * n)
    st = gdr.Stats(nrhs, ns)
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, params(cfg, gdr.GDR_PREC_F64), st)
    d = st.as_dict()
    say("  rc", rc, d)
    expect = gdr.GDR_OK if ref["resid"].max() <= cfg["tol"] else gdr.GDR_NOT_CONVERGED
    assert rc == expect
    assert d["mvp_dr"] == ref["runs"][0]["mvps"]
    assert d["mvp_extra"] == ref["extra"]["mvps"]
    assert d["mvp_proj"] == sum(r["mvps"] for r in ref["runs"][1:])
    Xh = host(X).reshape(nrhs, ns, n)
    worst = 0
    for j in range(nrhs):
        for i in range(ns):
            err = rel(Xh[j, i], ref["X"][j, i])
            worst = max(worst, err)
            assert abs(st.resid[j, i] - ref["resid"][j, i]) <= 1e-3 * ref["resid"][j, i] + 1e-13
    say("  worst rel err vs oracle", worst)
    assert worst <= 1e-10
    gdr.gdr_op_destroy(op)


def test_c2_mixed_batched(c2):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, ref = c2
    say("C2 mixed batched gdr_solve, tol 1e-8")
    op = make_op(links, kappa)
    n = op.n
    nrhs, ns = B.shape[0], len(sig)
    X = empty(nrhs * ns * n)
    st = gdr.Stats(nrhs, ns)
    p = params(cfg, gdr.GDR_PREC_MIXED)
    p.tol = 1e-8
    p.tol_extra = 1e-4
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, st)
    say("  rc", rc, st.as_dict())
    Xh = host(X).reshape(nrhs, ns, n)
    for j in range(nrhs):
        for i in range(ns):
            r = np.linalg.norm(gmres.true_residual(A, B[j], Xh[j, i], sig[i])) / np.linalg.norm(B[j])
            say("  rhs", j, "shift", sig[i], "true resid", r, "err vs oracle",
                rel(Xh[j, i], ref["X"][j, i]))
            assert r <= 1e-8
    assert rc == gdr.GDR_OK
    gdr.gdr_op_destroy(op)


def test_c2_mixed_batch_over_16_members(c2):
    """19 right-hand sides: the 18 later ones form one GMRES-Proj-Sh batch, so
    the batched projection on the shared deflation basis runs two member
    groups (16 members per block on the FP64 matrix cores, the second group
    holding two members, its second tile empty). Every (RHS, shift) pair
    reaches a true FP64 residual of at most 1e-8."""
    import synth
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, ref = c2
    B19 = np.stack([B[0]] + [synth.make_rhs(cfg, "z4", 5000 + j).ravel() for j in range(18)])
    say("C2 mixed gdr_solve, 19 RHS (Proj batch of 18), tol 1e-8")
    op = make_op(links, kappa)
    n = op.n
    assert n % 16 == 0   # the matrix-core projection needs 16-row chunks
    nrhs, ns = B19.shape[0], len(sig)
    X = empty(nrhs * ns * n)
    st = gdr.Stats(nrhs, ns)
    p = params(cfg, gdr.GDR_PREC_MIXED)
    p.tol = 1e-8
    p.tol_extra = 1e-4
    rc = gdr.gdr_solve(op, sig, dev(B19.ravel()), X, p, st)
    say("  rc", rc, st.as_dict())
    assert rc == gdr.GDR_OK
    Xh = host(X).reshape(nrhs, ns, n)
    worst = 0.0
    for j in range(nrhs):
        for i in range(ns):
            r = np.linalg.norm(gmres.true_residual(A, B19[j], Xh[j, i], sig[i])) / np.linalg.norm(B19[j])
            worst = max(worst, r)
            assert r <= 1e-8, (j, i, r)
    say("  worst true resid", worst)
    # the first RHS is C2's own: its error against the oracle, per shift
    for i in range(ns):
        say("  rhs 0 shift", sig[i], "err vs oracle", rel(Xh[0, i], ref["X"][0, i]))
    gdr.gdr_op_destroy(op)


def test_c2_related_rhs_fp64_parity(c2):
    """Related right-hand sides (Sec. 5, eq. (5.2)), sequential order: every
    later RHS is first projected over all earlier right-hand sides and their
    solutions. Same products and solutions as the oracle's driver."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, _ = c2
    say("oracle C2 related ...")
    ref = gmres.solve_all(A, B, sig, cfg["m_dr"], cfg["k"], cfg["m_proj"], cfg["tol"],
                          cfg["tol_extra"], related=True)
    say("C2 FP64 gdr_solve, related right-hand sides, sequential")
    op = make_op(links, kappa)
    n = op.n
    nrhs, ns = B.shape[0], len(sig)
    X = empty(nrhs * ns * n)
    st = gdr.Stats(nrhs, ns)
    p = params(cfg, gdr.GDR_PREC_F64)
    p.related_rhs = 1
    p.batch = 0
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, st)
    d = st.as_dict()
    say("  rc", rc, d, "oracle proj mvps", [r["mvps"] for r in ref["runs"][1:]])
    # the corrected shifts end where the extra right-hand side's tolerance
    # leaves them: the status follows the oracle's true residuals
    expect = gdr.GDR_OK if ref["resid"].max() <= cfg["tol"] else gdr.GDR_NOT_CONVERGED
    assert rc == expect
    assert d["mvp_proj"] == sum(r["mvps"] for r in ref["runs"][1:])
    Xh = host(X).reshape(nrhs, ns, n)
    worst = max(rel(Xh[j, i], ref["X"][j, i]) for j in range(nrhs) for i in range(ns))
    say("  worst rel err vs oracle", worst)
    assert worst <= 1e-10
    # the start is only as accurate as the earlier solutions, so non-base
    # shifts may end slightly above tol: the oracle's driver does the same
    for j in range(nrhs):
        for i in range(ns):
            assert abs(st.resid[j, i] - ref["resid"][j, i]) <= 1e-3 * ref["resid"][j, i] + 1e-13
    gdr.gdr_op_destroy(op)


def test_c2_related_rhs_mixed_batched(c2):
    """Related right-hand sides in a batch: each later RHS projects over the
    first one (solved before the batch); every true residual meets 1e-8."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, _ = c2
    op = make_op(links, kappa)
    n = op.n
    nrhs, ns = B.shape[0], len(sig)
    X = empty(nrhs * ns * n)
    st = gdr.Stats(nrhs, ns)
    p = params(cfg, gdr.GDR_PREC_MIXED)
    p.tol = 1e-8
    p.tol_extra = 1e-4
    p.related_rhs = 1
    rc = gdr.gdr_solve(op, sig, dev(B.ravel()), X, p, st)
    say("  rc", rc, st.as_dict())
    Xh = host(X).reshape(nrhs, ns, n)
    for j in range(nrhs):
        for i in range(ns):
            r = np.linalg.norm(gmres.true_residual(A, B[j], Xh[j, i], sig[i])) / np.linalg.norm(B[j])
            assert r <= 1e-8
    assert rc == gdr.GDR_OK
    gdr.gdr_op_destroy(op)


def test_k0_is_gmres_sh(c1):
    """k = 0: GMRES(m)-Sh (Sec. 2.1), same iterates as the oracle."""
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, _ = c1
    ref = gmres.gmres_dr_sh(A, B[0], sig[:3], 20, 0, 1e-9)
    op = make_op(links, kappa)
    x = empty(3 * op.n)
    st = gdr.Stats(1, 3)
    p = gdr.gdr_params_default(m_dr=20, k=0, m_proj=20, tol=1e-9)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig[:3], dev(B[0]), x, p, st, want_defl=False)
    assert st.s.mvp_dr == ref["mvps"]
    X = host(x).reshape(3, op.n)
    for i in range(3):
        assert rel(X[i], ref["x"][i]) <= 1e-10
    gdr.gdr_op_destroy(op)


def test_lucky_breakdown_plane_wave():
    """Free field and a plane-wave b: the Krylov space closes after <= 4
    steps; the library solves every shift exactly in one cycle."""
    from paper_0707_0502_amd import gdr
    import synth
    dims = (4, 4, 4, 4)
    links = synth.unit_links(dims)
    t, z, y, xx = np.meshgrid(range(4), range(4), range(4), range(4), indexing="ij")
    ph = np.exp(1j * (2 * np.pi * (xx + 2 * y) / 4 + np.pi * 3 * t / 4))
    chi = np.zeros((4, 3), complex)
    chi[0, 1] = 1
    chi[2, 1] = 0.5j
    b = (ph[..., None, None] * chi).ravel()
    op = make_op(links, 0.1)
    sig = [0.0, -0.3]
    x = empty(2 * op.n)
    st = gdr.Stats(1, 2)
    p = gdr.gdr_params_default(m_dr=10, k=3, m_proj=10, tol=1e-12)
    rc, defl = gdr.gdr_solve_dr_sh(op, sig, dev(b), x, p, st)
    assert rc == gdr.GDR_OK
    assert st.s.cycles_dr == 1 and st.s.mvp_dr == 10
    assert defl is None
    assert st.resid.max() <= 1e-13
    gdr.gdr_op_destroy(op)


def test_solver_argument_errors(c1):
    from paper_0707_0502_amd import gdr
    cfg, links, kappa, B, A, sig, _ = c1
    op = make_op(links, kappa)
    x = empty(len(sig) * op.n)
    for bad in (dict(m_dr=10, k=10), dict(m_dr=70, k=5), dict(m_proj=0), dict(tol=0.0),
                dict(precision=5), dict(sstep=9), dict(sstep_reorth=-1.0),
                dict(refine_floor=0.7), dict(refine_floor=-1e-3), dict(m_clean=65)):
        p = params(cfg, gdr.GDR_PREC_F64)
        for k_, v in bad.items():
            setattr(p, k_, v)
        with pytest.raises(gdr.GdrError) as e:
            gdr.gdr_solve_dr_sh(op, sig, dev(B[0]), x, p)
        assert e.value.code == gdr.GDR_ERR_ARG
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_solve_dr_sh(op, [], dev(B[0]), x, params(cfg, 0))
    assert e.value.code == gdr.GDR_ERR_ARG
    gdr.gdr_op_destroy(op)


def test_graph_replay_matches_eager(c2):
    """Arnoldi cycles captured once into HIP graphs and replayed (DR cycles
    alternate between two bases, the batched Proj-Sh cycles reuse one graph,
    with eager work and host synchronisation between replays): every product
    count and every solution equals the eager solve bit for bit."""
    from paper_0707_0502_amd import gdr
    from tests.gpu_common import torch_mod
    torch = torch_mod()
    cfg, links, kappa, B, A, sig, ref = c2
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = gdr.gdr_ctx_create(0, stream.cuda_stream)
        lt, lz, ly, lx = links.shape[1:5]
        op = gdr.gdr_wilson_create(gctx, (lx, ly, lz, lt), (1, 1, 1, -1), kappa,
                                   np.ascontiguousarray(links), 1)
        n = op.n
        nrhs, ns = B.shape[0], len(sig)
        out = {}
        for prec in (gdr.GDR_PREC_F64, gdr.GDR_PREC_MIXED):
            for graph in (0, 1):
                X = torch.zeros(nrhs * ns * n, dtype=torch.complex128, device="cuda")
                st = gdr.Stats(nrhs, ns)
                p = params(cfg, prec)
                if prec == gdr.GDR_PREC_MIXED:
                    p.tol, p.tol_extra = 1e-8, 1e-4
                p.use_graph = graph
                Bd = torch.from_numpy(np.ascontiguousarray(B.ravel())).cuda()
                rc = gdr.gdr_solve(op, sig, Bd, X, p, st)
                stream.synchronize()
                out[(prec, graph)] = (rc, st.as_dict(), X.cpu().numpy())
                say("  prec", prec, "graph", graph, "rc", rc, "t", st.s.t_total)
        for prec in (gdr.GDR_PREC_F64, gdr.GDR_PREC_MIXED):
            e, g = out[(prec, 0)], out[(prec, 1)]
            # plain FP64 at tol 1e-10 ends with its corrected shifts where the
            # extra right-hand side leaves them (the oracle's 2.4e-10 on C2)
            expect = gdr.GDR_OK
            if prec == gdr.GDR_PREC_F64 and ref["resid"].max() > cfg["tol"]:
                expect = gdr.GDR_NOT_CONVERGED
            assert e[0] == g[0] == expect
            for key in ("mvp_dr", "mvp_extra", "mvp_proj", "mvp_cleanup", "cycles_dr", "cycles_proj"):
                assert e[1][key] == g[1][key]
            assert np.array_equal(e[2], g[2])
        gdr.gdr_op_destroy(op)
        gdr.gdr_ctx_destroy(gctx)
