"""Several lattices in one call (gdr_solve_many). With params.persistent = 1
the first right-hand sides of all lattices run as one batch whose operator
applications are one persistent work-list launch over the tiles of lattices
of different sizes; every lattice must still follow the single-lattice
algorithm: the same Krylov space and stopping rule (so GMRES-DR-Sh takes the
same number of products as gdr_solve on that lattice alone, give or take one
cycle for rounding), FP64 true residuals at most tol, checked here again with
the oracle's operator, and solutions that agree with the single-lattice
solves to the accuracy the tolerance allows."""
import numpy as np
import pytest

import synth
from oracle import gmres, wilson
from tests.gpu_common import ctx, dev, empty, host, make_op, say, torch_mod

pytestmark = pytest.mark.gpu

SIG = [0.0, -0.02, -0.05, -0.1]


def _lattices():
    out = []
    for dims, seed in (((8, 8, 8, 8), 31), ((12, 12, 12, 12), 32), ((8, 8, 12, 16), 33)):
        links = synth.gauge_links(dims, 0.5, seed)
        # near the critical hopping parameter of the 12^4 fields of the batch
        # workload (the field's own kappa_c is not needed: every lattice only
        # has to be a well-posed, slowly converging system)
        kappa = 0.9 * synth.kappa("C5a1")
        cfg = dict(dims=dims, rhs=[("z4", 500 + seed), ("z4", 600 + seed)])
        B = np.stack([synth.make_rhs(cfg, k, s).ravel() for k, s in cfg["rhs"]])
        out.append(dict(dims=dims, links=links, kappa=kappa, B=B))
    return out


def _params(gdr, persistent, **kw):
    p = gdr.gdr_params_default(m_dr=40, k=15, m_proj=40, tol=1e-8, tol_extra=1e-4,
                               precision=gdr.GDR_PREC_MIXED, persistent=persistent)
    for k_, v in kw.items():
        setattr(p, k_, v)
    return p


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_persistent_batch_matches_single_lattice_solves(storage):
    from paper_0707_0502_amd import gdr
    lat = _lattices()
    lst = gdr.GDR_LINKS_F16 if storage == "f16" else gdr.GDR_LINKS_F32
    ops = [make_op(L["links"], L["kappa"], link_storage=lst) for L in lat]
    want = 96 if storage == "f16" else 192
    assert all(gdr.gdr_op_link_bytes(o, gdr.GDR_PREC_F32) == want for o in ops)
    ns, nrhs = len(SIG), 2
    # each lattice alone
    single = []
    for L, o in zip(lat, ops):
        X = empty(nrhs * ns * o.n)
        st = gdr.Stats(nrhs, ns)
        rc = gdr.gdr_solve(o, SIG, dev(L["B"].ravel()), X, _params(gdr, 0), st)
        assert rc == gdr.GDR_OK
        single.append((host(X).reshape(nrhs, ns, -1), st))
    # all together
    Xs = [empty(nrhs * ns * o.n) for o in ops]
    sts = [gdr.Stats(nrhs, ns) for _ in ops]
    rc = gdr.gdr_solve_many(ops, SIG, [dev(L["B"].ravel()) for L in lat], Xs, _params(gdr, 1), sts)
    say("gdr_solve_many rc", rc, [s_.resid.max() for s_ in sts])
    assert rc == gdr.GDR_OK
    for l, (L, o) in enumerate(zip(lat, ops)):
        X = host(Xs[l]).reshape(nrhs, ns, -1)
        Xs1, st1 = single[l]
        st = sts[l]
        say(L["dims"], storage, "batch", {k: v for k, v in st.as_dict().items() if k.startswith("mvp")},
            "alone", {k: v for k, v in st1.as_dict().items() if k.startswith("mvp")},
            "max resid %.2e" % st.resid.max())
        assert st.resid.max() <= 1e-8
        assert abs(st.s.mvp_dr - st1.s.mvp_dr) <= 40 - 15
        assert st.s.mvp_proj > 0
        A = wilson.WilsonOperator(L["links"], L["kappa"])
        for j in range(nrhs):
            for i in range(ns):
                r = np.linalg.norm(gmres.true_residual(A, L["B"][j], X[j, i], SIG[i]))
                assert r / np.linalg.norm(L["B"][j]) <= 1.01e-8, (L["dims"], j, i)
                # two solutions with relative residuals <= 1e-8 of a system whose
                # smallest eigenvalue is near 0.05 differ by well under 1e-5
                d = np.linalg.norm(X[j, i] - Xs1[j, i]) / np.linalg.norm(Xs1[j, i])
                assert d <= 1e-5, (L["dims"], j, i, d)
    for o in ops:
        gdr.gdr_op_destroy(o)


def test_sequential_many_equals_single_solves():
    """persistent = 0: the lattices one after another through the same code
    as gdr_solve, bit for bit."""
    from paper_0707_0502_amd import gdr
    lat = _lattices()[:2]
    ops = [make_op(L["links"], L["kappa"]) for L in lat]
    ns, nrhs = len(SIG), 2
    Xs = [empty(nrhs * ns * o.n) for o in ops]
    assert gdr.gdr_solve_many(ops, SIG, [dev(L["B"].ravel()) for L in lat], Xs,
                              _params(gdr, 0)) == gdr.GDR_OK
    for L, o, Xm in zip(lat, ops, Xs):
        X = empty(nrhs * ns * o.n)
        assert gdr.gdr_solve(o, SIG, dev(L["B"].ravel()), X, _params(gdr, 0)) == gdr.GDR_OK
        assert np.array_equal(host(X).view(np.float64), host(Xm).view(np.float64))
    for o in ops:
        gdr.gdr_op_destroy(o)


def test_persistent_requirements():
    from paper_0707_0502_amd import gdr
    lat = _lattices()[:2]
    ops = [make_op(L["links"], L["kappa"]) for L in lat]
    ns, nrhs = len(SIG), 2
    Bs = [dev(L["B"].ravel()) for L in lat]
    Xs = [empty(nrhs * ns * o.n) for o in ops]
    for bad in (dict(precision=gdr.GDR_PREC_F64), dict(sstep=1)):
        with pytest.raises(gdr.GdrError) as e:
            gdr.gdr_solve_many(ops, SIG, Bs, Xs, _params(gdr, 1, **bad))
        assert e.value.code == gdr.GDR_ERR_ARG
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_solve_many(ops, SIG, Bs, Xs, _params(gdr, 2))
    assert e.value.code == gdr.GDR_ERR_ARG
    # links that are not special unitary keep nine entries: not for the work list
    rng = np.random.default_rng(7)
    gen = lat[0]["links"] * (1.0 + 0.05 * rng.standard_normal(lat[0]["links"].shape[:-2]))[..., None, None]
    og = make_op(gen, lat[0]["kappa"])
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_solve_many([og, ops[1]], SIG, Bs, Xs, _params(gdr, 1))
    assert e.value.code == gdr.GDR_ERR_ARG
    # one FP16-stored and one FP32-stored lattice: one link precision per batch
    o16 = make_op(lat[0]["links"], lat[0]["kappa"], link_storage=gdr.GDR_LINKS_F16)
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_solve_many([o16, ops[1]], SIG, Bs, Xs, _params(gdr, 1))
    assert e.value.code == gdr.GDR_ERR_ARG
    for o in ops + [og, o16]:
        gdr.gdr_op_destroy(o)
