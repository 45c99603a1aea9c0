"""GPU parity of the lattice tables and the Wilson-Dirac operator (through
the C-ABI) against the oracle."""
import numpy as np
import pytest

import synth
from oracle import lattice, wilson
from tests.gpu_common import ctx, dev, empty, host, make_op, rel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (8, 2, 2, 4)])
def test_tables_bit_exact(dims):
    from paper_0707_0502_amd import gdr
    say("tables", dims)
    op = make_op(synth.unit_links(dims), 0.1)
    eo, nbr, sign = gdr.gdr_op_tables(op)
    e2, n2, s2 = lattice.tables(dims)
    assert np.array_equal(eo, e2)
    assert np.array_equal(nbr, n2)
    assert np.array_equal(sign, s2)
    gdr.gdr_op_destroy(op)


@pytest.mark.parametrize("dims,bc", [((4, 4, 4, 4), (1, 1, 1, -1)), ((2, 4, 6, 8), (1, 1, 1, -1)),
                                     ((6, 4, 2, 4), (1, -1, 1, 1)),
                                     ((4, 8, 4, 8), (-1, 1, -1, -1)), ((8, 4, 4, 4), (1, -1, 1, -1))])
def test_apply_matches_oracle(dims, bc):
    from paper_0707_0502_amd import gdr
    say("apply", dims, bc)
    links = synth.gauge_links(dims, 0.5, 3)
    kappa = 0.137
    sig = -0.13 + 0.05j
    X = np.stack([synth.rhs_gaussian(dims, 10 + v).ravel() for v in range(3)])
    ref = np.stack([wilson.apply_A(links, kappa, x.reshape(dims[::-1] + (4, 3)), sig, bc).ravel()
                    for x in X])
    for storage, prec, tol in [(gdr.GDR_LINKS_F32, gdr.GDR_PREC_F64, 1e-14),
                               (gdr.GDR_LINKS_F32, gdr.GDR_PREC_F32, 1e-6),
                               (gdr.GDR_LINKS_F16, gdr.GDR_PREC_F32, 2e-3)]:
        op = make_op(links, kappa, bc, storage)
        x = dev(X.ravel())
        y = empty(X.size)
        gdr.gdr_op_apply(op, sig, x, y, 3, prec)
        got = host(y).reshape(X.shape)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say("  storage", storage, "prec", prec, "max rel err", err)
        assert err <= tol
        gdr.gdr_op_destroy(op)


def test_apply_many_vectors_and_empty():
    from paper_0707_0502_amd import gdr
    dims = (2, 2, 2, 4)
    links = synth.gauge_links(dims, 0.3, 1)
    op = make_op(links, 0.12)
    nv = 19   # more than one launch chunk
    X = np.stack([synth.rhs_z4(dims, v).ravel() for v in range(nv)])
    y = empty(X.size)
    gdr.gdr_op_apply(op, 0.25, dev(X.ravel()), y, nv, gdr.GDR_PREC_F64)
    got = host(y).reshape(X.shape)
    for v in range(nv):
        ref = wilson.apply_A(links, 0.12, X[v].reshape(dims[::-1] + (4, 3)), 0.25).ravel()
        assert rel(got[v], ref) <= 1e-14
    assert gdr.gdr_op_apply(op, 0.0, dev(X[0]), empty(X[0].size), 0) == gdr.GDR_OK
    gdr.gdr_op_destroy(op)


@pytest.mark.parametrize("dims", [(4, 2, 6, 4), (8, 4, 8, 12)])
@pytest.mark.parametrize("nv", [1, 2, 5, 16, 19])
def test_apply_fp32_batches_against_oracle(dims, nv):
    """FP32 launches over batches of vectors: every vector of every batch size
    matches the oracle to FP32 rounding, with FP32 and FP16-stored links, on
    a lattice with 2-site tile extents (plain kernel) and on one cut into
    2x1x2x3 tiles of 4^4 (halo-staged kernel: faces across tiles, and the
    periodic wrap onto the tile itself in y)."""
    from paper_0707_0502_amd import gdr
    links = synth.gauge_links(dims, 0.4, 7)
    kappa = 0.13
    X = np.stack([synth.rhs_gaussian(dims, 40 + v).ravel() for v in range(nv)])
    ref = np.stack([wilson.apply_A(links, kappa, x.reshape(dims[::-1] + (4, 3)), -0.2).ravel()
                    for x in X])
    for storage, tol in [(gdr.GDR_LINKS_F32, 1e-6), (gdr.GDR_LINKS_F16, 2e-3)]:
        op = make_op(links, kappa, link_storage=storage)
        y = empty(X.size)
        gdr.gdr_op_apply(op, -0.2, dev(X.ravel()), y, nv, gdr.GDR_PREC_F32)
        got = host(y).reshape(X.shape)
        for v in range(nv):
            assert np.abs(got[v] - ref[v]).max() <= tol * np.abs(ref[v]).max(), (nv, storage, v)
        gdr.gdr_op_destroy(op)


def test_gamma5_hermiticity_through_abi():
    from paper_0707_0502_amd import gdr
    dims = (4, 4, 4, 4)
    links = synth.gauge_links(dims, 0.5, 2)
    op = make_op(links, 0.13)
    shape = dims[::-1] + (4, 3)
    x = synth.rhs_gaussian(dims, 1).ravel()
    yv = synth.rhs_gaussian(dims, 2).ravel()
    g5 = lambda v: wilson.gamma5_flat(v, shape)
    a = empty(x.size)
    gdr.gdr_op_apply(op, 0.0, dev(g5(x)), a)
    b = empty(x.size)
    gdr.gdr_op_apply(op, 0.0, dev(yv), b)
    lhs = np.vdot(yv, g5(host(a)))
    rhs = np.vdot(host(b), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)
    gdr.gdr_op_destroy(op)


def test_bad_operator_arguments():
    from paper_0707_0502_amd import gdr
    links = synth.unit_links((2, 2, 2, 2))
    # an odd extent (links sized for it, so the library itself rejects it)
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_wilson_create(ctx(), (3, 2, 2, 2), (1, 1, 1, -1), 0.1,
                              synth.unit_links((3, 2, 2, 2)))
    assert e.value.code == gdr.GDR_ERR_ARG
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_wilson_create(ctx(), (2, 2, 2, 2), (1, 1, 1, 0), 0.1, links)
    assert e.value.code == gdr.GDR_ERR_ARG
    with pytest.raises(gdr.GdrError) as e:
        gdr.gdr_wilson_create(ctx(), (2, 2, 2, 2), (1, 1, 1, -1), 0.1, links, 7)
    assert e.value.code == gdr.GDR_ERR_ARG


@pytest.mark.parametrize("nv", [1, 3, 12])
def test_fp32_link_storage_choice(nv):
    """FP32 storage of special unitary links on 4^4 tiles keeps two rows per
    link (192 B/site) and rebuilds the third in the operator, with the
    antiperiodic factors applied there; a field that is not special unitary
    keeps all nine entries (288 B/site). Both match the oracle to FP32
    rounding, one vector or several per launch, with every direction
    antiperiodic. FP16 storage does the same with half the bytes."""
    from paper_0707_0502_amd import gdr
    dims, bc = (8, 4, 4, 8), (-1, -1, -1, -1)
    kappa, sig = 0.124, 0.07 - 0.02j
    su3 = synth.gauge_links(dims, 0.6, 11)
    rng = np.random.default_rng(12)
    general = su3 * (1.0 + 0.05 * rng.standard_normal(su3.shape[:-2])[..., None, None])
    X = np.stack([synth.rhs_gaussian(dims, 60 + v).ravel() for v in range(nv)])
    for links, want in ((su3, 192), (general, 288)):
        ref = np.stack([wilson.apply_A(links, kappa, x.reshape(dims[::-1] + (4, 3)), sig, bc).ravel()
                        for x in X])
        op = make_op(links, kappa, bc, gdr.GDR_LINKS_F32)
        assert gdr.gdr_op_link_bytes(op, gdr.GDR_PREC_F32) == want
        assert gdr.gdr_op_link_bytes(op, gdr.GDR_PREC_F64) == 576
        y = empty(X.size)
        gdr.gdr_op_apply(op, sig, dev(X.ravel()), y, nv, gdr.GDR_PREC_F32)
        got = host(y).reshape(X.shape)
        err = max(np.abs(got[v] - ref[v]).max() / np.abs(ref[v]).max() for v in range(nv))
        say("  link bytes", want, "nv", nv, "max rel err", err)
        assert err <= 1e-6
        gdr.gdr_op_destroy(op)
    # FP16 storage: two rows (96 B/site) for special unitary links, nine
    # entries (144 B/site) otherwise; both to FP16 rounding
    for links, want in ((su3, 96), (general, 144)):
        ref = np.stack([wilson.apply_A(links, kappa, x.reshape(dims[::-1] + (4, 3)), sig, bc).ravel()
                        for x in X])
        op = make_op(links, kappa, bc, gdr.GDR_LINKS_F16)
        assert gdr.gdr_op_link_bytes(op, gdr.GDR_PREC_F32) == want
        y = empty(X.size)
        gdr.gdr_op_apply(op, sig, dev(X.ravel()), y, nv, gdr.GDR_PREC_F32)
        got = host(y).reshape(X.shape)
        err = max(np.abs(got[v] - ref[v]).max() / np.abs(ref[v]).max() for v in range(nv))
        say("  FP16 link bytes", want, "nv", nv, "max rel err", err)
        assert err <= 2e-3
        gdr.gdr_op_destroy(op)
