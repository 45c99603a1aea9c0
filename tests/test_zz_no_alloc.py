"""gdr_op_apply_noalloc against gdr_op_apply through the C-ABI: the variant
that keeps its staging buffers in the library's static device workspace
returns the same products, bit for bit (the same kernels on the same
inputs), on two calls in a row with the second on a smaller input, at the
largest size the workspace takes, and rejects a larger operator. The 8^4
products are also checked against the oracle's operator."""
import numpy as np
import pytest

import synth
from oracle import wilson
from tests.gpu_common import ctx, dev, empty, host, make_op, rel, say

pytestmark = pytest.mark.gpu


def _both(gdr, op, sigma, X, nvec, prec):
    x = dev(X.ravel())
    y_ref, y_na = empty(X.size), empty(X.size)
    gdr.gdr_op_apply(op, sigma, x, y_ref, nvec, prec)
    assert gdr.gdr_op_apply_noalloc(op, sigma, x, y_na, nvec, prec) == gdr.GDR_OK
    return host(y_ref), host(y_na)


def test_noalloc_matches_apply_two_calls():
    from paper_0707_0502_amd import gdr
    # call 1: 16^3x32 (n = 1,572,864), FP32, three vectors: the workspace
    # takes two FP32 vectors per chunk, so this runs as two chunks
    dims1 = (16, 16, 16, 32)
    links1 = synth.gauge_links(dims1, 0.5, 0)
    op1 = make_op(links1, 0.12)
    X1 = np.stack([synth.rhs_z4(dims1, 70 + v).ravel() for v in range(3)])
    say("call 1: 16^3x32, FP32, 3 vectors")
    ref1, na1 = _both(gdr, op1, -0.05, X1, 3, gdr.GDR_PREC_F32)
    assert np.array_equal(ref1, na1)
    # call 2, smaller: 8^4, FP64, two vectors, also against the oracle
    dims2 = (8, 8, 8, 8)
    links2 = synth.gauge_links(dims2, 0.3, 0)
    op2 = make_op(links2, 0.12)
    X2 = np.stack([synth.rhs_gaussian(dims2, 80 + v).ravel() for v in range(2)])
    say("call 2: 8^4, FP64, 2 vectors")
    ref2, na2 = _both(gdr, op2, complex(-0.1, 0.02), X2, 2, gdr.GDR_PREC_F64)
    assert np.array_equal(ref2, na2)
    got = na2.reshape(2, -1)
    for v in range(2):
        o = wilson.apply_A(links2, 0.12, X2[v].reshape(dims2[::-1] + (4, 3)),
                           complex(-0.1, 0.02)).ravel()
        assert rel(got[v], o) <= 1e-14
    # and again the larger operator after the smaller one (the workspace keeps
    # the last call's contents; every chunk is written before it is read)
    say("call 3: 16^3x32 again, FP64, 1 vector")
    ref3, na3 = _both(gdr, op1, 0.0, X1[:1], 1, gdr.GDR_PREC_F64)
    assert np.array_equal(ref3, na3)
    gdr.gdr_op_destroy(op1)
    gdr.gdr_op_destroy(op2)


def test_noalloc_size_limit():
    from paper_0707_0502_amd import gdr
    nmax = 1 << 21   # FP64: an input and an output vector fill the 64 MiB
    rng = np.random.default_rng(3)
    d = rng.standard_normal(nmax) + 1j * rng.standard_normal(nmax)
    e = rng.standard_normal(nmax - 1) + 0j
    op = gdr.gdr_bidiag_create(ctx(), d, e)
    x = rng.standard_normal(nmax) + 1j * rng.standard_normal(nmax)
    say("bidiagonal n = 2^21, FP64 and FP32")
    for prec in (gdr.GDR_PREC_F64, gdr.GDR_PREC_F32):
        ref, na = _both(gdr, op, 0.5, x[None, :], 1, prec)
        assert np.array_equal(ref, na)
    gdr.gdr_op_destroy(op)
    big = nmax + 1
    op = gdr.gdr_bidiag_create(ctx(), np.ones(big, complex), np.zeros(big - 1, complex))
    xb, yb = empty(big), empty(big)
    with pytest.raises(gdr.GdrError) as err:
        gdr.gdr_op_apply_noalloc(op, 0.0, xb, yb, 1, gdr.GDR_PREC_F64)
    say("n = 2^21 + 1 in FP64:", err.value)
    assert err.value.code == gdr.GDR_ERR_ARG
    # the same operator fits in FP32 (half the bytes per unknown)
    assert gdr.gdr_op_apply_noalloc(op, 0.0, xb, yb, 1, gdr.GDR_PREC_F32) == gdr.GDR_OK
    gdr.gdr_op_destroy(op)
