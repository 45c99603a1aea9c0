"""Launch tuning on the GPU: every form the tuner may pick for a launch gives
bit-identical results (which also match the oracle), decisions show up in the
report, and a decision read from a cache file is used as read."""
import os

import numpy as np
import pytest

import synth
from oracle import wilson
from tests.gpu_common import dev, empty, host, make_op, say, torch_mod

pytestmark = pytest.mark.gpu


def _tuning_on():
    return os.environ.get("GDR_TUNE", "1") != "0"


def _arch():
    return torch_mod().cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _applies(op, X, nv, sig, reps):
    from paper_0707_0502_amd import gdr
    x = dev(X.ravel())
    outs = []
    for _ in range(reps):
        y = empty(X.size)
        gdr.gdr_op_apply(op, sig, x, y, nv, gdr.GDR_PREC_F32)
        outs.append(host(y))   # synchronises, so the timings of earlier launches are complete
    return outs


@pytest.mark.parametrize("nv", [1, 4])
def test_tuned_forms_are_bit_identical(nv):
    """8x8x8x16 has even tile counts in z and t, so both tile orders are
    candidates, and with several vectors both operator kernels: 2 or 4 forms,
    each timed 3 times, then the decision. Every apply is the same bits."""
    from paper_0707_0502_amd import gdr
    if not _tuning_on():
        pytest.skip("tuning switched off (GDR_TUNE=0)")
    dims, bc = (8, 8, 8, 16), (1, 1, 1, -1)
    kappa, sig = 0.125, 0.05 + 0.01j
    links = synth.gauge_links(dims, 0.5, 21)
    X = np.stack([synth.rhs_gaussian(dims, 80 + v).ravel() for v in range(nv)])
    op = make_op(links, kappa, bc, gdr.GDR_LINKS_F32)
    nform = 4 if nv > 1 else 2
    say("tune forms", dims, "nv", nv, "forms", nform)
    outs = _applies(op, X, nv, sig, 3 * nform + 2)
    for o in outs[1:]:
        assert np.array_equal(o.view(np.float64), outs[0].view(np.float64))
    ref = np.stack([wilson.apply_A(links, kappa, x.reshape(dims[::-1] + (4, 3)), sig, bc).ravel()
                    for x in X])
    got = outs[0].reshape(X.shape)
    err = max(np.abs(got[v] - ref[v]).max() / np.abs(ref[v]).max() for v in range(nv))
    assert err <= 1e-6
    rep = gdr.gdr_tune_report()
    say(rep)
    line = [l for l in rep.splitlines()
            if l.startswith("dslash_r12|%s|8x8x8x16|%d|0 -> " % (_arch(), nv))]
    assert len(line) == 1
    assert 0 <= int(line[0].split("->")[1].split()[0]) < nform
    gdr.gdr_op_destroy(op)


def test_cached_decision_is_used(tmp_path):
    """A decision in a cache file (here the non-default second operator form
    for a shape this process has not launched) is taken without timing; a
    corrupt file contributes nothing and breaks nothing."""
    from paper_0707_0502_amd import gdr
    if not _tuning_on():
        pytest.skip("tuning switched off (GDR_TUNE=0)")
    bad = tmp_path / "corrupt.txt"
    bad.write_bytes(b"v1\nv9 dslash_r12|x|y 1 2\n\xff\xfe garbage\nv1 k|a|s -3 1.0\nv1 k|a|s 2 nan\n")
    assert gdr.gdr_tune_load(str(bad)) == 0
    assert gdr.gdr_tune_load(str(tmp_path / "absent.txt")) == gdr.GDR_ERR_ARG
    dims, bc = (8, 8, 4, 8), (1, 1, 1, -1)   # nt = 2,2,1,2: one tile order
    kappa, sig = 0.12, 0.1
    key = "dslash_r12|%s|8x8x4x8|3|0" % _arch()
    good = tmp_path / "tune.txt"
    good.write_text("v1 %s 1 7.25\n" % key)
    assert gdr.gdr_tune_load(str(good)) == 1
    links = synth.gauge_links(dims, 0.5, 22)
    X = np.stack([synth.rhs_gaussian(dims, 90 + v).ravel() for v in range(3)])
    op = make_op(links, kappa, bc, gdr.GDR_LINKS_F32)
    outs = _applies(op, X, 3, sig, 2)
    assert np.array_equal(outs[0].view(np.float64), outs[1].view(np.float64))
    rep = gdr.gdr_tune_report()
    say(rep)
    assert (key + " -> 1 (7.25 us per unit)") in rep.splitlines()
    ref = np.stack([wilson.apply_A(links, kappa, x.reshape(dims[::-1] + (4, 3)), sig, bc).ravel()
                    for x in X])
    got = outs[0].reshape(X.shape)
    assert max(np.abs(got[v] - ref[v]).max() / np.abs(ref[v]).max() for v in range(3)) <= 1e-6
    gdr.gdr_op_destroy(op)
