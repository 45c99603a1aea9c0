"""Host-only checks of the C-ABI library: it loads, exports every function
include/gdr.h declares, and the ctypes layouts of its structs agree with a
C compiler's view of the header. No GPU call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gdr.h")
LIB = os.path.join(ROOT, "paper_0707_0502_amd", "libgdr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gdr_[a-z_0-9]+)\s*\(", text)))


def test_library_built():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    from paper_0707_0502_amd import gdr
    assert sorted(gdr.SYMBOLS) == names


def test_struct_layouts_match_header(tmp_path):
    from paper_0707_0502_amd import gdr
    src = tmp_path / "lay.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gdr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gdr_params), sizeof(gdr_stats),
         offsetof(gdr_params, tol), offsetof(gdr_params, max_refine), offsetof(gdr_params, galerkin), offsetof(gdr_params, sstep), offsetof(gdr_params, sstep_reorth),
         offsetof(gdr_params, refine_floor),
         offsetof(gdr_stats, mvp_dr), offsetof(gdr_stats, t_phase),
         offsetof(gdr_stats, resid), offsetof(gdr_stats, theta_len),
         offsetof(gdr_stats, k_ms), offsetof(gdr_stats, k_launches));
  return 0;
}
""")
    exe = tmp_path / "lay"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    P, S = gdr.gdr_params, gdr.gdr_stats
    want = [ctypes.sizeof(P), ctypes.sizeof(S), P.tol.offset, P.max_refine.offset, P.galerkin.offset, P.sstep.offset, P.sstep_reorth.offset,
            P.refine_floor.offset,
            S.mvp_dr.offset, S.t_phase.offset, S.resid.offset, S.theta_len.offset,
            S.k_ms.offset, S.k_launches.offset]
    assert got == want


def test_params_default_host_only():
    from paper_0707_0502_amd import gdr
    p = gdr.gdr_params_default()
    assert (p.m_dr, p.k, p.m_proj, p.precision, p.batch, p.profile) == (40, 15, 40, gdr.GDR_PREC_F64, 1, 0)
    assert p.tol == 1e-8 and p.tol_extra == 0
    assert (p.proj_k, p.use_graph, p.galerkin, p.sstep, p.sstep_reorth) == (0, 0, 0, 4, 20.0)
    assert p.refine_floor == 0.0


def test_binding_rejects_missing_library(tmp_path):
    from paper_0707_0502_amd import gdr
    with pytest.raises(ImportError):
        gdr.load(str(tmp_path / "nope.so"))
