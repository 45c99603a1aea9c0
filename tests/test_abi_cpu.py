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
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gdr_params), sizeof(gdr_stats),
         offsetof(gdr_params, tol), offsetof(gdr_params, max_refine), offsetof(gdr_params, galerkin), offsetof(gdr_params, sstep), offsetof(gdr_params, sstep_reorth),
         offsetof(gdr_params, refine_floor), offsetof(gdr_params, persistent),
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
            P.refine_floor.offset, P.persistent.offset,
            S.mvp_dr.offset, S.t_phase.offset, S.resid.offset, S.theta_len.offset,
            S.k_ms.offset, S.k_launches.offset]
    assert got == want


def test_params_default_host_only():
    from paper_0707_0502_amd import gdr
    p = gdr.gdr_params_default()
    assert (p.m_dr, p.k, p.m_proj, p.precision, p.batch, p.profile) == (40, 15, 40, gdr.GDR_PREC_F64, 1, 0)
    assert p.tol == 1e-8 and p.tol_extra == 0
    assert (p.proj_k, p.use_graph, p.galerkin, p.sstep, p.sstep_reorth) == (0, 0, 0, 8, 20.0)
    assert p.refine_floor == 0.0


def test_binding_rejects_missing_library(tmp_path):
    from paper_0707_0502_amd import gdr
    with pytest.raises(ImportError):
        gdr.load(str(tmp_path / "nope.so"))


def test_tune_cache_parser(tmp_path):
    """The launch-tuning cache reader takes well-formed "v1 <key> <form> <us>"
    lines only and survives corrupt, absent and NULL inputs (host code only:
    nothing here touches a device)."""
    lib = ctypes.CDLL(LIB)
    lib.gdr_tune_load.argtypes = [ctypes.c_char_p]
    lib.gdr_tune_report.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    lib.gdr_tune_report.restype = ctypes.c_int64
    f = tmp_path / "tune.txt"
    f.write_bytes(b"v1 dslash_r12|gfx950|8x8x8x16|3|0 1 12.5\n"
                  b"garbage\n\n"
                  b"v2 dslash_r12|gfx950|8x8x8x16|3|0 1 12.5\n"
                  b"v1 blk_update|gfx950|1|1|1|1 -1 3\n"
                  b"v1 blk_update|gfx950|1|1|1|1 8 3\n"
                  b"v1 blk_update|gfx950|1|1|1|1 1 nan\n"
                  b"v1 blk_update|gfx950|1|1|1|1 1 -2\n"
                  b"\xff\xfe\x00 binary\n"
                  b"v1 onlykey\n"
                  b"v1 vcombine|gfx950|7962624|1|3|2 3 0.25\n")
    assert lib.gdr_tune_load(str(f).encode()) == 2
    assert lib.gdr_tune_load(str(tmp_path / "absent.txt").encode()) == -1
    assert lib.gdr_tune_load(None) == -1
    # decisions are reported once a launch has used them; none on the host
    assert lib.gdr_tune_report(None, 0) == 0
    buf = ctypes.create_string_buffer(4)
    assert lib.gdr_tune_report(buf, 4) == 0 and buf.value == b""
