"""The library's host code under AddressSanitizer (CPU only): builds the
ASan variant of the library (host compilation instrumented, device code as
usual), links a C driver against it with the same sanitizer runtime, and
runs it: argument checks on NULL handles, context creation without a device,
and the launch-tuning cache reader on corrupt, oversized and binary files.
A memory error aborts the driver; leaks of the library's own allocations
fail it (the HIP runtime's start-up allocations are suppressed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.fixture(scope="module")
def asan_lib():
    if not os.path.exists(CLANG) or shutil.which("/opt/rocm/bin/hipcc") is None:
        pytest.skip("ROCm clang/hipcc not available")
    from paper_0707_0502_amd import build
    return build.build(jobs=8, asan=True)


def test_host_paths_under_asan(asan_lib, tmp_path):
    exe = tmp_path / "asan_driver"
    libdir = os.path.dirname(asan_lib)
    subprocess.check_call([CLANG, "-fsanitize=address", "-fno-omit-frame-pointer", "-g",
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "asan_driver.c"),
                           "-L", libdir, "-lgdr_asan", "-Wl,-rpath," + libdir, "-o", str(exe)])
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n"
                    "leak:libdrm\nleak:libnuma\nleak:librocprofiler\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:abort_on_error=0"
    env["LSAN_OPTIONS"] = "suppressions=%s:print_suppressions=0" % supp
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    r = subprocess.run([str(exe), str(scratch)], capture_output=True, text=True, env=env,
                       timeout=300)
    print(r.stdout)
    print(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
