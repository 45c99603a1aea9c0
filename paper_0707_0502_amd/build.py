"""Build the HIP library libgdr.so for gfx950 with hipcc (in-tree).

usage: python -m paper_0707_0502_amd.build [-j N] [--asan]
(--asan: the host code built with AddressSanitizer into _build_asan/libgdr_asan.so)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgdr.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + SRC, "-I" + INCLUDE, "-Wno-unused-result",
]


# AddressSanitizer build of the host code (device code unchanged), for the
# CPU-only tests of the library's host paths: every -fsanitize= applies to the
# host compilation only
ASAN_OBJ = os.path.join(HERE, "_build_asan")
ASAN_LIB = os.path.join(ASAN_OBJ, "libgdr_asan.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sources():
    return sorted(f for f in os.listdir(SRC) if f.endswith((".hip", ".cpp")))


def _compile(src, asan=False):
    out = os.path.join(ASAN_OBJ if asan else OBJ, src + ".o")
    cmd = [HIPCC] + FLAGS + (ASAN_FLAGS if asan else []) + ["-c", os.path.join(SRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, out, r.returncode, r.stdout + r.stderr


def build(jobs=8, verbose=False, asan=False):
    os.makedirs(ASAN_OBJ if asan else OBJ, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda f: _compile(f, asan), srcs))
    failed = False
    for src, _, rc, log in results:
        noisy = [l for l in log.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if rc != 0:
            failed = True
            sys.stderr.write("compile failed: %s\n%s\n" % (src, "\n".join(noisy)))
        elif verbose and noisy:
            sys.stderr.write("%s:\n%s\n" % (src, "\n".join(noisy)))
    if failed:
        raise RuntimeError("HIP build failed")
    lib = ASAN_LIB if asan else LIB
    tmp = lib + ".tmp"
    cmd = ([HIPCC, "--offload-arch=gfx950", "-shared"] + (["-Xarch_host", "-fsanitize=address"] if asan else [])
           + ["-o", tmp] + [r[1] for r in results])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    j = 8
    if "-j" in sys.argv:
        j = int(sys.argv[sys.argv.index("-j") + 1])
    print(build(j, verbose="-v" in sys.argv, asan="--asan" in sys.argv))
