"""Build libqsv.so (HIP, gfx950) in-tree: paper_2604_03816_amd/_build/libqsv.so.

Every HIP translation unit is compiled for gfx950 only, with packed FP32 ops
disabled (-packed-fp32-ops), then linked into one shared library that exports the
C ABI of include/qsv.h.

``build(sanitize=True)`` writes a second library, _build_san/libqsv.so, whose host
code (planner, C-ABI layer, server) carries AddressSanitizer and
UndefinedBehaviorSanitizer instrumentation (device code is built as usual).  It is
for host-only tests on the CPU: the process must preload the sanitizer runtime
(``sanitizer_runtime()``) and point the binding at it with QSV_LIB=<path>.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libqsv.so")
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libqsv.so")
# host-side instrumentation only: each sanitizer flag applies to the host compilation
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-shared-libsan", "-O1"]

SOURCES = ["kernels.hip", "planner.cpp", "capi.cpp", "serve.cpp", "noalloc.hip", "sample_sort.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_DIR if sanitize else OUT_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + (SAN_FLAGS if sanitize else []) + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    # hipcc's host pass warns about the device-only feature flag; keep other warnings
    for line in r.stderr.splitlines():
        if "packed-fp32-ops" not in line and line.strip():
            print(line, file=sys.stderr)
    return obj


def build(sanitize: bool = False) -> str:
    out_dir, lib = (SAN_DIR, SAN_LIB) if sanitize else (OUT_DIR, LIB)
    os.makedirs(out_dir, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, lib)
    return lib


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime the sanitized library links against (to be
    preloaded into the host process)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


if __name__ == "__main__":
    print(build(sanitize="--sanitize" in sys.argv))
