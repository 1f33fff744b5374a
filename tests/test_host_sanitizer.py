"""The host side of libqsv (DAG fusion planner, pass scheduling and device-table
construction, host re-enactment of the tables, the serving core's admission and
scheduling in dry-run mode, argument checking of the C ABI) under AddressSanitizer and
UndefinedBehaviorSanitizer: the planner and serving CPU test modules run again, in a
child process, against a build whose host code is instrumented.  Any out-of-bounds
access, use after free, overflow or other undefined behaviour aborts that run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2604_03816_amd import build as qsv_build  # noqa: E402


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(qsv_build.CSRC, f) for f in os.listdir(qsv_build.CSRC)]
    srcs.append(os.path.join(ROOT, "include", "qsv.h"))
    return any(os.path.getmtime(f) > t for f in srcs)


@pytest.mark.slow
def test_planner_and_server_host_code_under_asan_and_ubsan():
    lib = qsv_build.SAN_LIB
    if _stale(lib):
        qsv_build.build(sanitize=True)
    runtime = qsv_build.sanitizer_runtime()
    assert os.path.exists(runtime), runtime
    env = dict(os.environ, QSV_LIB=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",      # the interpreter itself leaks
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_planner.py"), os.path.join(ROOT, "tests", "test_serve.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    # the child really ran the instrumented library
    probe = subprocess.run([sys.executable, "-c",
                            "from paper_2604_03816_amd import qsv; qsv.lib(); print(qsv.LIB_PATH); "
                            "print(open('/proc/self/maps').read().count('_build_san/libqsv.so') > 0)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0 and probe.stdout.split() == [lib, "True"], probe.stdout + probe.stderr
