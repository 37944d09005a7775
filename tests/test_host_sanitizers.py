"""The C-ABI's host code and the job server under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: the library's host-sanitizer build
(host pass instrumented, device code as usual; paper_2508_18221_amd.build with
hostsan=True) runs the ABI and dry-server tests in a child process with the
sanitizer runtime preloaded.  Any heap overflow, use after free or undefined
behaviour in the validation, size queries, operator construction, server
bookkeeping (admission, arena, retirement, statistics) aborts the child."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = glob.glob(os.path.join(ROOT, "paper_2508_18221_amd", "csrc", "*")) + \
        glob.glob(os.path.join(ROOT, "include", "*.h"))
    return any(os.path.getmtime(s) > t for s in srcs)


def test_abi_and_server_under_host_sanitizers():
    rt = _runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this ROCm install")
    from paper_2508_18221_amd import build
    lib = build.HOSTSAN_LIB
    if _stale(lib):
        build.build(hostsan=True)
    sym = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in sym and "__ubsan_handle" in sym, "library is not instrumented"
    env = dict(os.environ, GRMHD_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:verify_asan_link_order=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_server_dry.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
