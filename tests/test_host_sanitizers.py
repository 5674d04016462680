"""The host side of the library (argument checks, layouts, size limits, the
batch and server bookkeeping reached without a GPU) under AddressSanitizer
and UndefinedBehaviorSanitizer (CPU only): the C-ABI tests run in a child
process against libtlb_hostsan.so, with the sanitizer runtime preloaded, and
any report fails them."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


def test_abi_tests_clean_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    from paper_1710_09534_amd import build
    lib = build.SAN_LIB
    if not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib)
                                      for s in build.sources()):
        build.build(sanitize=True)
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "TLB_LIBRARY": lib,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
