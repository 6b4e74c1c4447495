"""The host code of the library (Remez fits, parameter packing, validation,
the batch and server set-up paths, the C ABI) under AddressSanitizer and
UndefinedBehaviorSanitizer: the CPU tests of the ABI run in a child process
against libmact_san.so (build.py --sanitize; host code instrumented, UB
fatal) with the clang ASan runtime preloaded.  CPU only; builds the
sanitized library first when it is missing or older than a source."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1009_0854_amd")


def _stale(lib):
    if not os.path.exists(lib):
        return True
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + [os.path.join(ROOT, "include", "mact.h")]
    return max(os.path.getmtime(s) for s in srcs) > os.path.getmtime(lib)


@pytest.fixture(scope="module")
def san_env():
    from paper_1009_0854_amd import build as B
    rt = B.sanitizer_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this ROCm install")
    if _stale(B.OUT_SAN):
        B.build(jobs=8, sanitize=True)
    env = dict(os.environ, MACT_LIB_VARIANT="san", LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    return env


def test_sanitized_library_is_the_one_loaded(san_env):
    code = ("import paper_1009_0854_amd as M; M.lib(); "
            "maps = open('/proc/self/maps').read(); "
            "assert 'libmact_san.so' in maps and 'libmact.so' not in maps, 'wrong library'; "
            "assert 'libclang_rt.asan' in maps, 'no ASan runtime'; print('ok')")
    r = subprocess.run([sys.executable, "-c", code], env=san_env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-3000:]


def test_abi_host_paths_under_asan_and_ubsan(san_env):
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-m", "not gpu",
                        "-q", "-x", "-p", "no:cacheprovider"],
                       env=san_env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
