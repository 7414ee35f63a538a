"""Every C-ABI argument-error path, on the CPU: a context without a device
(OICA_NO_DEVICE) returns each documented code, and OICA_E_DEVICE where device
work would begin.  Run twice: against the library as built, and against a copy
whose host code is instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer (any report fails the test)."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import abi_args_cases  # noqa: E402


def test_argument_errors():
    from paper_2408_17118_amd import oica
    if not os.path.exists(oica.lib_path()):
        pytest.skip("liboica.so not built")
    assert abi_args_cases.run(oica.load()) == []


@pytest.mark.slow
def test_argument_errors_under_sanitizers():
    from paper_2408_17118_amd import build
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no ASan runtime in this toolchain")
    lib = build.build(san=True)
    env = dict(os.environ, LD_PRELOAD=rt[-1],
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "abi_args_cases.py"), lib],
                       capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 mismatches" in out
