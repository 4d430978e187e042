"""CPU checks under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle and the host code of the HIP library (argument validation, plan and
configuration bookkeeping of the C ABI) are built with both sanitizers, and
the CPU tests that exercise them run in a child process with the clang
sanitizer runtime preloaded.  Any report aborts the child, so the test fails
on the first one."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


def asan_runtime():
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def san_libs():
    if not os.path.exists(CLANG) or asan_runtime() is None:
        pytest.skip("no clang sanitizer runtime")
    import oracle
    from paper_2006_04784_amd import build as B
    return oracle.build(sanitize=True), B.build(verbose=False, sanitize=True)


def test_cpu_suite_under_sanitizers(san_libs):
    ora, lib = san_libs
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               FCH_LIB=lib, FCH_ORACLE_LIB=ora, LD_PRELOAD=asan_runtime())
    tests = ["tests/test_boundary_cpu.py", "tests/test_oracle_transforms.py",
             "tests/test_oracle_model.py", "tests/test_oracle_schemes.py",
             "tests/test_oracle_nn.py", "tests/test_oracle_etd.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
    # the child really ran the sanitized builds
    probe = subprocess.run(
        [sys.executable, "-c",
         "from paper_2006_04784_amd import fch; import oracle; fch.lib(); oracle._load();"
         "m = open('/proc/self/maps').read();"
         "print(all(s in m for s in ('libfch_san.so', 'liboracle_san.so', 'asan')))"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.stdout.strip().endswith("True"), probe.stdout + probe.stderr
