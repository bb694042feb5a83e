"""AddressSanitizer and UBSan on the host, on the CPU: the C oracle (gcc)
under its own tests, and the host code of libslh (validation, sizes and
footprints; hipcc's host pass instrumented, the device code as usual) under
the ABI tests.  Each runs in a child process with the sanitizer runtime
preloaded, and a sanitizer report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _run(env_extra, files):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_and_ubsan():
    from oracle import oracle as O
    O.build(sanitize=True)
    rt = [_gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")]
    if not all(rt):
        pytest.skip("gcc sanitizer runtimes not installed")
    out = _run({"SLH_ORACLE_SANITIZED": "1", "LD_PRELOAD": " ".join(rt),
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
               ["tests/test_oracle_points.py", "tests/test_oracle_mc.py",
                "tests/test_oracle_dg.py", "tests/test_oracle_hybrid.py"])
    assert " passed" in out


def test_host_code_under_asan_and_ubsan():
    from paper_2511_16821_amd import build as B
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("the clang ASan runtime is not installed")
    if not B.sanitized_is_current():
        B.build(sanitize_host=True)
    out = _run({"SLH_LIB": B.SAN_LIB, "LD_PRELOAD": rt[-1],
                "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
               ["tests/test_abi.py"])
    assert " passed" in out
