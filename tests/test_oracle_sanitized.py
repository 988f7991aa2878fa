"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): its own test files, except the long statistical price and Fig. 3
runs, are run again in a child process against a sanitizer build of the same
sources; any out-of-bounds access, use after free or undefined operation
aborts the child."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["test_oracle_rng.py", "test_oracle_sampler.py", "test_oracle_schemes.py",
         "test_oracle_conditional.py", "test_oracle_rhee_glynn.py", "test_oracle_driver.py",
         "test_oracle_cv.py", "test_oracle_closed_form.py"]


def test_oracle_suite_under_asan_and_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc is not installed")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the gcc AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from oracle import build
    lib = build.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"]
    cmd += [os.path.join(ROOT, "tests", f) for f in FILES]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert "runtime error" not in r.stderr, tail
