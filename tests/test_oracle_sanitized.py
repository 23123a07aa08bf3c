"""The CPU reference under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the sanitizer variant of the reference (oracle/build.sh sanitize) and
runs its closed-form pins in a child interpreter with the ASan runtime
preloaded and that build loaded in place of the plain one. Any out-of-bounds
access, use after free or undefined behaviour aborts the child and fails
this test. Leak checking is off: the interpreter itself holds memory at exit.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_lbm3d.py", "tests/test_oracle_np3d.py", "tests/test_oracle_np.py",
        "tests/test_oracle_geometry.py", "tests/test_oracle_potential.py", "tests/test_oracle_np_implicit.py",
        "tests/test_oracle_diagnostics.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's ASan runtime is not installed")
def test_oracle_pins_pass_under_asan_and_ubsan():
    subprocess.run(["sh", os.path.join(ROOT, "oracle", "build.sh"), "sanitize"], check=True)
    env = dict(os.environ)
    env["ORACLE_LIB"] = os.path.join(ROOT, "oracle", "liboracle_san.so")
    env["LD_PRELOAD"] = _runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:xdist", "-m", "not gpu",
                        "-k", "not thread_count", *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1500)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
