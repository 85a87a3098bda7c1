"""Host sanitizer runs (CPU only): the oracle and libhj's argument validation
under AddressSanitizer and UndefinedBehaviorSanitizer (tests/sanitize/).  The
binaries are built by __graft_entry__.build() (or here, if missing)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "sanitize"))
import build as sanitize_build  # noqa: E402


@pytest.fixture(scope="module")
def binaries():
    if not (os.path.exists(sanitize_build.ORACLE_BIN) and os.path.exists(sanitize_build.HJ_BIN)):
        sanitize_build.build()
    return sanitize_build.ORACLE_BIN, sanitize_build.HJ_BIN


def _run(path, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={int(leaks)}:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    p = subprocess.run([path], env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out, out
    return out


def test_oracle_under_address_and_ub_sanitizers(binaries):
    out = _run(binaries[0], leaks=True)
    assert "0 failed checks" in out


def test_libhj_validation_under_address_and_ub_sanitizers(binaries):
    # leak checking off: the HIP runtime keeps allocations until exit
    out = _run(binaries[1], leaks=False)
    assert "0 failures" in out
