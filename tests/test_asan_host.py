"""The host side of the library (argument and state checks, the weight-table
fit, the host-only context) under AddressSanitizer: build.py --asan
instruments the host code, and the ABI tests run against that build in a
fresh interpreter with the sanitizer runtime preloaded.  Any invalid access
or use after free in the host code aborts that run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_run_clean_under_address_sanitizer():
    from paper_2110_15113_amd import build
    try:
        lib = build.build(asan=True)
    except RuntimeError as e:
        pytest.skip(f"AddressSanitizer build unavailable: {e}")
    rt = build.asan_runtime()
    if not rt or not os.path.exists(rt):
        pytest.skip("AddressSanitizer runtime not found")
    env = dict(os.environ, ORAS_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
