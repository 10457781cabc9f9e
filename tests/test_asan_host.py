"""The library's host translation units under AddressSanitizer (host side
only; the device code is unchanged), driven by tests/asan/host_checks.cpp with
well-formed and malformed descriptors through the validation, scratch sizing,
candidate, register-bound, batch-table and allocation-free entry points.  No
GPU is needed: every call returns before any HIP call."""
import os
import subprocess

from paper_2007_01277_amd import build as B


def test_host_code_is_clean_under_address_sanitizer():
    exe = B.build_asan()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host checks ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr
