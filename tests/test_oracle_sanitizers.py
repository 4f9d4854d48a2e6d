"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds oracle/pdf_oracle.c with tests/oracle_sanitize_main.c (a driver that
calls every exported oracle function on edge-case grids and points) using gcc
with both sanitizers and no recovery, runs it, and requires a clean exit.
Host code only; the GPU library is not involved.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", *flags,
                    "-o", exe, os.path.join(ROOT, "oracle", "pdf_oracle.c"),
                    os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-lm", "-lpthread"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "oracle sanitizer run clean" in r.stdout
