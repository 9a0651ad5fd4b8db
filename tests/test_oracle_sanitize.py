"""The oracle's C sources under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's own tests (every tests/test_oracle_*.py) run again in a child
process that loads a sanitizer build of the same sources: any out-of-bounds
access, use after free, signed overflow, misaligned or out-of-range shift in
the reconstruction, network, splatting, target or rasterisation code ends
that process with a report, and the test fails with it.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

import pytest

import oracle

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime() -> str | None:
    try:
        out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                             check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_tests_pass_under_sanitizers(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    files = sorted(f for f in glob.glob(os.path.join(_ROOT, "tests", "test_oracle_*.py"))
                   if os.path.basename(f) != os.path.basename(__file__))
    assert files
    env = dict(os.environ)
    env.update({"LS_ORACLE_LIB": lib,
                # the Python interpreter is not built with the sanitizer, so
                # its runtime goes first; leaks of the interpreter are not ours
                "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "OMP_NUM_THREADS": "4"})
    check = subprocess.run([sys.executable, "-c", "import oracle; oracle._load(); print(oracle._LIB_PATH)"],
                           cwd=_ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert check.returncode == 0, check.stderr[-4000:]
    assert check.stdout.strip() == lib
    run = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                         + files, cwd=_ROOT, env=env, capture_output=True, text=True, timeout=900)
    report = run.stdout[-4000:] + run.stderr[-4000:]
    assert run.returncode == 0, report
    assert "AddressSanitizer" not in run.stderr and "runtime error:" not in run.stderr, report
