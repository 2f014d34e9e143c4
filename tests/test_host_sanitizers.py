"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The host sources (problem validation, operator tables, triangle meshes,
workspace layout, argument checks) are compiled with both sanitizers into a
separate library; a child process preloads the sanitizer runtime and drives
every host-only path through the C ABI (tests/sanitize_driver.py).  Any
out-of-bounds access, use after free or undefined operation aborts the child
with a report."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized_lib():
    sys.path.insert(0, ROOT)
    from paper_2112_05946_amd import build
    rt = build.sanitizer_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime next to hipcc")
    return build.build_sanitized(reuse_device_objects=True), rt


def test_host_paths_are_clean_under_asan_and_ubsan(sanitized_lib):
    lib, rt = sanitized_lib
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, PYTHONMALLOC="malloc",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_driver.py"), lib],
                       capture_output=True, text=True, env=env, timeout=600)
    report = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, report
    assert "sanitized host checks passed" in r.stdout, report
