"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The sanitizer variant of libptyg.so (paper_2106_07575_amd.build with
sanitize=True: -fsanitize=address,undefined on the host pass only, device
code as usual) is built when missing or older than the sources, and the
no-GPU ABI tests (tests/test_abi.py: argument validation, status text,
workspace and tile-list size queries, rejection of short buffers) run
against it in a subprocess with the ASan runtime preloaded.  Any sanitizer
report fails the run (UBSan does not recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_calls_under_sanitizers():
    from paper_2106_07575_amd import build as B
    try:
        B.hipcc()
        rt = B.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    if B.sources_newer_than(B.SAN_LIB):
        B.build(verbose=False, sanitize=True)
    env = dict(os.environ, PTYG_LIBRARY=B.SAN_LIB, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "Sanitizer" not in out and "runtime error" not in out
    assert " passed" in r.stdout and " skipped" not in r.stdout
