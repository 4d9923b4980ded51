"""The host runtime (C ABI, planner, batch builder, serving loop with its
scheduler and completion threads) under AddressSanitizer and
ThreadSanitizer, on the CPU: the library is rebuilt with its host code
instrumented (device code is not), the sanitizer runtime is preloaded into
a fresh interpreter, and the CPU tests of the ABI and of the serving loop
(in its no-device mode, which runs the same admission, batching and
completion code) must pass with no sanitizer report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

REPORTS = ("ERROR: AddressSanitizer", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer")


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_runtime_under_sanitizer(kind):
    from paper_1702_07961_amd import build
    lib = build.build(sanitize=kind)
    rt = build.sanitizer_runtime(kind)
    env = dict(os.environ, MMS_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")
    short = {"address": "asan", "thread": "tsan"}[kind]
    probe = subprocess.run([sys.executable, "-c",
                            "import paper_1702_07961_amd._lib as L; L.lib(); "
                            f"print(open('/proc/self/maps').read().count('libclang_rt.{short}'), L.LIB_PATH)"],
                           env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr
    count, path = probe.stdout.split()
    assert int(count) > 0 and path == lib          # the runtime and the instrumented build are loaded
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_server_dry.py", "tests/test_abi.py"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert not any(tag in out for tag in REPORTS), out[-4000:]
