"""The serving pool's host runtime (gbees.cpp) on the CPU, under
AddressSanitizer and ThreadSanitizer, against a fake HIP backend
(tests/fakehip/): streams are worker threads that run copies and fake kernels
after the enqueuing call returns, as a GPU does, so lifetime and ordering
mistakes of host memory that the device reads or writes show up as sanitizer
reports.  The stress driver runs groups of eight requests per driver thread,
fetches results from four threads (every fifth request from two threads at
once), releases them, and sends requests past their capacity (rolled back and
moved into larger slices, or failed when the arena is full).

Defects this found and that are fixed: two concurrent gbees_pool_result calls
for one request freed its context under the other (heap-use-after-free), and
a new context's Dev block was modified while its upload copy could still be
reading it (data race)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "fakehip"))


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_pool_stress_under_sanitizer(kind, tmp_path):
    import build as fake_build
    exe = fake_build.build(kind, out_dir=str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1", TSAN_OPTIONS="halt_on_error=1")
    for _ in range(2):
        r = subprocess.run([exe, "300"], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "pool_stress ok" in r.stdout
        assert "after a resize" in r.stdout and " 0 after a resize" not in r.stdout
