"""Host code of the library under sanitizers (CPU only, no device).

The planner, the C ABI's host side and the planner pool are rebuilt with
AddressSanitizer + UndefinedBehaviorSanitizer, and again with
ThreadSanitizer, and driven by ``tests/sanitize/driver.cpp``: plans of many
shapes, dtypes, splits and schedules, rejected arguments, every host query,
batches prepared in host memory, the planner pool fed and polled from several
threads and destroyed with work pending, fault injection from several threads.
A sanitizer report aborts the driver, so the exit status says it all.
"""
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize"))
import run as sanitize_run  # noqa: E402


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_code_is_sanitizer_clean(kind):
    res = sanitize_run.run(kind)
    assert res.returncode == 0, res.stdout + res.stderr[-6000:]
    assert "sanitizer driver: ok" in res.stdout
