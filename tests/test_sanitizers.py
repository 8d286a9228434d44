"""Host code of the library under sanitizers (CPU only, no device).

The planner, the C ABI's host side and the planner pool are rebuilt with
AddressSanitizer + UndefinedBehaviorSanitizer, and again with
ThreadSanitizer, and driven by ``tests/sanitize/driver.cpp``: plans of many
shapes, dtypes, splits and schedules, rejected arguments, every host query,
batches prepared in host memory, the planner pool fed and polled from several
threads and destroyed with work pending, fault injection from several threads.
A sanitizer report aborts the driver, so the exit status says it all.
"""
import importlib.util
import os

import pytest

RUNNER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize", "run.py")


def _runner():
    # imported when the test runs, not at collection: a GPU-only test
    # selection must not depend on the sanitizer driver being present
    spec = importlib.util.spec_from_file_location("fht_sanitize_run", RUNNER)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_code_is_sanitizer_clean(kind):
    res = _runner().run(kind)
    assert res.returncode == 0, res.stdout + res.stderr[-6000:]
    assert "sanitizer driver: ok" in res.stdout
