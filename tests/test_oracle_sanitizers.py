"""The CPU oracle under AddressSanitizer + UBSan and ThreadSanitizer (gcc, host only).

``oracle/sanitize.sh`` builds the oracle's C source with each sanitizer and runs its pin
tests against those builds; any out-of-bounds access, undefined behaviour or data race in
the oracle (including its threaded form) aborts the run and fails this test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPT = os.path.join(ROOT, "oracle", "sanitize.sh")


def _runtime(name):
    if not shutil.which("gcc"):
        return None
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(not (_runtime("libasan.so") and _runtime("libtsan.so")),
                    reason="gcc sanitizer runtimes not available")
def test_checker_is_clean_under_sanitizers():
    env = dict(os.environ, PYTHON=sys.executable)
    res = subprocess.run(["bash", SCRIPT], capture_output=True, text=True, timeout=900,
                         cwd=ROOT, env=env)
    assert res.returncode == 0, (res.stdout[-3000:], res.stderr[-3000:])
    assert res.stdout.count(" passed") == 2, res.stdout[-2000:]
