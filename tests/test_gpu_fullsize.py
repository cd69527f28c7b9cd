"""The batched-4096 workload at full size in bench.py's launch
configuration (all three models), sampled graphs against the oracle (tests/fullsize_batch_check.py,
run as a child process so its input generator can fork before any GPU use)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_full_size_batch_sampled_parity():
    script = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_batch_check.py")
    r = subprocess.run([sys.executable, "-u", script], capture_output=True, text=True, timeout=900)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["ok"] and rec["fp32"]["lds"] == 1 and rec["fp32"]["schedule"] == 2
    for leg in ("chordal_fp32", "info_fp32"):
        assert rec[leg]["lds"] == 1 and rec[leg]["schedule"] == 2, leg
