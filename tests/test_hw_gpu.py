"""The model against the hardware: a short validation run in its own process
(GPU_MAX_HW_QUEUES=16 must be set before HIP initialises).  Checks that the
run completes and reports finite, positive makespans and a rank correlation;
the correlation itself is a finding, not a pass/fail criterion."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_hardware_validation_run():
    env = dict(os.environ, GPU_MAX_HW_QUEUES="16")
    cmd = [sys.executable, "-u", "-m", "paper_1511_07983_amd.hw", "--sets", "2", "--random-orders", "3",
           "--target-ms", "20", "--reps", "1", "--mem-blocks", "64,100000"]
    print("[hw-gpu]", " ".join(cmd), file=sys.stderr, flush=True)
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout[-3000:], r.stderr[-2000:], file=sys.stderr, flush=True)
    assert r.returncode == 0
    lines = [json.loads(l) for l in r.stdout.splitlines() if l.startswith("{")]
    rows = [l for l in lines if "set" in l]
    assert len(rows) == 2
    for row in rows:
        m = np.array(row["measured_ms"])
        assert len(m) == 4 and np.all(np.isfinite(m)) and np.all(m > 0)
        assert np.all(np.array(row["simulated_cycles"]) > 0)
        assert -1.0 <= row["spearman"] <= 1.0
        # contention never shortens an order; a cap no set reaches changes nothing
        assert set(row["spearman_contended"]) == {"64", "100000"}
        assert row["spearman_contended"]["100000"] == row["spearman"]
    assert lines[-1].get("summary")
