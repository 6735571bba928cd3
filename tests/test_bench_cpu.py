"""Host side of bench.py: more than one GPU is refused with a message, and the
traffic figure of a committed counter summary is used only while the
kernel sources it was measured with are unchanged."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_needs_matching_sources():
    t = bench.measured_traffic()
    assert t is None or t > 0
    # a source list whose hash the summary does not carry gives no figure
    assert bench.measured_traffic("k_apply_pipe_sphere_h0.02_counters.md", ("schwarz.hip",)) is None
    # the hash covers the named files in order
    assert bench.sources_sha(bench.APPLY_SOURCES) == bench.apply_sources_sha()
    assert bench.sources_sha(("apply.hip", "device.h")) != bench.sources_sha(("device.h", "apply.hip"))
