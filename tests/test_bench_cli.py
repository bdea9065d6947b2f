"""Host-side checks of bench.py (no GPU work).

* --gpus other than 1 exits with status 2 and one JSON line naming the reason,
  before anything touches a GPU;
* the traffic figure of the roofline object comes from the committed
  counter summary only while that summary was taken on the current operator
  source (its sha256 matches), and is absent for workloads it does not cover.
"""
import hashlib
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        line = json.loads(r.stdout.strip().splitlines()[-1])
        assert "one GPU" in line["error"]


def test_traffic_tracks_the_operator_source():
    prof = os.path.join(ROOT, "profiles", "ax_e_fp64_E4096_N9_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2005_13425_amd", "csrc", "ax_kernels.hip")
    txt = open(prof).read()
    sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt).group(1)
    recorded = float(re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt).group(1))
    current = hashlib.sha256(open(src, "rb").read()).hexdigest()
    got = bench.traffic_bytes(9, 4096)
    if sha == current:
        assert got == recorded
        # the calibrated counters cannot read less than the operator's
        # algorithmic 64 B per point
        assert got >= 64 * 4096 * 1000
    else:
        assert got is None
    assert bench.traffic_bytes(7, 4096) is None
