"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte counts the roofline divides by, and the rule that a committed traffic
measurement counts only for the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_of_the_transform_kernel():
    """Per site: four links of R reals and G (12 reals) read, Delta (8 reals)
    written, all in doubles; at 32^4 and 12 reals that is 570,425,344 bytes."""
    V = 32 ** 4
    ab = bench.alg_bytes(V, 8, 12)
    assert ab["transform_measure"] == V * 8 * (4 * 12 + 12 + 8) == 570425344
    assert bench.alg_bytes(V, 8, 18)["transform_measure"] == V * 8 * (4 * 18 + 12 + 8)


def test_traffic_counts_only_for_its_sources(tmp_path, monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        rec = json.load(fh)
    key = "transform_measure@32x32x32x32/12"
    assert key in rec and rec[key]["bytes_per_launch"] > 0
    monkeypatch.setattr(bench, "source_digest", lambda: rec[key]["source_digest"])
    assert bench.measured_traffic("transform_measure", (32, 32, 32, 32), 12) == rec[key]["bytes_per_launch"]
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.measured_traffic("transform_measure", (32, 32, 32, 32), 12) is None
