"""Host-side checks of the benchmark's work accounting (no GPU): the sample
counts its roofline divides by equal the oracle's count of (ray, step) pairs
with a tap inside the image, for the parallel and the fan workload shapes,
and several GPUs are refused."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("lvl", [0, 1, 2, 3])
def test_parallel_sample_counts_match_oracle(lvl):
    assert bench.sample_counts(64, 90, 92, lvl) == oracle.count_samples(oracle.Geometry(64, 90, 92), lvl)


@pytest.mark.parametrize("lvl", [0, 1, 2, 3])
def test_fan_sample_counts_match_oracle(lvl):
    g = oracle.Geometry(64, 30, 96, src_dist=4.0, det_dist=2.0)
    assert bench.fan_sample_counts(64, 30, 96, 4.0, 2.0, lvl) == oracle.count_samples(g, lvl)


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
