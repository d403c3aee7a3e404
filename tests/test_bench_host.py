"""Host-side checks of bench.py: the tunings the GPU tests pin are the ones the
bench times, the counter-measured traffic is reported only for the tuning
and kernel sources it was taken on, and the multi-GPU request is refused."""
import hashlib
import os
import subprocess
import sys

import bench
# the GPU tests' modules: importing them touches no GPU
from tests import test_gpu_bench_config as c2cfg
from tests import test_gpu_stress as c5cfg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gpu_tests_pin_the_bench_tunings():
    assert c2cfg.BENCH_TUNING == bench.TRAFFIC["tuning"]
    assert c2cfg.FP64_TUNING == bench.FP64_TUNING
    assert c5cfg.C5_PINNED == bench.C5_TUNING


def test_traffic_only_for_the_tuning_and_sources_it_was_taken_on(monkeypatch):
    t = dict(bench.TRAFFIC["tuning"], field=0, seconds=0.0)
    kernel = "PCG_APPLY (f32)"

    def sha16(name):
        with open(os.path.join(ROOT, "paper_2111_11788_amd", "csrc", name), "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:16]

    srcs_match = all(sha16(name) == want for name, want in bench.TRAFFIC["sha256_16"].items())
    got = bench.measured_traffic(kernel, t)
    assert got == (bench.TRAFFIC["bytes_per_launch"][kernel] if srcs_match else None)
    # another batch size changes the launch mix: no counter figure
    assert bench.measured_traffic(kernel, dict(t, max_batch=1024)) is None
    # a kernel class without counters
    assert bench.measured_traffic("COARSEST (f32)", t) is None
    # a changed kernel source: no counter figure
    sha = dict(bench.TRAFFIC["sha256_16"], **{"stencil.hip": "0" * 16})
    monkeypatch.setitem(bench.TRAFFIC, "sha256_16", sha)
    assert bench.measured_traffic(kernel, t) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
