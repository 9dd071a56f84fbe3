"""Host-side parts of bench.py's contract (no GPU): the one-GPU refusal, and
the measured-traffic lookup that feeds the roofline entry."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_measured_kernels_and_shape():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    sites = data["sites"]
    region, sweeps = data["region"], data["inner_sweeps"]
    if data["kernel_source_digest"] == bench.kernel_source_digest():
        got = bench.measured_traffic("iterate", sites, region, sweeps)
        assert got == data["kernels"]["iterate"]["bytes_per_site"] * sites
    # Another launch shape, or a kernel class without counters: no figure.
    assert bench.measured_traffic("iterate", sites, "64x16", sweeps) is None
    assert bench.measured_traffic("iterate", sites, region, sweeps + 1) is None
    assert bench.measured_traffic("stage_sweep", sites, region, sweeps) is None


def test_algorithmic_bytes_cover_every_kernel_class():
    # Every class the library's profiler reports has a byte model.
    from paper_2003_04345_amd import mb4 as M
    lib = M.load_library()
    names = [lib.mb4_profile_name(k).decode() for k in range(lib.mb4_profile_classes())]
    assert set(names) <= set(bench.BYTES_PER_SITE)
