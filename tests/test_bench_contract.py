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


def _counter_csv(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (kernel, value) in enumerate(rows):
            fh.write(f'{i},"{kernel}",{counter},{value}\n')


def test_traffic_summary_from_counter_runs(tmp_path):
    # Synthetic counter CSVs in rocprofv3's layout: the copy calibrates the
    # counters (FETCH_SIZE reading half of the bytes moved), the k_iterate
    # dispatches alternate between the 48 and the 16 B/site writers.
    mib, sites = 512, bench.L.CONFIGS["lattice2048"].sites
    kib_per_site = sites / 1024.0

    def k(name):
        return f"void mb4::(anonymous namespace)::{name}(mb4::Lattice, int)"

    it = k("k_iterate<32, 32, 2, double>")
    first, prev = k("k_stage_solve<32, 32, 2, 2, double>"), k("k_stage_solve<32, 32, 2, 3, double>")
    fin = "mb4::(anonymous namespace)::k_final_update(mb4::Lattice, int)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(str(tmp_path / "pmc_fetch_copy" / "copy_counter_collection.csv"), "FETCH_SIZE",
                 [(copy, mib * 1024 / 2)] * 3)
    _counter_csv(str(tmp_path / "pmc_write_copy" / "copy_counter_collection.csv"), "WRITE_SIZE",
                 [(copy, mib * 1024)] * 3)
    _counter_csv(str(tmp_path / "pmc_fetch" / "bench_counter_collection.csv"), "FETCH_SIZE",
                 [(first, 13 * kib_per_site), (it, 38 * kib_per_site), (it, 37 * kib_per_site),
                  (prev, 21 * kib_per_site), (it, 38 * kib_per_site), (it, 37 * kib_per_site),
                  (fin, 16 * kib_per_site)])
    _counter_csv(str(tmp_path / "pmc_write" / "bench_counter_collection.csv"), "WRITE_SIZE",
                 [(first, 48 * kib_per_site), (it, 48 * kib_per_site), (it, 16 * kib_per_site),
                  (prev, 64 * kib_per_site), (it, 48 * kib_per_site), (it, 16 * kib_per_site),
                  (fin, 16 * kib_per_site)])
    out = tmp_path / "traffic.json"
    assert bench.write_traffic(str(tmp_path), str(out), copy_mib=mib) == 0
    data = json.loads(out.read_text())
    assert data["calibration"] == {"copy_mib": 512, "fetch_factor": 2.0, "write_factor": 1.0}
    assert data["kernel_source_digest"] == bench.kernel_source_digest()
    kern = data["kernels"]
    assert kern["iterate"]["bytes_per_site"] == 76 + 48 and kern["iterate"]["dispatches"] == 2
    assert kern["iterate_last"]["bytes_per_site"] == 74 + 16
    assert kern["stage_solve_first"]["bytes_per_site"] == 26 + 48
    assert kern["final_first"]["bytes_per_site"] == 42 + 64
    assert kern["final_update"]["bytes_per_site"] == 32 + 16
