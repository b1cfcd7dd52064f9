"""The benchmark's own logic, on the CPU: the one-GPU contract, the
algorithmic byte model behind the roofline figures, and the link between the
committed profile summaries and the kernel source they were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_1m_sweep():
    """One launch of the simulation-cell kernel at 1,048,576 disks, eta 0.72,
    64 x 64 cells, one chain per disk: 36 B per disk (own id and position read,
    position written), 20 B per disk of the frozen band (about a quarter of
    the disks) and 20 B per chain draw: 61 B per disk, 64.0 MB."""
    n = 1 << 20
    b = bench.cell_kernel_bytes(n, 0.72, 64, n)
    assert abs(b / n - 61.0) < 0.3
    assert abs(b / 1e6 - 64.0) < 0.2
    # the whole sweep adds the rebin kernels (21 + 9 B per disk) and the draws written
    s = bench.sweep_bytes(n, 0.72, 64, n)
    assert abs((s - b) / n - (21 + 9 + 20)) < 1e-9


def test_committed_profiles_match_the_kernel_source():
    """The figures bench.py reads from profiles/ (HBM bytes per launch, cycles
    per event) are taken on the current kernel source; a change of the source
    without new counters would make them null in the bench line."""
    traffic = bench.measured_traffic("k_sweep_cells", "pec_1m")
    cycles = bench.measured_cycles_per_event("k_sweep_cells", "pec_1m")
    assert traffic is not None and 5e7 < traffic < 5e8
    assert cycles is not None and 100 < cycles < 10000
    sha = bench._kernel_source_sha()
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        if "ec_kernels.hip" in text:
            assert sha in text, name
