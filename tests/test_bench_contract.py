"""Host-side parts of the benchmark contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_units_and_profile_lookup():
    """Every timed kernel class has algorithmic bytes/flops, and the traffic
    lookup names kernels the profile summary lists (or returns None when the
    kernel sources changed since it was taken)."""
    sys.path.insert(0, ROOT)
    import bench
    assert set(bench.PROFILED_KERNEL) == set(bench.KERNEL_UNITS) == set(bench.STATE_BYTES)
    for cls, (b64, bmx, fl) in bench.KERNEL_UNITS.items():
        assert b64 > bmx > 0 and fl > 0
        assert 0 < bench.STATE_BYTES[cls] <= b64
        for prec in ("fp64", "mixed"):
            t = bench.profiled_traffic(cls, f"cpa512 {prec}")
            assert t is None or t > 0.3 * (b64 if prec == "fp64" else bmx) * 512 ** 3


def test_workload_label_names_the_timed_scheme():
    sys.path.insert(0, ROOT)
    import bench
    lab = bench.workload_label(512)
    assert "512^3" in lab and "MP5" in lab and "SSP-RK3" in lab and "FP64" in lab
    assert "MC" not in lab and "HO" not in lab
    lab = bench.workload_label(256, "mixed", recon="mc", time_order=2)
    assert "linear MC" in lab and "SSP-RK2" in lab and "FP32" in lab
    assert "HO" in bench.workload_label(512, high_order=True)
    # the default run is the 512^3 plain FP64 wave
    import argparse  # noqa: F401
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--n", type=int, default=512)' in src
