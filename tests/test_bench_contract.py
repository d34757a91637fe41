"""Host-side parts of the benchmark contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

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


def test_step_bytes_with_intermediates():
    """The bytes a step's kernels must move (intermediates included), from the
    launch counts of one SSP-RK3 step with the fused update: 1 inversion,
    3 x-y and 3 z flux passes, 3 x 3 UCT orientations, 2 fused updates, 1 plain."""
    sys.path.insert(0, ROOT)
    import bench
    steps = 4
    launches = {"c2p": 1, "flux_xy": 3, "flux_z": 3, "uct_x": 3, "uct_y": 3, "uct_z": 3,
                "update": 1, "update_c2p": 2, "dt": 1}
    kernels = {k: {"launches": v * steps} for k, v in launches.items()}
    fp64 = (144 + 3 * 256 + 488 + 9 * 88 + (352 + 416) + 336)
    mixed = (124 + 3 * 128 + 244 + 9 * 48 + (272 + 336) + 276)
    assert bench.step_bytes_with_intermediates(kernels, steps, "fp64") == pytest.approx(fp64)
    assert bench.step_bytes_with_intermediates(kernels, steps, "mixed") == pytest.approx(mixed)
    # without the fusion the plain update runs every stage at its 3-stage average
    plain = {k: {"launches": v * steps} for k, v in launches.items() if k != "update_c2p"}
    plain["update"]["launches"] = 3 * steps
    plain["c2p"]["launches"] = 3 * steps
    assert bench.step_bytes_with_intermediates(plain, steps, "fp64") == pytest.approx(
        3 * 144 + 3 * 256 + 488 + 9 * 88 + 944)


def test_profiled_kernel_names_cover_the_timing_classes():
    """Every timing class of the library except the timestep kernel has
    algorithmic bytes and rocprofv3 names, in both forms."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2401_03008_amd import binding as B
    assert set(B.KCLASS_NAMES) - {"dt"} == set(bench.KERNEL_UNITS)
    assert bench.profiled_name("k_flux_xy<double, false, 0, 4>", True) == \
        "k_flux_xy<float, false, 0, 8>"
    assert bench.profiled_name("k_uct<0, double, 0, true>", True) == "k_uct<0, float, 0, true>"
