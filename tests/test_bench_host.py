"""CPU checks of the measurement plumbing: the flop count the rates are quoted on, the
roofline's per-launch figures in the committed counter summary, the source-hash guard on the
traffic figure, and the one-GPU contract of bench.py. No GPU calls."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def band_entries(n, p):
    """Nonzeros of an n x n matrix with half-bandwidth p (brute force over the index pairs)."""
    return sum(1 for i in range(n) for j in range(n) if abs(i - j) <= p)


def projected_flops(r0, n, r1, p, R0, R1, ncol):
    """Flops of one operator of the projected local matvec (eq. KKT_red), stage by stage:
    left interface sum over a, banded core over (alpha, j), right interface over (beta, b),
    2 flops per multiply-add, for ncol columns of the block vector."""
    left = 2 * r0 * r0 * R0 * n * r1
    band = 2 * r0 * r1 * R0 * R1 * band_entries(n, p)
    right = 2 * r0 * n * R1 * r1 * r1
    return ncol * (left + band + right)


@pytest.mark.parametrize("shape", [(32, 64, 32, 3, 10, 60), (40, 128, 40, 3, 15, 80), (7, 9, 5, 2, 1, 3),
                                   (3, 4, 2, 3, 2, 2)])
def test_library_flop_count_matches_stagewise_count(shape):
    r, n, r1, p, RM, RK = shape
    from paper_1811_06797_amd import iga
    # the KKT block operator applies M to (y, u, lambda) and K to (y, lambda)
    want = projected_flops(r, n, r1, p, RM, RM, 3) + projected_flops(r, n, r1, p, RK, RK, 2)
    got = iga.local_matvec_flops(r, n, r1, p, RM, RM, RK, RK)
    assert got == pytest.approx(want, rel=1e-15)


def test_c2_shape_flop_figures():
    # the band of a degree-3 factor at n = 64 has 7 n - 2 (3 + 2 + 1) nonzeros
    assert band_entries(64, 3) == 436
    from paper_1811_06797_amd import iga
    assert iga.local_matvec_flops(32, 64, 32, 3, 10, 10, 60, 60) == 7955251200.0
    # the banded K stage (2 columns) is the roofline kernel's work per launch
    txt = open(os.path.join(ROOT, "profiles", "band_stage_K_c2shape_traffic.txt")).read()
    flops = float(re.search(r"^algorithmic_flops_per_launch:\s*(\S+)", txt, re.M).group(1))
    assert flops == pytest.approx(2 * 2 * 32 * 32 * 60 * 60 * 436, rel=1e-6)
    # algorithmic bytes: t1's window read once, t2 written once, the re-laid K core read once
    t1 = (64 + 6) * 60 * 2 * 32 * 32
    t2 = 64 * 60 * 2 * 32 * 32
    core = 64 * 7 * 60 * 60
    nbytes = float(re.search(r"^algorithmic_bytes_per_launch:\s*(\S+)", txt, re.M).group(1))
    assert nbytes == pytest.approx(8 * (t1 + t2 + core), rel=1e-6)


def test_traffic_figure_only_for_matching_kernel_sources(monkeypatch):
    import bench
    if not os.path.exists(bench.TRAFFIC_FILE):
        # no counter summary for the roofline kernel: the line reports traffic as null
        assert bench.traffic_from_profile() is None
        return
    txt = open(bench.TRAFFIC_FILE).read()
    recorded = re.search(r"^source_hash:\s*(\S+)", txt, re.M).group(1)
    traffic = float(re.search(r"^traffic_bytes_per_launch:\s*(\S+)", txt, re.M).group(1))
    if recorded == bench.kernel_source_hash():
        assert bench.traffic_from_profile() == traffic
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.traffic_from_profile() is None


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""
