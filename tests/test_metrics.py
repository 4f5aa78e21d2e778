"""The benchmark's metric arithmetic against the paper's own tables
(Section V-B Table 2 and Table 3; Section VI for the 51-flop convention)."""
import pytest

from _pins import read_table
from paper_2204_03775_amd import metrics


def test_table2_throughput_definition():
    # Gcell/s = nx * ny * nz * 1000 steps / time; times carry 4 digits.
    for nx, ny, nz, g, t, _ in read_table("table2_weak_scaling.txt"):
        got = metrics.gpts_per_s(int(nx), int(ny), int(nz), 1000, float(t))
        assert got == pytest.approx(float(g), rel=1e-3), (nx, ny)


def test_table3_throughput_definition():
    for nz, b, g, t, _ in read_table("table3_nz_sweep.txt"):
        got = metrics.gpts_per_s(755, 994, int(nz), 100000, float(t))
        assert got == pytest.approx(float(g), rel=1e-3), nz


def test_paper_flop_rate():
    # 51 flop per cell at the largest Table 2 row gives the 503 TFLOP/s of
    # Section VI, and 670 MFLOP/s per processing element over 755 x 994.
    g = float(read_table("table2_weak_scaling.txt")[-1][3])
    tf = metrics.paper_tflops(g)
    assert tf == pytest.approx(503.0, abs=0.5)
    assert tf * 1e6 / (755 * 994) == pytest.approx(670.3, abs=0.5)


def test_roofline_arithmetic():
    assert metrics.hbm_gbs(500.0) == 8000.0
    assert metrics.roofline_fraction(350.0) == pytest.approx(0.7)
