"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message (the propagator runs on one GPU), the paper's
scaling-table figures it prints beside the MI355X rates are the tables'
own values, and the 16-bit pattern probe is left out for tilings it does
not mirror."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_paper_scaling_figures():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2204_03775_amd import inputs

    # every shape of the two tables has its figures, and nothing else
    assert set(bench.PAPER_TABLE2) == set(inputs.PAPER_TABLE2_SHAPES)
    assert set(bench.PAPER_TABLE3) == set(inputs.PAPER_TABLE3_SHAPES)
    # Table 2: throughput = cells x 1000 steps / WSE-2 time (Gcell/s), within
    # the rounding of the printed times
    for (nx, ny, nz), (thr, t_wse, _) in bench.PAPER_TABLE2.items():
        assert abs(nx * ny * nz * 1000 / t_wse / 1e9 - thr) / thr < 0.01
    # Table 3: 100,000 steps
    for (nx, ny, nz), (thr, t_wse) in bench.PAPER_TABLE3.items():
        assert abs(nx * ny * nz * 100000 / t_wse / 1e9 - thr) / thr < 0.01


def test_16bit_probe_is_skipped_for_tilings_it_does_not_cover():
    # the probe mirrors 128-cell-wide tiles of 8, 16 or 32 thread rows; other
    # tilings get no pattern ceiling (None) rather than a mismatched one
    sys.path.insert(0, ROOT)
    import bench

    for name in ("t256x8_r1", "t64x16_r1", "t128x24_r1", "t128x32_r4", "naive", "auto"):
        assert bench.step_stream16(None, name, 128, True) is None, name
