"""Throughput and roofline arithmetic for the propagator.

Throughput counts interior grid-point updates per second, the unit the
paper's Tables 2 and 3 use (cells x steps / time).  The paper's FLOP rate
counts 51 floating-point operations per cell (Section VI: 25 multiplies and
25 adds for the stencil plus one subtraction for the time update).

Algorithmic HBM bytes per update of the FP32 step: read u^n, u^{n-1} and k,
write u^{n+1}; neighbours are re-used on chip.  Halo re-reads, trace writes
and the sponge profiles are not counted.
"""
from __future__ import annotations

PAPER_FLOP_PER_CELL = 51
BYTES_PER_POINT_F32 = 16
BYTES_PER_POINT_16 = 8  # FP16 / BF16 storage of u^n, u^{n-1}, k and u^{n+1}
BYTES_PER_POINT_16UV = 10  # 16-bit u^n, d^n, k read; u^{n+1}, d^{n+1} written
MI355X_HBM_PEAK_GBS = 8000.0  # published HBM3E bandwidth, GB/s


def gpts_per_s(nx: int, ny: int, nz: int, steps: int, seconds: float) -> float:
    """Interior point updates per second, in units of 1e9."""
    return nx * ny * nz * steps / seconds / 1e9


def paper_tflops(gpts: float) -> float:
    """FLOP rate under the paper's 51-flop-per-cell convention, TFLOP/s."""
    return gpts * PAPER_FLOP_PER_CELL / 1e3


def hbm_gbs(gpts: float, bytes_per_point: int = BYTES_PER_POINT_F32) -> float:
    return gpts * bytes_per_point


def roofline_fraction(gpts: float, bytes_per_point: int = BYTES_PER_POINT_F32,
                      peak_gbs: float = MI355X_HBM_PEAK_GBS) -> float:
    return hbm_gbs(gpts, bytes_per_point) / peak_gbs
