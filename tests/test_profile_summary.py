"""The counter-summary helper picks kernels by exact name fragments; a
library kernel whose name merely contains the probe's name must not be
taken for it."""
import pytest

from paper_2204_03775_amd import profile_summary as ps


def test_probe_copy_is_not_confused_with_a_library_copy_kernel():
    by_grid = {("(anonymous namespace)::copy_k((anonymous namespace)::f4 const*, f4*, long long)", 79872): [1.0],
               ("void at::native::direct_copy_kernel_cuda(at::TensorIteratorBase&)", 512): [2.0]}
    assert ps.pick(by_grid, ps.PROBE_COPY)[1] == 79872
    by_name = {k[0]: v for k, v in by_grid.items()}
    assert ps.pick(by_name, ps.PROBE_COPY).startswith("(anonymous namespace)::copy_k(")


def test_ambiguous_or_missing_matches_fail_loudly():
    d = {"void wavek::step_tiled<0, 64, 8, 1>(wavek::StepArgs)": [1.0],
         "void wavek::step_tiled<1, 32, 16, 2>(wavek::StepArgs)": [2.0]}
    with pytest.raises(SystemExit):
        ps.pick(d, "step_tiled")
    with pytest.raises(SystemExit):
        ps.pick(d, "step_batch")
    assert ps.pick(d, "step_tiled<0, 64, 8, 1>") in d


def test_overlap_counts_concurrent_time():
    # two queues: [0, 10) and [5, 20) overlap for 5 ns; then [20, 30) alone
    rows = [{"Start_Timestamp": "0", "End_Timestamp": "10", "Queue_Id": "1"},
            {"Start_Timestamp": "5", "End_Timestamp": "20", "Queue_Id": "2"},
            {"Start_Timestamp": "20", "End_Timestamp": "30", "Queue_Id": "1"}]
    n, q, busy, span, multi = ps.overlap_of(rows)
    assert (n, q, busy, span, multi) == (3, 2, 35, 30, 5)
    # back to back on one queue: no overlap
    assert ps.overlap_of(rows[:1] + rows[2:])[4] == 0


def test_occupancy_from_registers_and_lds():
    # 512 threads = 8 waves; 68 registers: 512 // 68 = 7 waves per SIMD,
    # 28 wave slots per CU hold 3 work-groups; 33792 B of LDS allow 4
    assert ps.occupancy(68, 0, 33792, 512) == (3, 6.0)
    # 184 registers: 2 waves per SIMD, one 512-thread work-group per CU
    assert ps.occupancy(184, 0, 0, 512) == (1, 2.0)
    # the LDS binds: 4 work-groups by registers, 2 by 70 KiB of LDS
    assert ps.occupancy(64, 0, 70 * 1024, 512) == (2, 4.0)
    # accumulation registers come out of the same file: 256 in all, 2 waves per SIMD
    assert ps.occupancy(128, 128, 0, 256) == (2, 2.0)
    # no registers reported: the wave limit of 8 per SIMD
    assert ps.occupancy(0, 0, 0, 64) == (32, 8.0)


def test_trace_register_counts_are_doubled_on_granule_8_gpus():
    # what the trace printed for three kernels whose allocation the compiler
    # reports as 130, 176 and 186 registers (136, 176 and 192 allocated)
    assert [ps.allocated_vgprs(n, "gfx950") for n in (68, 88, 96)] == [136, 176, 192]
    assert ps.allocated_vgprs(68, "gfx1100") == 68
