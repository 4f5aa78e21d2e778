"""The step-shaped streaming probes (libwave_probe.so: FP32 step, 16-bit
steps, fused adjoint step) that the benchmark
reports as each form's bandwidth ceiling: every measurement first checks one
launch against the probe's definition, cell by cell over the whole padded
fields, so a probe that skipped or misplaced cells would raise here.  Small
ragged grids: tiles and z-chunks with partial last ones."""
import pytest

pytestmark = pytest.mark.gpu


def test_fp32_step_stream_matches_its_definition(wave_mod):
    from paper_2204_03775_amd import probe

    print("case: probe_step_stream 260x37x23, zc 7", flush=True)
    r = probe.measure_step_stream(260, 37, 23, zc=7, launches=2)
    assert r["ascending_gbs"] > 0 and r["alternating_gbs"] > 0


@pytest.mark.parametrize("uv", [False, True])
@pytest.mark.parametrize("ty,ry", [(8, 2), (16, 2), (16, 1)])
def test_16bit_step_stream_matches_its_definition(wave_mod, uv, ty, ry):
    from paper_2204_03775_amd import probe

    print(f"case: probe_step_stream16 260x37x23, zc 7, tile 32x{ty} r{ry}, uv {uv}", flush=True)
    r = probe.measure_step_stream16(260, 37, 23, 7, ty, ry, uv, launches=2)
    assert r["bytes_per_point"] == (10 if uv else 8)
    assert r["ascending_gbs"] > 0 and r["alternating_gbs"] > 0


def test_16bit_step_stream_refuses_bad_shapes(wave_mod):
    # argument checks happen on the host, before any launch
    import torch

    from paper_2204_03775_amd import probe

    lib = probe._load()
    t = torch.zeros(1 << 16, dtype=torch.int16, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    p = t.data_ptr()
    assert lib.probe_step_stream16(p, p, None, p, 6, 4, 4, 64, 8, 4, 8, 2, 0, s) == -1   # nx not a multiple of 4
    assert lib.probe_step_stream16(p, p, None, p, 8, 4, 4, 64, 8, 4, 4, 2, 0, s) == -1   # unsupported tile
    assert lib.probe_step_stream16(p, p, None, p, 64, 4, 4, 64, 8, 4, 8, 2, 0, s) == -1  # pitch too small
    assert lib.probe_step_stream16(p + 2, p, None, p, 8, 4, 4, 64, 8, 4, 8, 2, 0, s) == -1  # misaligned


@pytest.mark.parametrize("ty", [8, 16])
def test_adjoint_stream_matches_its_definition(wave_mod, ty):
    from paper_2204_03775_amd import probe

    print(f"case: probe_adjoint_stream 260x37x23, zc 7, tile 32x{ty}", flush=True)
    r = probe.measure_adjoint_stream(260, 37, 23, 7, ty, launches=2)
    assert r["bytes_per_point"] == 36
    assert r["ascending_gbs"] > 0 and r["alternating_gbs"] > 0
