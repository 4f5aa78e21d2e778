"""Failure detection and resume.

  - the non-finite watchdog (wave_check) reads zero on a healthy run and
    counts the cells and trace values a planted NaN reaches (FP32 and FP16
    bit patterns; the NaN is written from the host, no kernel faults);
  - resume: 100 steps in one run equal, bit for bit, 50 steps, a new
    context started from the saved (u^n, u^{n-1}) and 50 more steps with
    the source values offset (the oracle's restart is pinned on the CPU);
  - the binding refuses source arrays too short or of the wrong type."""
import numpy as np
import pytest
import torch

from paper_2204_03775_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prob():
    return inputs.random_problem(40, 36, 30, 100, seed=21, sponge_width=4, nrec=12)


def make(wave, p, **kw):
    prop = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                           sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, **kw)
    prop.record(p.nt)
    return prop


def test_watchdog_clean_run(wave_mod, prob):
    p = prob
    prop = make(wave_mod, p)
    prop.run(p.nt, torch.tensor(p.s, dtype=torch.float32, device="cuda"))
    assert prop.check() == (0, 0)
    prop.close()


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_watchdog_counts_a_planted_nan(wave_mod, prob, dtype):
    p = prob
    prop = make(wave_mod, p, dtype=dtype)
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    prop.run(10, s)
    prop.sync()
    cur, _, _ = prop.fields()
    z, y, x = (int(v) for v in p.rec[0])
    view = prop.interior(cur)
    if dtype == "f32":
        view[z, y, x] = float("nan")
    else:
        view.view(torch.int16)[z, y, x] = 0x7E00  # an FP16 NaN
    torch.cuda.synchronize()
    f0, t0 = prop.check()
    assert f0 == 1 and t0 == 0
    prop.run(3, s[10:])
    f1, t1 = prop.check()
    print(f"{dtype}: non-finite cells {f1}, trace values {t1}")
    assert f1 > 1 and t1 >= 1
    prop.close()


def test_resume_is_bitwise(wave_mod, prob):
    p = prob
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    full = make(wave_mod, p)
    full.run(p.nt, s)
    full.sync()
    cur, prev, _ = full.fields()
    ref = (full.interior(cur).clone(), full.interior(prev).clone(), full.traces.clone())
    full.close()

    half = make(wave_mod, p)
    half.run(50, s)
    half.sync()
    cur, prev, _ = half.fields()
    saved = (half.interior(cur).cpu().numpy(), half.interior(prev).cpu().numpy())
    first = half.traces[:50].clone()
    half.close()

    resumed = make(wave_mod, p, u_cur=saved[0], u_prev=saved[1])
    resumed.run(p.nt - 50, s[50:])
    resumed.sync()
    cur, prev, _ = resumed.fields()
    assert torch.equal(resumed.interior(cur), ref[0])
    assert torch.equal(resumed.interior(prev), ref[1])
    assert torch.equal(first, ref[2][:50])
    assert torch.equal(resumed.traces[:p.nt - 50], ref[2][50:])
    resumed.close()


def test_binding_refuses_short_or_wrong_arrays(wave_mod, prob):
    """The library reads source values without knowing the array's length,
    so the binding refuses what would be read past its end, and arrays of
    the wrong type, before anything is enqueued."""
    p = prob
    prop = make(wave_mod, p)
    short = torch.zeros(p.nt - 1, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="needed"):
        prop.run(p.nt, short)
    with pytest.raises(ValueError, match="FP32"):
        prop.run(4, torch.zeros(8, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="FP32"):
        prop.run(4, torch.zeros(8, dtype=torch.float32))  # host memory
    with pytest.raises(ValueError, match="needed"):
        prop.forward_checkpointed(p.nt, short)
    b = wave_mod.Batch([prop])
    with pytest.raises(ValueError, match="needed"):
        b.run(p.nt, [short])
    b.close()
    assert wave_mod.wave_fields(prop.ctx)[2] == 0  # nothing ran
    prop.close()
