"""Graph replay of single runs (wave_set_graph): bit for bit the eager
launches, over several replays with other GPU work and resets in between,
for FP32 and 16-bit storage; a changed source array is captured anew; the
legacy default stream is refused."""
import numpy as np
import pytest
import torch

from paper_2204_03775_amd import inputs

pytestmark = pytest.mark.gpu


def snapshot(prop):
    cur, prev, n = prop.fields()
    return (prop.padded(cur).clone(), prop.padded(prev).clone(), prop.traces.clone(), n)


def same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a[:3], b[:3])) and a[3] == b[3]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16uv"])
def test_graph_replays_equal_eager(wave_mod, dtype):
    p = inputs.small_parity()
    stream = torch.cuda.Stream()
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")

    def make():
        prop = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                                   stream=stream, dtype=dtype)
        prop.record(p.nt)
        return prop

    eager = make()
    eager.run(p.nt, s)
    stream.synchronize()
    ref = snapshot(eager)
    eager.close()

    prop = make()
    prop.use_graph(True)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        print(f"case: graph replay {rep}, {dtype}, 64^3 x {p.nt}", flush=True)
        with torch.cuda.stream(stream):
            prop.reset()
        prop.run(p.nt, s)
        junk.mul_(1.0001)  # other work on the default stream in between
        stream.synchronize()
        assert same(snapshot(prop), ref), rep
    # another source array: captured anew, still the eager result
    s2 = s.clone()
    with torch.cuda.stream(stream):
        prop.reset()
    prop.run(p.nt, s2)
    stream.synchronize()
    assert same(snapshot(prop), ref)
    # runs split in parts replay part by part
    with torch.cuda.stream(stream):
        prop.reset()
    prop.run(37, s)
    prop.run(p.nt - 37, s[37:])
    stream.synchronize()
    assert same(snapshot(prop), ref)
    prop.close()


def test_graph_needs_a_stream(wave_mod):
    p = inputs.random_problem(20, 18, 16, 5, seed=3)
    prop = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src,
                               stream=torch.cuda.default_stream())
    with pytest.raises(wave_mod.WaveError) as e:
        prop.use_graph(True)
    assert e.value.code == wave_mod.WAVE_EINVAL
    prop.close()
