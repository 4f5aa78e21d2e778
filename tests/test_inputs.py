"""The seeded synthetic workloads match their stated recipes (shapes, time
step, velocities, source and receivers) and are reproducible.  The same
generators feed the oracle and the GPU path, so they hold no propagator
arithmetic; these checks pin them to the recipes the benchmark and the
parity tests quote."""
import math

import numpy as np
import pytest

from paper_2204_03775_amd import inputs


def test_stability_limit_and_time_step():
    # 3-D limit of the 8th-order leapfrog: (v dt / h)^2 * 3 * 2048/315 <= 4
    lim = math.sqrt(4.0 / (3 * 2048 / 315))
    assert inputs.stable_courant_limit(3) == pytest.approx(lim, rel=1e-15)
    # the large shot's dt: 0.8 of the limit at 4500 m/s and h = 10 m
    assert inputs.cfl_dt(4500.0, 10.0, 0.8) == pytest.approx(0.805076e-3, abs=5e-10)


def test_ricker_and_point_source():
    dt, f = 1e-3, 15.0
    w = inputs.ricker(f, 200, dt)
    assert w.shape == (200,) and w.dtype == np.float64
    # peak at t0 = 1/f (66.67 ms: between samples, so the sampled maximum is
    # just under 1), zero crossings at t0 +- 1/(pi f sqrt 2)
    assert np.argmax(w) == round(1 / f / dt) and 0.999 < w.max() < 1.0
    t = np.arange(200) * dt
    cross = 1 / f + np.array([-1, 1]) / (math.pi * f * math.sqrt(2))
    for c in cross:
        i = int(c / dt)
        assert w[i] * w[i + 1] <= 0
    s = inputs.point_source_values(w, 1500.0, dt, (10.0, 10.0, 10.0))
    assert np.allclose(s, (1500.0 * dt) ** 2 * w / 1000.0, rtol=1e-15)


def test_small_parity_workload():
    p = inputs.small_parity()
    assert (p.nx, p.ny, p.nz, p.nt, p.dt) == (64, 64, 64, 100, 1e-3)
    assert p.src == (32, 32, 32) and p.sponge_width == 0
    assert np.all(p.k64() == pytest.approx(2.25))
    rec = p.rec
    assert rec.shape == (16, 3) and len({tuple(r) for r in rec}) == 16
    assert np.all((rec >= 0) & (rec < 64))
    assert np.array_equal(rec, inputs.small_parity().rec)  # seeded


def test_large_shot_workload():
    p = inputs.large_shot()
    assert (p.nx, p.ny, p.nz, p.nt) == (512, 512, 512, 1000)
    assert (p.sponge_width, p.sponge_alpha) == (20, 0.015)
    assert p.src == (25, 256, 256)
    xs = p.rec[:, 2]
    assert p.rec.shape == (256, 3) and np.all(p.rec[:, 0] == 22) and np.all(p.rec[:, 1] == 256)
    assert np.array_equal(xs, [20 + round(r * 471 / 255) for r in range(256)])
    v = p.v
    # five equal layers 1500..4500 m/s, each times (1 + 0.05 p) with |p| <= 1
    for i, base in enumerate([1500.0, 2250.0, 3000.0, 3750.0, 4500.0]):
        layer = v[i * 512 // 5 + 1:(i + 1) * 512 // 5 - 1]
        assert layer.min() >= base * 0.95 * (1 - 1e-6) and layer.max() <= base * 1.05 * (1 + 1e-6)
    assert abs(v / np.repeat(np.array([1500.0, 2250.0, 3000.0, 3750.0, 4500.0], np.float32),
                             [103, 102, 103, 102, 102])[:, None, None] - 1).max() == pytest.approx(0.05, rel=1e-3)
    # stable: the largest Courant number stays under the limit
    assert v.max() * p.dt / 10.0 < inputs.stable_courant_limit(3)


def test_batch_shots_recipe_and_seed():
    a, b = inputs.batch_shots(), inputs.batch_shots()
    assert len(a) == 32
    for p, q in zip(a, b):
        assert (p.nx, p.ny, p.nz) == (q.nx, q.ny, q.nz) and np.array_equal(p.v, q.v)
        assert 96 <= p.nx <= 320 and 96 <= p.ny <= 320 and 96 <= p.nz <= 256
        assert p.nt == 600 and p.sponge_width == 20 and p.rec.shape == (128, 3)
        assert 1500.0 <= p.v.min() and p.v.max() <= 4500.0
        m = 25
        assert all(m <= c < d - m for c, d in zip(p.src, (p.nz, p.ny, p.nx)))


def test_paper_shapes():
    assert len(inputs.PAPER_TABLE2_SHAPES) == 8 and len(inputs.PAPER_TABLE3_SHAPES) == 7
    assert inputs.PAPER_TABLE2_SHAPES[-1] == (755, 994, 1000)
    p = inputs.paper_shape(10, 200, 200, 100)
    assert (p.nx, p.ny, p.nz) == (200, 200, 100) and p.src == (50, 100, 100)
    assert len({tuple(r) for r in p.rec}) == p.rec.shape[0] == 160  # distinct, within the line
