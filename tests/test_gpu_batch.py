"""Batched multi-shot runs: one persistent launch per step for many shots
(schedule 0), every shot with its own kernel over several streams
(schedule 1), one launch for the whole run with shots pinned to XCDs and
per-tile step counters (schedule 2, switched off), or one cooperative
launch for the whole run with a grid barrier between steps (schedule 3),
optionally replayed from a HIP graph.

Exact: every shot of a batch reproduces, bit for bit, the same shot run
alone with the same kernel configuration -- fields, buffer roles and
traces -- for mixed sizes, kernel variants (several launch groups) and
storage types, eagerly and from a graph replayed several times with other
work in between.  Spot checks against the FP64 oracle: rel-L2 <= 1e-5."""
import numpy as np
import pytest
import torch

from paper_2204_03775_amd import inputs

pytestmark = pytest.mark.gpu


def make_shots():
    sizes = [(41, 37, 29), (64, 48, 40), (97, 33, 21), (30, 70, 45), (128, 16, 24), (56, 56, 56)]
    return [inputs.random_problem(nx, ny, nz, 23, seed=100 + i, sponge_width=4, nrec=7)
            for i, (nx, ny, nz) in enumerate(sizes)]


CONFIGS = [("t256x8_r1", 0), ("t64x16_r1", 16), ("t128x8_r1", 7), ("t64x32_r2", 0),
           ("t128x16_r1", 24), ("t256x8_r1", 56)]


def build(wave, shots, dtype="f32", configs=CONFIGS):
    props = []
    for p, (v, zc) in zip(shots, configs):
        pr = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dtype)
        pr.configure(v, zc)
        pr.record(p.nt)
        props.append(pr)
    srcs = [torch.tensor(p.s, dtype=torch.float32, device="cuda") for p in shots]
    return props, srcs


def snapshot(pr):
    cur, prev, n = pr.fields()
    view = torch.int16 if cur.element_size() == 2 else torch.int32
    return (pr.padded(cur).view(view).cpu().numpy().copy(),
            pr.padded(prev).view(view).cpu().numpy().copy(),
            pr.traces.cpu().numpy().copy(), n, cur.data_ptr() == pr.buf[0].data_ptr())


def alone(wave, shots, dtype):
    props, srcs = build(wave, shots, dtype)
    out = []
    for pr, s, p in zip(props, srcs, shots):
        pr.run(p.nt, s)
        pr.sync()
        out.append(snapshot(pr))
        pr.close()
    return out


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3])) and a[3:] == b[3:]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_individual_runs(wave_mod, dtype, graph):
    shots = make_shots()
    ref = alone(wave_mod, shots, dtype)
    props, srcs = build(wave_mod, shots, dtype)
    b = wave_mod.Batch(props, use_graph=graph)
    groups, _, pts = b.info()
    assert groups == 5 and pts == sum(p.points for p in shots)
    nt = shots[0].nt
    # split the run (odd + even part) to exercise the role bookkeeping
    b.run(9, srcs)
    b.run(nt - 9, [s[9:] for s in srcs])
    b.sync()
    for i, pr in enumerate(props):
        print(f"case: {dtype} graph={graph} shot {i} {shots[i].name}", flush=True)
        assert same(snapshot(pr), ref[i]), i
    b.close()
    for pr in props:
        pr.close()


def test_graph_replays_match_eager(wave_mod):
    shots = make_shots()
    ref = alone(wave_mod, shots, "f32")
    props, srcs = build(wave_mod, shots, "f32")
    b = wave_mod.Batch(props, use_graph=True)
    nt = shots[0].nt
    for rep in range(4):
        for pr in props:
            pr.reset()
        junk = torch.randn(1 << 20, device="cuda").sum().item()  # eager work in between
        b.run(nt, srcs)
        b.sync()
        for i, pr in enumerate(props):
            assert same(snapshot(pr), ref[i]), (rep, i)
        assert np.isfinite(junk)
    b.close()
    for pr in props:
        pr.close()


def test_batch_parity_with_oracle(wave_mod, oracle_lib):
    shots = make_shots()[:2]
    props, srcs = build(wave_mod, shots, "f32", CONFIGS[:2])
    b = wave_mod.Batch(props, use_graph=True)
    b.run(shots[0].nt, srcs)
    b.sync()
    for p, pr in zip(shots, props):
        ref = oracle_lib.run(p.k64(), p.h, p.nt, s=p.s, src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
        cur, _, _ = pr.fields()
        got = pr.interior(cur).cpu().numpy()
        tr = pr.traces.cpu().numpy()[:, :pr.nrec]
        e_f = np.linalg.norm(got - ref[0]) / np.linalg.norm(ref[0])
        e_t = np.linalg.norm(tr - ref[2]) / np.linalg.norm(ref[2])
        print(f"{p.name}: rel-L2 field {e_f:.3e} traces {e_t:.3e}")
        assert e_f <= 1e-5 and e_t <= 1e-5
    b.close()
    for pr in props:
        pr.close()


@pytest.mark.timeout(900)
def test_batch_workload_shots_against_oracle(wave_mod, oracle_lib, tmp_path, monkeypatch):
    # The 32-shot batch workload (seed 2207, 600 steps) run as the benchmark
    # runs it: schedule and kernels chosen by the tuner, replayed from a HIP
    # graph.  Its two smallest shots are compared with the FP64 oracle's
    # full 600-step runs of the same shots, field and traces.
    from paper_2204_03775_amd import autotune

    monkeypatch.setenv("WAVE_TUNE_CACHE", str(tmp_path / "tune.json"))
    shots = inputs.batch_shots()
    nt = shots[0].nt
    props = []
    for p in shots:
        pr = wave_mod.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                                 sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
        pr.record(nt)
        props.append(pr)
    srcs = [torch.tensor(p.s, dtype=torch.float32, device="cuda") for p in shots]
    stream = torch.cuda.Stream()
    choice = autotune.tune_batch(props, srcs, stream)
    print(f"case: 32-shot batch, tuned schedule {choice['schedule']} on {choice['nstreams']} "
          f"stream(s), {nt} steps", flush=True)
    b = wave_mod.Batch(props, stream=stream, use_graph=True)
    b.set_schedule(choice["schedule"], choice["nstreams"])
    for pr in props:
        pr.reset()
    b.run(nt, srcs)
    b.sync()
    small = sorted(range(len(shots)), key=lambda i: shots[i].points)[:2]
    for i in small:
        p, pr = shots[i], props[i]
        ref = oracle_lib.run(p.k64(), p.h, p.nt, s=p.s, src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
        cur, _, n = pr.fields()
        got = pr.interior(cur).cpu().numpy()
        tr = pr.traces.cpu().numpy()[:, :pr.nrec]
        e_f = np.linalg.norm(got - ref[0]) / np.linalg.norm(ref[0])
        e_t = np.linalg.norm(tr - ref[2]) / np.linalg.norm(ref[2])
        print(f"{p.name}: rel-L2 field {e_f:.3e} traces {e_t:.3e}")
        assert n == nt
        assert e_f <= 1e-5 and e_t <= 1e-5
    b.close()
    for pr in props:
        pr.close()


def test_batch_state_errors(wave_mod):
    shots = make_shots()[:3]
    props, srcs = build(wave_mod, shots, "f32", CONFIGS[:3])
    b = wave_mod.Batch(props, use_graph=False)
    props[1].step(0.0)  # out of step with the others
    with pytest.raises(wave_mod.WaveError) as e:
        b.run(2, srcs)
    assert e.value.code == wave_mod.WAVE_ESTATE
    for pr in props:
        pr.reset()
    props[2].configure("t128x8_r1", 5)  # reconfigured after creation
    with pytest.raises(wave_mod.WaveError) as e:
        b.run(2, srcs)
    assert e.value.code == wave_mod.WAVE_ESTATE
    props[2].configure(*CONFIGS[2])
    with pytest.raises(wave_mod.WaveError) as e:
        b.run(shots[0].nt + 1)  # more rows than the trace buffers hold
    assert e.value.code == wave_mod.WAVE_EINVAL
    b.run(2, srcs)
    b.sync()
    assert all(pr.fields()[2] == 2 for pr in props)
    b.close()
    naive = wave_mod.Propagator(8, 8, 8, (10.0, 10.0, 10.0), np.full((8, 8, 8), 1.0, np.float32))
    naive.configure("naive", 0)
    with pytest.raises(wave_mod.WaveError):
        wave_mod.Batch([naive], use_graph=False)
    naive.close()
    for pr in props:
        pr.close()


def test_autotune_choice_is_applied(wave_mod, tmp_path, monkeypatch):
    from paper_2204_03775_amd import autotune

    monkeypatch.setenv("WAVE_TUNE_CACHE", str(tmp_path / "tune.json"))
    shots = make_shots()
    props, srcs = build(wave_mod, shots, "f32")
    stream = torch.cuda.Stream()
    # per-class choice (schedule 0), served from the cache the second time
    classes = autotune.tune_classes(props, srcs, stream, nsteps=5)
    assert set(classes) == {autotune.size_class(p.nx) for p in shots}
    for p, pr in zip(shots, props):
        name, parts = classes[autotune.size_class(p.nx)]
        v, zc, _ = pr.config()
        assert wave_mod.wave_variant_name(v) == name and zc == -(-p.nz // parts)
    assert autotune.tune_classes(props, srcs, stream) == classes
    # per-shot choice, cached per shape
    one = autotune.tune_single(props[0], srcs[0], stream, nsteps=5)
    assert autotune.tune_single(props[0], srcs[0], stream) == one
    # the whole batch: a schedule, and the shots configured for it
    choice = autotune.tune_batch(props, srcs, stream, nsteps=5)
    assert choice["schedule"] in (0, 1, 3) and choice["nstreams"] >= 1
    if choice["schedule"] == 1:
        for pr, (name, zc) in zip(props, choice["shots"]):
            v, zc_used, _ = pr.config()
            assert wave_mod.wave_variant_name(v) == name and (zc == 0 or zc_used == zc)
    b = wave_mod.Batch(props, stream=stream)
    b.set_schedule(choice["schedule"], choice["nstreams"])
    b.run(shots[0].nt, srcs)
    b.sync()
    b.close()
    for pr in props:
        pr.close()


# 16 streams for 6 shots: streams left without shots are neither forked nor
# captured
@pytest.mark.parametrize("nstreams,graph", [(1, False), (3, False), (3, True), (16, True), (16, False)])
def test_per_shot_schedule_matches_individual_runs(wave_mod, nstreams, graph):
    shots = make_shots()
    ref = alone(wave_mod, shots, "f32")
    props, srcs = build(wave_mod, shots, "f32")
    b = wave_mod.Batch(props, use_graph=graph)
    b.set_schedule(1, nstreams)
    nt = shots[0].nt
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3 if graph else 1):
        print(f"case: schedule 1, {nstreams} streams, graph={graph}, replay {rep}", flush=True)
        for pr in props:
            pr.reset()
        if graph:  # the same run each time: captured once, then replayed
            b.run(nt, srcs)
        else:  # split in an odd and an even part (role bookkeeping)
            b.run(9, srcs)
            b.run(nt - 9, [s[9:] for s in srcs])
        junk.mul_(1.0001)
        b.sync()
        torch.cuda.synchronize()
        for i, pr in enumerate(props):
            assert same(snapshot(pr), ref[i]), (rep, i)
    b.close()
    for pr in props:
        pr.close()


# schedule 3: one cooperative launch per kernel group for the whole run,
# a grid barrier between steps
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_single_launch_schedule_matches_individual_runs(wave_mod, dtype):
    shots = make_shots()
    ref = alone(wave_mod, shots, dtype)
    props, srcs = build(wave_mod, shots, dtype)
    b = wave_mod.Batch(props, use_graph=True)
    b.set_schedule(3)
    nt = shots[0].nt
    junk = torch.randn(1 << 20, device="cuda")
    for rep, split in enumerate((True, False, False)):
        print(f"case: schedule 3, {dtype}, run {rep}, split={split}", flush=True)
        for pr in props:
            pr.reset()
        if split:  # an odd and an even part (role bookkeeping across launches)
            b.run(9, srcs)
            b.run(nt - 9, [s[9:] for s in srcs])
        else:
            b.run(nt, srcs)
        junk.mul_(1.0001)
        b.sync()
        torch.cuda.synchronize()
        for i, pr in enumerate(props):
            assert same(snapshot(pr), ref[i]), (rep, i)
    b.close()
    for pr in props:
        pr.close()


def test_single_launch_schedule_one_group_and_failure_path(wave_mod):
    # every shot with the same kernel: the whole run of all shots is one
    # launch; then the failure hook (every barrier wait gives up at once)
    # stops it early, the kernel exits normally and the run is reported
    # failed; a normal run afterwards is exact again
    shots = make_shots()
    cfgs = [("t128x16_r1", zc) for zc in (0, 16, 7, 0, 24, 56)]
    props, srcs = build(wave_mod, shots, "f32", cfgs)
    ref = []
    for pr, s, p in zip(props, srcs, shots):
        pr.run(p.nt, s)
        pr.sync()
        ref.append(snapshot(pr))
        pr.reset()
    b = wave_mod.Batch(props, use_graph=False)
    assert b.info()[0] == 1
    b.set_schedule(3)
    print("case: schedule 3, one group", flush=True)
    b.run(shots[0].nt, srcs)
    b.sync()
    for i, pr in enumerate(props):
        assert same(snapshot(pr), ref[i]), i
    for pr in props:
        pr.reset()
    b.set_wait_limit(-1)
    print("case: schedule 3, failure path", flush=True)
    b.run(shots[0].nt, srcs)
    with pytest.raises(wave_mod.WaveError) as e:
        b.sync()
    assert e.value.code == wave_mod.WAVE_EHIP
    b.set_wait_limit(1 << 24)
    for pr in props:
        pr.reset()
    print("case: schedule 3, after the failure path", flush=True)
    b.run(shots[0].nt, srcs)
    b.sync()
    for i, pr in enumerate(props):
        assert same(snapshot(pr), ref[i]), i
    b.close()
    for pr in props:
        pr.close()


def test_one_launch_tuner_choice(wave_mod):
    # tune_one_launch leaves every shot with the same kernel from its
    # candidates (so the batch is one launch group), and the single-launch
    # run with that choice is bit for bit the shots run alone with it
    from paper_2204_03775_amd import autotune

    shots = make_shots()
    props, srcs = build(wave_mod, shots, "f32")
    stream = torch.cuda.Stream()
    print("case: tune_one_launch on the six test shots", flush=True)
    name, zc = autotune.tune_one_launch(props, srcs, stream, nsteps=8)
    assert name in autotune.VARIANTS and zc in autotune.ONE_LAUNCH_CHUNKS
    assert {pr.config()[0] for pr in props} == {wave_mod.variants()[name]}
    ref = []
    for pr, s, p in zip(props, srcs, shots):
        pr.reset()
        pr.run(p.nt, s)
        pr.sync()
        ref.append(snapshot(pr))
        pr.reset()
    b = wave_mod.Batch(props, stream=stream, use_graph=False)
    assert b.info()[0] == 1
    b.set_schedule(3)
    print(f"case: schedule 3 with the tuned {name}, z-chunk {zc}", flush=True)
    b.run(shots[0].nt, srcs)
    b.sync()
    for i, pr in enumerate(props):
        assert same(snapshot(pr), ref[i]), i
    b.close()
    for pr in props:
        pr.close()


def test_schedule_switch_and_bad_arguments(wave_mod):
    shots = make_shots()
    ref = alone(wave_mod, shots, "f32")
    props, srcs = build(wave_mod, shots, "f32")
    b = wave_mod.Batch(props, use_graph=True)
    # schedule 2 is switched off and rejected
    for sched, ns in ((1, 0), (1, 17), (4, 1), (-1, 1), (2, 1)):
        with pytest.raises(wave_mod.WaveError) as e:
            wave_mod.wave_batch_set_schedule(b.handle, sched, ns)
        assert e.value.code == wave_mod.WAVE_EINVAL
    nt = shots[0].nt
    # every switch drops the captured graph; each run is checked in full
    for sched, ns in ((1, 2), (0, 1), (3, 1), (1, 4), (3, 1), (1, 4)):
        print(f"case: schedule {sched}, {ns} streams, graph", flush=True)
        b.set_schedule(sched, ns)
        for pr in props:
            pr.reset()
        b.run(nt, srcs)
        b.sync()
        for i, pr in enumerate(props):
            assert same(snapshot(pr), ref[i]), (sched, ns, i)
    b.close()
    for pr in props:
        pr.close()


# schedule 2 (one launch for the whole run, shots pinned to XCDs): short
# z-chunks make a chunk's halo reach 1..4 neighbouring chunks
FLOW_CONFIGS = [("t256x8_r1", 1), ("t64x16_r1", 2), ("t128x8_r1", 3), ("t64x32_r2", 5),
                ("t128x16_r1", 8), ("t256x8_r1", 0)]


@pytest.mark.skip(reason="schedule 2 is switched off: its first GPU run (in the schedule-switch test) "
                  "did not complete within the test time limit, and the cause is not known")
@pytest.mark.parametrize("graph", [False, True])
def test_flow_schedule_matches_individual_runs(wave_mod, graph):
    shots = make_shots()
    ref = []
    props, srcs = build(wave_mod, shots, "f32", FLOW_CONFIGS)
    for pr, s, p in zip(props, srcs, shots):
        pr.run(p.nt, s)
        pr.sync()
        ref.append(snapshot(pr))
        pr.close()
    props, srcs = build(wave_mod, shots, "f32", FLOW_CONFIGS)
    b = wave_mod.Batch(props, use_graph=graph)
    b.set_schedule(2)
    nt = shots[0].nt
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3 if graph else 1):
        print(f"case: schedule 2, graph={graph}, replay {rep}", flush=True)
        for pr in props:
            pr.reset()
        if graph:
            b.run(nt, srcs)
        else:  # an odd and an even part (role bookkeeping across launches)
            b.run(9, srcs)
            b.run(nt - 9, [s[9:] for s in srcs])
        junk.mul_(1.0001)
        b.sync()
        torch.cuda.synchronize()
        for i, pr in enumerate(props):
            assert same(snapshot(pr), ref[i]), (rep, i)
    b.close()
    for pr in props:
        pr.close()


@pytest.mark.skip(reason="schedule 2 is switched off: its first GPU run (in the schedule-switch test) "
                  "did not complete within the test time limit, and the cause is not known")
def test_flow_schedule_larger_shots(wave_mod):
    # many work-groups per XCD and long dependency chains: 9 shots (one XCD
    # holds two), 60 steps
    sizes = [(200, 96, 64), (96, 200, 48), (130, 70, 90), (64, 64, 64), (256, 40, 40),
             (72, 150, 33), (100, 100, 20), (48, 48, 160), (160, 24, 100)]
    shots = [inputs.random_problem(nx, ny, nz, 60, seed=300 + i, sponge_width=6, nrec=11)
             for i, (nx, ny, nz) in enumerate(sizes)]
    cfgs = [("t128x16_r1", 16), ("t256x8_r1", 32), ("t128x16_r1", 0), ("t128x16_r1", 4),
            ("t256x8_r1", 0), ("t128x16_r1", 11), ("t128x16_r1", 6), ("t256x8_r1", 40), ("t128x16_r1", 25)]
    props, srcs = build(wave_mod, shots, "f32", cfgs)
    ref = []
    for pr, s, p in zip(props, srcs, shots):
        pr.run(p.nt, s)
        pr.sync()
        ref.append(snapshot(pr))
        pr.reset()
    b = wave_mod.Batch(props, use_graph=True)
    b.set_schedule(2)
    print("case: schedule 2, 9 larger shots, 60 steps", flush=True)
    b.run(shots[0].nt, srcs)
    b.sync()
    for i, pr in enumerate(props):
        assert same(snapshot(pr), ref[i]), i
    b.close()
    for pr in props:
        pr.close()


@pytest.mark.skip(reason="schedule 2 is switched off: its first GPU run (in the schedule-switch test) "
                  "did not complete within the test time limit, and the cause is not known")
def test_flow_schedule_rejects_16bit_and_reports_a_failed_wait(wave_mod):
    shots = make_shots()
    props, srcs = build(wave_mod, shots, "f16", FLOW_CONFIGS)
    b = wave_mod.Batch(props)
    with pytest.raises(wave_mod.WaveError) as e:
        b.set_schedule(2)
    assert e.value.code == wave_mod.WAVE_EINVAL
    b.close()
    for pr in props:
        pr.close()
    ref = alone(wave_mod, shots, "f32")
    props, srcs = build(wave_mod, shots, "f32")
    b = wave_mod.Batch(props, use_graph=True)
    b.set_schedule(2)
    # every wait after the first step gives up: the launch stops early, the
    # kernel exits normally and the failure is reported
    b.set_wait_limit(-1)
    print("case: schedule 2, failure path", flush=True)
    b.run(shots[0].nt, srcs)
    with pytest.raises(wave_mod.WaveError) as e:
        b.sync()
    assert e.value.code == wave_mod.WAVE_EHIP
    # a normal limit again: the next run is exact
    b.set_wait_limit(1 << 24)
    for pr in props:
        pr.reset()
    print("case: schedule 2, after the failure path", flush=True)
    b.run(shots[0].nt, srcs)
    b.sync()
    for i, pr in enumerate(props):
        assert same(snapshot(pr), ref[i]), i
    b.close()
    for pr in props:
        pr.close()
