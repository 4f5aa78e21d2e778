#!/usr/bin/env python3
"""Throughput of the FP32 25-point leapfrog propagator on one MI355X.

One benchmark step is one complete shot of the large-shot workload: the
fields are cleared and 1000 time steps of 512^3 are run (source injection,
sponge and 256 receivers fused into every step).  Inputs are resident in
HBM before timing starts.  The JSON line on stdout carries:

  value      interior grid-point updates per second (Gpts/s) over the timed
             shots, wall clock between two device synchronisations;
  roofline   the step kernel against the 8 TB/s HBM peak (and against two
             ceilings measured in the same run: a plain copy, and the step's
             own access pattern streamed without its arithmetic, launches
             alternating their z-direction as the library's do, which lets
             each launch start on planes still in the GPU's memory-side
             cache): 16 algorithmic bytes per update (read u^n, u^{n-1}, k;
             write u^{n+1}) divided by its average launch time from HIP
             events on its stream;
             `traffic` is the HBM byte count per launch measured with
             rocprofv3 counters (profiles/), reported only while the kernel
             source matches the one profiled;
  cpu_baseline  the CPU leg: the FP64 oracle, as it stands, timed on the
             whole 1000-step shot on the host cores (about two minutes on
             16 cores; --cpu-steps bounds it), and on the 64^3 parity shot
             with one thread and with all of them.  The same leg runs the
             oracle's reference results that the accuracy figures of the
             other legs compare with (the oracle runs in no other leg;
             without the CPU leg those figures are absent);
  accuracy   the timed shot's final field and traces against the oracle's
             whole run of the same shot (relative L2);
  forms      the 16-bit storage forms (FP32 arithmetic) on the same shot:
             FP16 and BF16 holding two time levels (8 algorithmic bytes per
             update) or u and its step change (10 bytes): throughput,
             speedup over FP32 and HBM fraction (also against the
             bandwidth of the form's own access pattern streamed without
             arithmetic, with its tiles and z-chunks), and the accuracy of every
             storage type against the FP64 oracle on a 128^3 crop of the
             same model (500 steps) and, with the CPU leg, over the whole
             timed shot (against the oracle's whole run);
  batched    32 uneven shots (96..320 x 96..320 x 96..256, 600 steps each,
             FP32) as one autotuned batch replayed from a HIP graph (the
             tuner picks the schedule: one persistent launch per step, or
             every shot with its own tuned kernel on a few streams): shots/s
             and aggregate Gpts/s, against the same 32 shots run one after
             another with the library's automatic configuration (their
             traces must agree bit for bit).
  launch     the 64^3 x 100-step parity shot (launch-bound): eager launches
             against graph replay of the whole run, and what one step costs
             if the work-groups of a single launch synchronise between steps
             instead (grid barrier, neighbour flags; a probe kernel);
  gradient   the least-squares misfit gradient with respect to k on a 256^3
             layered model with a Gaussian anomaly (800 steps, 128
             receivers): checkpointed forward run (every 50 steps, and with
             every level kept), FP64 misfit, adjoint run with FP64
             accumulation; time against one FP32 forward run of the same
             shot, and, on a 48^3 crop (300 steps), accuracy and speed
             against the FP64 oracle's adjoint.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "large_shot": "512^3 x 1000 steps FP32, dx=10 m, dt=0.8 CFL at 4500 m/s, 5 layers "
                  "1500-4500 m/s x (1+0.05 p) smoothed noise, 20-cell sponge, 12 Hz Ricker "
                  "at z=25, 256 receivers on a line (synthetic, seeded)",
    "small_parity": "64^3 x 100 steps FP32, v=1500 m/s, dt=1 ms, 15 Hz Ricker at the "
                    "centre, 16 random receivers, zero ghost layer (synthetic, seeded)",
    "paper_shape": "755x994x1000 x 1000 steps FP32 (the paper's largest Table 2 shape), "
                   "v=1500 m/s constant, dt=0.8 CFL, no sponge, 15 Hz Ricker at the centre, "
                   "256 receivers (synthetic; context for the paper's cell rates)",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_large_shot.json")
# the sources of the FP32 step kernel (types, device code, instantiation)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2204_03775_amd", "csrc", f)
                  for f in ("wave_dev.h", "wave_step.h", "k_fwd_f32.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_name: str, zchunk: int):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source and launch configuration."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("source_sha256") != source_digest() or t.get("kernel") != kernel_name
            or t.get("zchunk") != zchunk):
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(p, max_steps: int = 0, gpu_final=None, other_finals=None):
    """The FP64 oracle, as it stands, on the host cores: the whole shot (or
    its first max_steps steps), run in segments with a progress line after
    each.  When the whole shot ran and the GPU's final field and traces are
    given, their relative L2 error against it is returned too, and likewise
    for other_finals ({name: (field, traces)}, the 16-bit storage forms)."""
    import oracle

    threads = oracle.default_threads()
    n = p.nt if max_steps <= 0 else min(p.nt, max_steps)

    def progress(done, nt, sec):
        log(f"oracle {p.nx}x{p.ny}x{p.nz}: {done}/{nt} steps, {sec:.0f} s")

    cur, _, tr, sec = oracle.run_segments(p.k64(), p.h, n, 100, s=p.s, src=p.src, rec=p.rec,
                                          sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha,
                                          nthreads=threads, progress=progress)
    what = "the whole" if n == p.nt else f"the first {n} steps of the"
    base = {"value": round(p.points * n / sec / 1e9, 4), "unit": "Gpts/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{what} {p.nt}-step {p.nx}x{p.ny}x{p.nz} shot, FP64, {sec:.1f} s, "
                      f"OpenMP threads={threads} (nproc {os.cpu_count()}), cpu={_cpu_model()}"}
    acc = None
    others = {}
    if n == p.nt:
        def against(final):
            return {"rel_l2_field": rel_l2(final[0], cur), "rel_l2_traces": rel_l2(final[1], tr),
                    "workload": f"the whole {p.nx}x{p.ny}x{p.nz} x {p.nt}-step shot",
                    "reference": "FP64 oracle"}

        if gpu_final is not None:
            acc = against(gpu_final)
        for name, final in (other_finals or {}).items():
            others[name] = against(final)
    return base, acc, others


def cpu_small_shot():
    """The oracle on the 64^3 x 100-step parity shot, on one host thread and
    on all of them (Gpts/s of each, best of three runs)."""
    import oracle
    from paper_2204_03775_amd import inputs

    q = inputs.small_parity()
    k64 = q.k64()
    out = {"workload": "64^3 x 100 steps (the parity shot), FP64"}
    for label, threads in (("one_thread", 1), ("all_cores", oracle.default_threads())):
        best = None
        for _ in range(3):
            t = time.perf_counter()
            oracle.run(k64, q.h, q.nt, s=q.s, src=q.src, rec=q.rec, nthreads=threads)
            sec = time.perf_counter() - t
            best = sec if best is None else min(best, sec)
        out[label] = {"gpts_per_s": round(q.points * q.nt / best / 1e9, 4), "seconds": round(best, 4),
                      "threads": threads}
    return out


# Relative L2 bounds against the FP64 oracle on the 128^3 crop (500 steps):
# FP32 as for the plain path; the 16-bit bounds are those proposed for
# reduced-precision storage (FP16 5e-3, BF16 5e-2).  The two-level forms
# are reported against them as measured, met or not.
ACCURACY_BOUNDS = {"f32": 1e-5, "f16": 5e-3, "bf16": 5e-2, "f16uv": 5e-3, "bf16uv": 5e-2}


def step_stream16(p, kernel: str, zchunk: int, uv: bool):
    """The 16-bit step-stream probe with the form's tiles and z-chunk (None
    for a tiling the probe does not cover or without the probe library)."""
    import re

    m = re.fullmatch(r"t(\d+)x(\d+)_r(\d+)", kernel)
    if not m or int(m.group(1)) != 128:
        return None
    rows, ry = int(m.group(2)), int(m.group(3))
    if rows % ry or (rows // ry, ry) not in ((8, 1), (8, 2), (16, 1), (16, 2), (32, 1)):
        return None
    try:
        from paper_2204_03775_amd import probe
    except ImportError:
        return None
    return probe.measure_step_stream16(p.nx, p.ny, p.nz, zchunk, rows // ry, ry, uv)


def rel_l2(a, b) -> float:
    import numpy as np

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_references(crop_out, grad_out):
    """The other part of the CPU leg: the oracle's results that the GPU
    legs' outputs are compared with.  Returns (accuracy of every storage
    type on the 128^3 crop, accuracy and oracle time of the 48^3 gradient);
    either is None when its GPU leg did not run."""
    import numpy as np

    import oracle
    from paper_2204_03775_amd import inputs

    threads = oracle.default_threads()
    crop_acc = None
    if crop_out:
        p = inputs.crop_shot()
        ref = oracle.run(p.k64(), p.h, p.nt, s=p.s, src=p.src, rec=p.rec, sponge_width=p.sponge_width,
                         sponge_alpha=p.sponge_alpha, nthreads=threads)
        crop_acc = {dt: {"rel_l2_field": rel_l2(f, ref[0]), "rel_l2_traces": rel_l2(tr, ref[2]),
                         "workload": "128^3 crop of the large-shot model, own 20-cell sponge, 500 steps",
                         "reference": "FP64 oracle"}
                    for dt, (f, tr) in crop_out.items()}
    grad_acc = None
    if grad_out:
        cg = inputs.gradient_crop()
        c, co = cg.shot, cg.observed()
        kw = dict(sponge_width=c.sponge_width, sponge_alpha=c.sponge_alpha, nthreads=threads)
        t0 = time.perf_counter()
        _, _, tr = oracle.run(c.k64(), c.h, c.nt, s=c.s, src=c.src, rec=c.rec, **kw)
        t_fwd = time.perf_counter() - t0
        _, _, tr_obs = oracle.run(co.k64(), co.h, co.nt, s=co.s, src=co.src, rec=co.rec, **kw)
        r = tr - tr_obs
        t0 = time.perf_counter()
        ref = oracle.adjoint(c.k64(), c.h, c.nt, r, s=c.s, src=c.src, rec=c.rec, **kw)
        t_orc = time.perf_counter() - t0 + t_fwd
        J_ref = 0.5 * float(np.sum(r * r))
        grad_acc = {"rel_l2_gradient_vs_oracle": rel_l2(grad_out["grad"], ref),
                    "rel_misfit_vs_oracle": abs(grad_out["misfit"] - J_ref) / J_ref,
                    "oracle_s": round(t_orc, 3), "oracle_threads": threads,
                    "speedup_vs_oracle": round(t_orc / grad_out["gpu_s"], 1)}
    return crop_acc, grad_acc


def time_shots(prop, p, s, steps, warmup):
    """Run warmup + steps complete shots; return (wall seconds of the timed
    shots, average step-kernel seconds from HIP events on the stream, and
    the median shot in seconds from the same events)."""
    import torch

    stream = prop.stream
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]

    def shot(i=None):
        prop.reset()
        if i is not None:
            starts[i].record(stream)
        prop.run(p.nt, s)
        if i is not None:
            ends[i].record(stream)

    for _ in range(warmup):
        shot()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        shot(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prop.sync()
    shot_s = sorted(a.elapsed_time(b) / 1e3 for a, b in zip(starts, ends))
    kernel_s = sum(shot_s) / (steps * p.nt)
    return wall, kernel_s, shot_s[len(shot_s) // 2]


def result_ok(prop) -> bool:
    import torch

    field = prop.export(0)
    tr = prop.traces[:, :prop.nrec]
    return bool(torch.isfinite(field).all().item() and torch.isfinite(tr).all().item()
                and tr.abs().max().item() > 0)


def crop_runs():
    """Final field and traces of the 128^3 crop (500 steps) for every
    storage type, on the GPU (compared with the oracle in the CPU leg)."""
    import numpy as np
    import torch

    from paper_2204_03775_amd import inputs, wave

    p = inputs.crop_shot()
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    out = {}
    for dt in ("f32", "f16", "bf16", "f16uv", "bf16uv"):
        prop = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                               sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dt)
        prop.record(p.nt)
        prop.run(p.nt, s)
        f = prop.export(0).cpu().numpy().astype(np.float64)
        prop.sync()
        tr = prop.traces[:, :prop.nrec].cpu().numpy().astype(np.float64)
        prop.close()
        out[dt] = (f, tr)
    return out


def batched_leg(reps: int, single_launch: bool = True):
    import numpy as np
    import torch

    from paper_2204_03775_amd import autotune, inputs, wave

    shots = inputs.batch_shots()
    nt = shots[0].nt
    props = [wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                             sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
             for p in shots]
    for pr in props:
        pr.record(nt)
    srcs = [torch.tensor(p.s, dtype=torch.float32, device="cuda") for p in shots]
    points = sum(p.points for p in shots)

    # sequential: each shot alone, automatic configuration, launched eagerly
    props[0].run(20, srcs[0])
    torch.cuda.synchronize()
    for pr in props:
        pr.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pr, sv in zip(props, srcs):
        pr.run(nt, sv)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    seq_traces = [pr.traces.clone() for pr in props]

    stream = torch.cuda.Stream()
    t = time.perf_counter()
    # the tuner leaves the single-launch schedule out: a cooperative launch
    # costs this process the overlap of its later multi-stream replays, so
    # that schedule is measured below, after the tuned run
    choice = autotune.tune_batch(props, srcs, stream, log=log)
    t_tune = time.perf_counter() - t
    b = wave.Batch(props, stream=stream, use_graph=True)
    b.set_schedule(choice["schedule"], choice["nstreams"])
    groups, wgs, _ = b.info()

    def once():
        for pr in props:
            pr.reset()
        b.run(nt, srcs)

    once()
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        once()
    b.sync()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    equal = all(torch.equal(a, pr.traces) for a, pr in zip(seq_traces, props))
    b.close()

    one = None
    if single_launch:
        one = one_launch_run(props, shots, srcs, stream, choice, nt, reps, points, seq_traces, t_seq)
    for pr in props:
        pr.close()
    gpts = points * nt / t_batch / 1e9
    sched = {0: "one persistent launch per step and kernel group",
             3: "one launch per kernel group for the whole run (grid barrier between steps)"}.get(
        choice["schedule"], f"every shot with its own tuned kernel on {choice['nstreams']} streams")
    log(f"batched ({sched}): 32 shots in {t_batch * 1e3:.1f} ms ({32 / t_batch:.1f} shots/s, "
        f"{gpts:.1f} Gpts/s); sequential {t_seq * 1e3:.1f} ms; speedup {t_seq / t_batch:.2f}x; "
        f"traces equal: {equal}; tuning {t_tune:.1f} s")
    return {"workload": "32 shots (seed 2207), 96..320 x 96..320 x 96..256, 3..6 layers, "
                        "10..20 Hz Ricker, 20-cell sponge, 128 receivers, 600 steps, FP32",
            "shots_per_s": round(32 / t_batch, 3), "value": round(gpts, 3), "unit": "Gpts/s",
            "batched_ms": round(t_batch * 1e3, 2), "sequential_ms": round(t_seq * 1e3, 2),
            "speedup_vs_sequential": round(t_seq / t_batch, 3), "graph": True,
            "schedule": choice["schedule"], "schedule_name": sched, "nstreams": choice["nstreams"],
            "tuning_us_per_step": {k: (round(v, 1) if v is not None else None)
                                   for k, v in choice["us_per_step"].items()},
            "launch_groups": groups if choice["schedule"] in (0, 3) else None,
            "traces_bitwise_equal_to_sequential": bool(equal),
            "one_launch": one,
            "repeats": reps}


def one_launch_run(props, shots, srcs, stream, choice, nt, reps, points, seq_traces, t_seq):
    """The 32 shots in one launch (schedule 3): every shot with the same
    kernel and z-chunk length, the pair timed fastest for that schedule."""
    import torch

    from paper_2204_03775_amd import autotune, wave

    common, zc = autotune.tune_one_launch(props, srcs, stream)
    b1 = wave.Batch(props, stream=stream, use_graph=False)
    b1.set_schedule(3)
    one_groups = b1.info()[0]

    def once1():
        for pr in props:
            pr.reset()
        b1.run(nt, srcs)

    once1()
    b1.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        once1()
    b1.sync()
    torch.cuda.synchronize()
    t_one = (time.perf_counter() - t0) / reps
    equal1 = all(torch.equal(a, pr.traces) for a, pr in zip(seq_traces, props))
    b1.close()
    log(f"batched in one launch ({common}, z-chunk {zc or 'whole depth'}, {one_groups} group): {t_one * 1e3:.1f} ms "
        f"({32 / t_one:.1f} shots/s, {points * nt / t_one / 1e9:.1f} Gpts/s); traces equal: {equal1}")
    return {"schedule": 3, "kernel": common, "zchunk": zc or "whole depth", "launch_groups": one_groups,
            "ms": round(t_one * 1e3, 2), "shots_per_s": round(32 / t_one, 3),
            "gpts_per_s": round(points * nt / t_one / 1e9, 3),
            "speedup_vs_sequential": round(t_seq / t_one, 3),
            "traces_bitwise_equal_to_sequential": bool(equal1)}


def gradient_leg(reps: int):
    import numpy as np
    import torch

    from paper_2204_03775_amd import inputs, wave

    gp = inputs.gradient_shot()
    p, q = gp.shot, gp.observed()

    def make(pp):
        pr = wave.Propagator(pp.nx, pp.ny, pp.nz, pp.h, pp.k32(), src=pp.src, rec=pp.rec,
                             sponge_width=pp.sponge_width, sponge_alpha=pp.sponge_alpha)
        pr.record(pp.nt)
        return pr

    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    obs = make(q)
    obs.run(q.nt, s)
    obs.sync()
    d_obs = obs.traces[:, :obs.nrec].clone()
    obs.close()
    prop = make(p)

    def forward():
        prop.reset()
        prop.run(p.nt, s)

    def forward_all_levels():
        prop.reset()
        prop.forward_checkpointed(p.nt, s, 0)

    def gradient(every):
        prop.reset()
        prop.forward_checkpointed(p.nt, s, every)
        J, res = wave.misfit(prop.traces[:, :prop.nrec].contiguous(), d_obs)
        return J, prop.adjoint(res)

    def timed(fn, *a):
        fn(*a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn(*a)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    t_fwd, _ = timed(forward)
    t_g50, (J50, g50) = timed(gradient, gp.every)
    info50 = prop.grad_info()
    t_all, (Jall, gall) = timed(gradient, 0)
    info_all = prop.grad_info()
    # the adjoint pass alone: every level kept, minus the forward run that stores them
    t_fall, _ = timed(forward_all_levels)
    t_adj = t_all - t_fall
    wave.wave_set_adjoint_fusion(prop.ctx, False)
    t_sep, (_, gsep) = timed(gradient, 0)
    wave.wave_set_adjoint_fusion(prop.ctx, True)
    same_sep = bool(torch.equal(gsep, gall))
    same = bool(torch.equal(g50, gall) and J50.item() == Jall.item())
    gpts = p.points * p.nt / 1e9
    log(f"gradient 256^3 x {p.nt}: forward {t_fwd * 1e3:.1f} ms; gradient every {gp.every}: "
        f"{t_g50 * 1e3:.1f} ms ({t_g50 / t_fwd:.2f}x forward); every level kept ({info_all[1]}): "
        f"{t_all * 1e3:.1f} ms ({t_all / t_fwd:.2f}x); two passes per adjoint step: {t_sep * 1e3:.1f} ms; "
        f"equal: {same} {same_sep}; misfit {J50.item():.6e}; adjoint pass {t_adj * 1e3:.1f} ms = "
        f"{36 * p.points * p.nt / t_adj / 1e9:.0f} GB/s at 36 B/pt")
    finite = bool(torch.isfinite(g50).all().item() and g50.abs().max().item() > 0)
    prop.close()

    # crop: accuracy and speed against the oracle's adjoint
    cg = inputs.gradient_crop()
    c, co = cg.shot, cg.observed()
    cs = torch.tensor(c.s, dtype=torch.float32, device="cuda")
    o2 = wave.Propagator(co.nx, co.ny, co.nz, co.h, co.k32(), src=co.src, rec=co.rec,
                         sponge_width=co.sponge_width, sponge_alpha=co.sponge_alpha)
    o2.record(co.nt)
    o2.run(co.nt, cs)
    cp = wave.Propagator(c.nx, c.ny, c.nz, c.h, c.k32(), src=c.src, rec=c.rec,
                         sponge_width=c.sponge_width, sponge_alpha=c.sponge_alpha)
    cp.record(c.nt)
    d2 = None

    def crop_gradient():
        cp.reset()
        cp.forward_checkpointed(c.nt, cs, cg.every)
        J, res = wave.misfit(cp.traces[:, :cp.nrec].contiguous(), d2)
        return J, cp.adjoint(res)

    o2.sync()
    d2 = o2.traces[:, :o2.nrec].clone()
    t_gpu_crop, (Jc, gc) = timed(crop_gradient)
    gc = gc.cpu().numpy()
    o2.close()
    cp.close()
    log(f"gradient crop 48^3 x {c.nt}: GPU {t_gpu_crop * 1e3:.2f} ms, misfit {Jc.item():.6e}")
    crop_out = {"grad": gc, "misfit": Jc.item(), "gpu_s": t_gpu_crop}
    return {"workload": "256^3 x 800 steps FP32, 5 layers 1500-4500 m/s, +5% Gaussian anomaly "
                        "(sigma 8 cells, seed 2208), data from the model without it, 12 Hz "
                        "Ricker at (25,128,128), 128 receivers at z=22, 20-cell sponge",
            "grid": [p.nx, p.ny, p.nz],
            "forward_ms": round(t_fwd * 1e3, 3),
            "gradient_ms": round(t_g50 * 1e3, 3), "checkpoint_every": info50[1],
            "checkpoint_gb": round(info50[3] / 1e9, 3),
            "gradient_over_forward": round(t_g50 / t_fwd, 3),
            "gradient_ms_all_levels": round(t_all * 1e3, 3),
            "all_levels_gb": round(info_all[3] / 1e9, 3),
            "all_levels_over_forward": round(t_all / t_fwd, 3),
            "gradient_ms_all_levels_two_passes": round(t_sep * 1e3, 3),
            "forward_all_levels_ms": round(t_fall * 1e3, 3),
            "adjoint_pass_ms": round(t_adj * 1e3, 3),
            "adjoint_pass_gbs": round(36 * p.points * p.nt / t_adj / 1e9, 1),
            "gradient_gpts_per_s": round(gpts / t_g50, 3),
            "bitwise_equal_across_checkpointing": same, "bitwise_equal_fused_two_passes": same_sep,
            "finite": finite,
            "misfit": J50.item(),
            "crop": {"workload": "48^3 block around the anomaly, 8-cell sponge, 300 steps, "
                                 "28 receivers, checkpoints every 50",
                     "gpu_ms": round(t_gpu_crop * 1e3, 3)},
            "repeats": reps}, crop_out


def launch_leg(reps: int, single_launch: bool = True):
    """The 64^3 x 100-step parity shot, launch-bound: eager launches
    against graph replay (wave_set_graph), ms per shot."""
    import torch

    from paper_2204_03775_amd import inputs, wave

    p = inputs.small_parity()
    stream = torch.cuda.Stream()
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    prop = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec, stream=stream)
    prop.record(p.nt)

    def timed():
        with torch.cuda.stream(stream):
            prop.reset()
        prop.run(p.nt, s)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            with torch.cuda.stream(stream):
                prop.reset()
            prop.run(p.nt, s)
        stream.synchronize()
        return (time.perf_counter() - t0) / reps

    t_eager = timed()
    prop.use_graph(True)
    t_graph = timed()
    prop.close()
    log(f"launch: 64^3 x {p.nt}: eager {t_eager * 1e3:.3f} ms/shot, graph {t_graph * 1e3:.3f} ms/shot")
    # what a launch per step is weighed against: synchronising the
    # work-groups of one launch between steps instead
    sync = None
    if single_launch:
        from paper_2204_03775_amd import probe

        sync = probe.measure_sync()
        log(f"launch: in-launch step synchronisation {sync}")
    return {"workload": "64^3 x 100 steps FP32 (the parity shot), 16 receivers",
            "eager_ms_per_shot": round(t_eager * 1e3, 4), "graph_ms_per_shot": round(t_graph * 1e3, 4),
            "graph_speedup": round(t_eager / t_graph, 3),
            "graph_us_per_step": round(t_graph / p.nt * 1e6, 3),
            "graph_gpts_per_s": round(p.points * p.nt / t_graph / 1e9, 3),
            "in_launch_sync_us_per_step": sync, "repeats": reps}


# The paper's measurements for its scaling shapes, for context beside the
# MI355X rates.  Table 2: 1000 steps; throughput in Gcell/s on the WSE-2,
# and elapsed seconds on the WSE-2 and on an A100.  Table 3: 755 x 994 x nz,
# 100,000 steps; throughput in Gcell/s and elapsed seconds on the WSE-2.
PAPER_TABLE2 = {(200, 200, 1000): (533.64, 0.0750, 0.7892),
                (400, 400, 1000): (2097.60, 0.0763, 3.5828),
                (600, 600, 1000): (4731.53, 0.0761, 8.0000),
                (755, 500, 1000): (4956.17, 0.0762, 8.5499),
                (755, 600, 1000): (5945.40, 0.0762, 10.1362),
                (755, 900, 1000): (8922.08, 0.0762, 15.5070),
                (755, 990, 1000): (9782.14, 0.0764, 17.4991),
                (755, 994, 1000): (9862.78, 0.0761, 17.4186)}
PAPER_TABLE3 = {(755, 994, 100): (8688.76, 0.8637), (755, 994, 200): (9303.26, 1.6133),
                (755, 994, 300): (9492.89, 2.3716), (755, 994, 400): (9614.15, 3.1223),
                (755, 994, 500): (9786.51, 3.8342), (755, 994, 700): (9885.04, 5.3143),
                (755, 994, 1000): (9936.79, 7.5524)}


def paper_shapes_leg(nt: int):
    """Every grid shape of the paper's two scaling tables, FP32 with the
    library's automatic plan, nt steps after a short warm-up: Gcell/s on
    this GPU beside the paper's WSE-2 rate and the A100 rate its Table 2
    times imply (cells x 1000 steps / seconds)."""
    import numpy as np
    import torch

    from paper_2204_03775_amd import inputs, wave

    rows = []
    for table, shapes in (("Table 2", inputs.PAPER_TABLE2_SHAPES),
                          ("Table 3", inputs.PAPER_TABLE3_SHAPES)):
        for nx, ny, nz in shapes:
            p = inputs.paper_shape(nt, nx, ny, nz)
            kval = float(np.float32((np.float64(1500.0) * p.dt) ** 2))
            stream = torch.cuda.Stream()
            k = torch.full((1, 1, 1), kval, dtype=torch.float32, device="cuda").expand(nz, ny, nx)
            prop = wave.Propagator(nx, ny, nz, p.h, k, src=p.src, rec=p.rec, stream=stream)
            del k
            prop.record(nt)
            s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
            with torch.cuda.stream(stream):
                prop.reset()
            prop.run(20, s)
            with torch.cuda.stream(stream):
                prop.reset()
            stream.synchronize()
            t0 = time.perf_counter()
            prop.run(nt, s)
            stream.synchronize()
            sec = time.perf_counter() - t0
            ok = result_ok(prop)
            variant, zchunk, nwg = prop.config()
            kname = wave.wave_variant_name(variant)
            prop.close()
            del prop, s
            torch.cuda.empty_cache()
            gcell = p.points * nt / sec / 1e9
            row = {"table": table, "nx": nx, "ny": ny, "nz": nz, "mi355x_gcell_per_s": round(gcell, 1),
                   "kernel": kname, "zchunk": zchunk, "workgroups": nwg, "finite": ok}
            if table == "Table 2":
                wse, t_wse, t_a100 = PAPER_TABLE2[(nx, ny, nz)]
                row.update(wse2_gcell_per_s=wse,
                           a100_gcell_per_s=round(p.points * 1000 / t_a100 / 1e9, 1),
                           vs_a100=round(gcell * t_a100 / (p.points * 1000 / 1e9), 2))
            else:
                wse, t_wse = PAPER_TABLE3[(nx, ny, nz)]
                row.update(wse2_gcell_per_s=wse)
            row["vs_wse2"] = round(gcell / wse, 4)
            log(f"paper shape {table} {nx}x{ny}x{nz}: {gcell:.1f} Gcell/s ({kname}, z-chunk {zchunk}, "
                f"{nwg} work-groups); WSE-2 {wse} Gcell/s" +
                (f", A100 {row['a100_gcell_per_s']}" if table == "Table 2" else ""))
            rows.append(row)
    return {"workload": f"the paper's Table 2 and Table 3 grid shapes, {nt} steps each, FP32, "
                        "v=1500 m/s constant, no sponge, automatic launch plan",
            "steps": nt, "rows": rows}


def _git_sha():
    """HEAD of the source tree when it is a git checkout, else None."""
    import subprocess

    try:
        r = subprocess.run(["git", "-C", ROOT, "rev-parse", "HEAD"], capture_output=True, text=True,
                           timeout=10)
        return r.stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed shots")
    ap.add_argument("--warmup", type=int, default=1, help="untimed shots before timing")
    ap.add_argument("--workload", default="large_shot", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="auto", help="kernel variant name (auto = library choice)")
    ap.add_argument("--zchunk", type=int, default=0, help="z planes per work-group (0 = auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16/BF16 storage forms")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-shot batched run")
    ap.add_argument("--no-single-launch", action="store_true",
                    help="leave cooperative launches out (the single-launch batch schedule and the "
                         "in-launch synchronisation probe): rocprofv3 does not survive them")
    ap.add_argument("--no-gradient", action="store_true", help="skip the adjoint gradient leg")
    ap.add_argument("--no-launch", action="store_true", help="skip the 64^3 graph-replay leg")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the sweep over the paper's Table 2 and Table 3 grid shapes")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU leg (0 = the whole shot, which also gives the "
                         "GPU result's accuracy over it)")
    args = ap.parse_args()

    if args.gpus != 1:
        log(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the propagator "
            "is single-GPU; how it would shard across GPUs is a design note only).")
        return 2

    if not os.path.exists(os.path.join(ROOT, "paper_2204_03775_amd", "libwave.so")):
        import __graft_entry__

        __graft_entry__.build()  # nothing built yet
    import numpy as np
    import torch

    from paper_2204_03775_amd import inputs, metrics, wave

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)

    t = time.perf_counter()
    p = getattr(inputs, args.workload)()
    log(f"workload {args.workload}: {p.nx}x{p.ny}x{p.nz} x {p.nt} steps "
        f"(generated in {time.perf_counter() - t:.1f} s)")

    prop = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                           sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha)
    prop.configure(args.variant, args.zchunk)
    variant, zchunk, nwg = prop.config()
    kname = wave.wave_variant_name(variant)
    log(f"kernel {kname}, z-chunk {zchunk}, {nwg} work-groups per step")
    prop.record(p.nt)
    s = torch.tensor(p.s, dtype=torch.float32, device="cuda")
    wall, kernel_s, shot_median = time_shots(prop, p, s, args.steps, args.warmup)
    if not result_ok(prop):
        log("error: non-finite or empty result")
        return 1
    # the last timed shot's output, compared with the oracle in the CPU leg
    gpu_final = None
    if not args.no_cpu_baseline:
        gpu_final = (prop.export(0).cpu().numpy(), prop.traces[:, :prop.nrec].cpu().numpy())

    gpts = metrics.gpts_per_s(p.nx, p.ny, p.nz, p.nt * args.steps, wall)
    launch_bytes = metrics.BYTES_PER_POINT_F32 * p.points
    achieved = launch_bytes / kernel_s / 1e9
    traffic = measured_traffic(kname, zchunk) if args.workload == "large_shot" else None
    copy_gbs = None
    step_stream = None
    probe_res = {}
    try:
        from paper_2204_03775_amd import probe

        probe_res = probe.measure(wave.wave_layout(512, 512, 512).elems, repeats=10,
                                  with_adjoint_mix=not args.no_gradient)
        copy_gbs = probe_res["copy_gbs"]
        if args.workload == "large_shot":
            step_stream = probe.measure_step_stream(p.nx, p.ny, p.nz, zchunk)
    except ImportError:
        pass
    log(f"{gpts:.1f} Gpts/s wall, kernel {kernel_s * 1e6:.1f} us/launch = {achieved:.0f} GB/s "
        f"({achieved / metrics.MI355X_HBM_PEAK_GBS:.3f} of peak), paper-convention "
        f"{metrics.paper_tflops(gpts):.1f} TFLOP/s")

    forms = None
    form_finals = {}
    crop_out = grad_crop_out = None
    if not args.no_forms and args.workload == "large_shot":
        prop.close()
        forms = {}
        for dt in ("f16", "bf16", "f16uv", "bf16uv"):
            bpp = metrics.BYTES_PER_POINT_16UV if dt.endswith("uv") else metrics.BYTES_PER_POINT_16
            pr = wave.Propagator(p.nx, p.ny, p.nz, p.h, p.k32(), src=p.src, rec=p.rec,
                                 sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha, dtype=dt)
            pr.configure(args.variant, args.zchunk)
            v16, zc16, _ = pr.config()
            pr.record(p.nt)
            w16, k16, _ = time_shots(pr, p, s, args.steps, args.warmup)
            if not result_ok(pr):
                log(f"error: non-finite or empty {dt} result")
                return 1
            if not args.no_cpu_baseline and not args.cpu_steps:
                # the last timed shot's output, for the whole-shot comparison in the CPU leg
                form_finals[dt] = (pr.export(0).cpu().numpy(), pr.traces[:, :pr.nrec].cpu().numpy())
            pr.close()
            g16 = metrics.gpts_per_s(p.nx, p.ny, p.nz, p.nt * args.steps, w16)
            a16 = bpp * p.points / k16 / 1e9
            kname16 = wave.wave_variant_name(v16)
            stream16 = step_stream16(p, kname16, zc16, dt.endswith("uv"))
            forms[dt] = {"value": round(g16, 3), "unit": "Gpts/s", "speedup_vs_f32": round(g16 / gpts, 3),
                         "kernel": kname16, "zchunk": zc16,
                         "roofline": {"bound": "hbm", "achieved": round(a16, 1),
                                      "peak": metrics.MI355X_HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": round(a16 / metrics.MI355X_HBM_PEAK_GBS, 4),
                                      "bytes_per_point": bpp,
                                      "step_stream_measured": stream16,
                                      "frac_of_step_stream": (round(a16 / stream16["alternating_gbs"], 4)
                                                              if stream16 else None)}}
            log(f"{dt}: {g16:.1f} Gpts/s ({g16 / gpts:.2f}x FP32), kernel {k16 * 1e6:.1f} us = "
                f"{a16:.0f} GB/s at {bpp} B/pt"
                + (f"; its access pattern alone streams {stream16['alternating_gbs']:.0f} GB/s"
                   if stream16 else ""))
        crop_out = crop_runs()

    batched = None
    if not args.no_batched and args.workload == "large_shot":
        prop.close()
        batched = batched_leg(max(1, args.steps // 2), single_launch=not args.no_single_launch)
        one = batched["one_launch"]
        if not (batched["traces_bitwise_equal_to_sequential"]
                and (one is None or one["traces_bitwise_equal_to_sequential"])):
            log("error: batched traces differ from the sequential runs")
            return 1

    launch = None
    if not args.no_launch and args.workload == "large_shot":
        launch = launch_leg(20, single_launch=not args.no_single_launch)

    paper_shapes = None
    if not args.no_paper_shapes and args.workload == "large_shot":
        prop.close()
        paper_shapes = paper_shapes_leg(300)
        if not all(r["finite"] for r in paper_shapes["rows"]):
            log("error: a paper-shape run produced non-finite or empty output")
            return 1

    gradient = None
    if not args.no_gradient and args.workload == "large_shot":
        prop.close()
        gradient, grad_crop_out = gradient_leg(max(2, args.steps))
        mix = probe_res.get("adjoint_mix_gbs")
        gradient["adjoint_mix_ceiling_gbs"] = mix  # a plain streaming kernel with the same access mix
        gradient["adjoint_pass_frac_of_mix_ceiling"] = round(gradient["adjoint_pass_gbs"] / mix, 3) if mix else None
        # the fused adjoint step's own access pattern without arithmetic, with
        # the tiling the adjoint picks on this grid (128 x 16 tiles, 32-plane
        # chunks: 256 work-groups)
        adj_stream = None
        try:
            from paper_2204_03775_amd import probe

            gx, gy, gz = gradient["grid"]
            adj_stream = probe.measure_adjoint_stream(gx, gy, gz, 32, 16)
        except ImportError:
            pass
        gradient["adjoint_stream_measured"] = adj_stream
        gradient["adjoint_pass_frac_of_adjoint_stream"] = (
            round(gradient["adjoint_pass_gbs"] / adj_stream["alternating_gbs"], 3) if adj_stream else None)
        if adj_stream:
            log(f"adjoint step's access pattern alone: {adj_stream['alternating_gbs']:.0f} GB/s alternating; "
                f"adjoint pass {gradient['adjoint_pass_frac_of_adjoint_stream']:.3f} of it")
        if not (gradient["finite"] and gradient["bitwise_equal_across_checkpointing"]
                and gradient["bitwise_equal_fused_two_passes"]):
            log("error: gradient not finite or dependent on the checkpoint interval")
            return 1

    # the CPU leg: the oracle timed on the host cores, and its references
    # for the accuracy reports of the other legs
    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        cpu, accuracy, form_acc = cpu_baseline(p, args.cpu_steps, gpu_final, form_finals)
        del gpu_final
        form_finals.clear()
        for dt, a in form_acc.items():
            bound = ACCURACY_BOUNDS[dt]
            a["bound"] = bound
            a["meets_bound"] = bool(a["rel_l2_field"] <= bound and a["rel_l2_traces"] <= bound)
            forms[dt]["accuracy_large_shot"] = a
            log(f"{dt} accuracy over the whole shot: field {a['rel_l2_field']:.3e} traces "
                f"{a['rel_l2_traces']:.3e} (bound {bound:g}: {'met' if a['meets_bound'] else 'NOT met'})")
        log(f"oracle: {cpu['value']} Gpts/s ({cpu['sample']})")
        if accuracy:
            log(f"FP32 accuracy over the whole shot: field {accuracy['rel_l2_field']:.3e} "
                f"traces {accuracy['rel_l2_traces']:.3e}")
        cpu["small_shot"] = cpu_small_shot()
        log(f"oracle 64^3 x 100: {cpu['small_shot']['one_thread']['gpts_per_s']} Gpts/s on one thread, "
            f"{cpu['small_shot']['all_cores']['gpts_per_s']} on {cpu['small_shot']['all_cores']['threads']}")
        crop_acc, grad_acc = oracle_references(crop_out, grad_crop_out)
        for dt, a in (crop_acc or {}).items():
            bound = ACCURACY_BOUNDS[dt]
            a["bound"] = bound
            a["meets_bound"] = bool(a["rel_l2_field"] <= bound and a["rel_l2_traces"] <= bound)
            if dt == "f32":
                forms["f32_accuracy"] = a
            else:
                forms[dt]["accuracy"] = a
                forms[dt]["meets_accuracy_bound"] = a["meets_bound"]
            log(f"{dt} accuracy on the crop: field {a['rel_l2_field']:.3e} traces {a['rel_l2_traces']:.3e} "
                f"(bound {bound:g}: {'met' if a['meets_bound'] else 'NOT met'})")
        if forms is not None and accuracy:
            forms["f32_accuracy_large_shot"] = accuracy
        if grad_acc:
            gradient["crop"].update(grad_acc)
            log(f"gradient crop: rel-L2 vs oracle {grad_acc['rel_l2_gradient_vs_oracle']:.3e}, misfit rel "
                f"{grad_acc['rel_misfit_vs_oracle']:.2e}; oracle {grad_acc['oracle_s']:.2f} s")

    rec = {
        "metric": "Gpts/s stencil updates + % HBM roofline (FP32 vs FP16-store); shots/s",
        "value": round(gpts, 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "step": f"one benchmark step = one complete shot of {p.nt} time steps "
                           f"(ms_per_step is milliseconds per shot)",
                   "nx": p.nx, "ny": p.ny, "nz": p.nz, "time_steps": p.nt,
                   "kernel": kname, "zchunk": zchunk, "workgroups": nwg,
                   "shots_per_s": round(args.steps / wall, 4),
                   "median_shot_ms": round(shot_median * 1e3, 3),
                   "gpts_per_s_median_shot": round(p.points * p.nt / shot_median / 1e9, 3),
                   "paper_tflops_51flop": round(metrics.paper_tflops(gpts), 2),
                   "parallelism": "single GPU",
                   "step_kernel_source_sha256": source_digest(),
                   "git": _git_sha()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": metrics.MI355X_HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / metrics.MI355X_HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "copy_gbs_measured": copy_gbs,
                     "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
                     "step_stream_measured": step_stream,
                     "frac_of_step_stream": (round(achieved / step_stream["alternating_gbs"], 4)
                                             if step_stream else None)},
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "forms": forms,
        "batched": batched,
        "gradient": gradient,
        "launch": launch,
        "paper_shapes": paper_shapes,
    }
    prop.close()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
