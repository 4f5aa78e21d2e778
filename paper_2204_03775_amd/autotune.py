"""Tile, z-chunk and schedule selection, measured on the GPU.

Single shots: every (variant, z-chunk) candidate is timed on the shot's
own grid (``tune_single``).

Batches (``tune_batch``) can run in three ways.  Schedule 0 puts all shots
into one persistent launch per step and kernel group, and schedule 3 runs
the same work in one launch per group for the whole run (a grid barrier
between steps); there shots are grouped into size classes by the x extent
of their grid (the axis tiles are widest along, so it decides how many
lanes of the last tile idle), and every class gets a kernel variant and a
z-chunk fraction, timed on the batch itself one class at a time
(coordinate descent from a common start), because a configuration that is
best for a shot alone is not best when all shots share each launch.
Schedule 1 launches every shot with its own tuned configuration, spread
over a few streams and replayed from one graph per stream.  The fastest is
kept (schedule 3 only on request: see ``tune_batch``).  ``tune_one_launch``
picks the common kernel and z-chunk for running a whole batch as a single
cooperative launch.

Results are cached in a JSON file keyed by (GPU architecture, storage type,
class); ``WAVE_TUNE_CACHE`` overrides its location.
"""
from __future__ import annotations

import json
import os

import torch

from . import wave

VARIANTS = ("t256x8_r1", "t128x16_r1", "t128x8_r1", "t64x16_r1", "t64x32_r1")
CHUNK_FRACTIONS = (1, 2, 4, 8)  # z split into this many chunks
DEFAULT = ("t256x8_r1", 1)


def cache_path() -> str:
    return os.environ.get("WAVE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "wave25", "tune.json"))


def arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover
        return "unknown"


def size_class(nx: int) -> str:
    """x-extent bucket: 1..127, 128..191, 192..255, 256..383, 384.."""
    for hi, name in ((128, "x<128"), (192, "x<192"), (256, "x<256"), (384, "x<384")):
        if nx < hi:
            return name
    return "x>=384"


def _key(dtype: int, cls: str) -> str:
    return f"{arch()}|{dtype}|{cls}"


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    with open(p + ".tmp", "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(p + ".tmp", p)


def apply(props, choice: dict) -> None:
    """Configure every Propagator from {class: (variant name, chunks)}."""
    for p in props:
        name, parts = choice.get(size_class(p.nx), DEFAULT)
        zc = -(-p.nz // int(parts))
        p.configure(name, zc)


def steps_available(prop, src) -> int:
    """Steps a timing run may take from a reset: bounded by the source
    values given (the library reads one per step and trusts the caller for
    the length) and by the trace rows recorded."""
    n = 1 << 30
    if src is not None:
        n = min(n, int(src.numel()))
    if getattr(prop, "traces", None) is not None and prop.nrec > 0:
        n = min(n, int(prop.traces.shape[0]))
    return n


def _timed_steps(props, srcs, wanted: int, before: int = 0) -> int:
    """wanted, capped so that before + steps fit every shot; ValueError when
    the shots are too short to time at all."""
    avail = min(steps_available(p, s) for p, s in zip(props, srcs)) - before
    if avail < 4:
        raise ValueError(f"too few source values or trace rows to time: {avail + before} steps "
                         f"available, at least {before + 4} needed")
    return min(wanted, avail)


def time_batch(props, srcs, nsteps: int, stream, schedule: int = 0, nstreams: int = 1) -> float:
    """Seconds per step of one batched run, after a short warm-up; fields
    are reset before and after.  Schedule 0 launches eagerly (one launch per
    step and group); schedule 1 is captured once and the replay is timed;
    schedule 3 is one launch per group for the whole run."""
    nsteps = _timed_steps(props, srcs, nsteps)
    b = wave.Batch(props, stream=stream, use_graph=(schedule == 1))
    try:
        if schedule:
            b.set_schedule(schedule, nstreams)
        for p in props:
            p.reset()
        b.run(3 if not schedule else nsteps, srcs)
        b.sync()
        for p in props:
            p.reset()
        with torch.cuda.stream(stream):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.run(nsteps, srcs)
            e1.record(stream)
        b.sync()
        return e0.elapsed_time(e1) / 1e3 / nsteps
    finally:
        b.close()
        for p in props:
            p.reset()


SINGLE_CHUNKS = (0, 8, 16, 32, 64)  # z-chunk (0: the library's automatic choice)
STREAM_COUNTS = (1, 2, 4)


def _single_key(p) -> str:
    return f"{arch()}|{p.dtype}|shot|{p.nx}x{p.ny}x{p.nz}"


def tune_single(prop, src, stream, nsteps: int = 20, use_cache: bool = True, log=None):
    """The fastest (variant, z-chunk) for one Propagator alone, measured on
    its own grid (cached per GPU architecture, storage type and shape);
    leaves it configured with that choice and returns it."""
    cache = load_cache() if use_cache else {}
    key = _single_key(prop)
    if key in cache and cache[key][0] in wave.variants():  # a stale entry is re-tuned
        name, zc = cache[key]
        prop.configure(name, zc)
        return name, zc
    nsteps = _timed_steps([prop], [src], nsteps, before=3)
    best = None
    for name in VARIANTS:
        for zc in SINGLE_CHUNKS:
            if zc > prop.nz:
                continue
            prop.configure(name, zc)
            prop.reset()
            prop.run(3, src)
            ps = prop.stream  # the Propagator's own stream
            with torch.cuda.stream(ps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(ps)
                prop.run(nsteps, src[3:] if src is not None else None)
                e1.record(ps)
            ps.synchronize()
            t = e0.elapsed_time(e1) / nsteps
            if best is None or t < best[0]:
                best = (t, name, zc)
    prop.reset()
    _, name, zc = best
    if log:
        log(f"tune {prop.nx}x{prop.ny}x{prop.nz}: {name} zc {zc}: {best[0] * 1e3:.1f} us/step")
    prop.configure(name, zc)
    if use_cache:
        cache = load_cache()
        cache[key] = [name, zc]
        save_cache(cache)
    return name, zc


def tune_batch(props, srcs, stream, nsteps: int = 30, use_cache: bool = True, log=None,
               single_launch: bool = False) -> dict:
    """Choose how to run this batch: schedule 0 (one persistent launch per
    step and group) or schedule 3 (one launch per group for the whole run)
    with a (variant, chunks) per size class, or schedule 1 (every shot with
    its own tuned configuration on 1, 2 or 4 streams), whichever is fastest.  Configures the Propagators and returns
    {"schedule", "nstreams", "classes" or "shots", "us_per_step"}; create
    the Batch afterwards and call its set_schedule(schedule, nstreams).
    Schedule 3 (a cooperative launch) is timed only with
    ``single_launch=True``: once a process has made a cooperative launch,
    its later multi-stream graph replays (schedule 1) lose their overlap
    (measured: the 32-shot batch on 4 streams 442.6 -> 567.9 ms)."""
    classes = tune_classes(props, srcs, stream, nsteps, use_cache, log)
    t_queue = time_batch(props, srcs, nsteps, stream)
    t_run = time_batch(props, srcs, nsteps, stream, schedule=3) if single_launch else float("inf")
    shots = [tune_single(p, s, stream, use_cache=use_cache, log=log) for p, s in zip(props, srcs)]
    t_streams = {k: time_batch(props, srcs, nsteps, stream, schedule=1, nstreams=k) for k in STREAM_COUNTS}
    k_best = min(t_streams, key=t_streams.get)
    if log:
        log(f"tune batch: schedule 0 {t_queue * 1e6:.1f} us/step; schedule 3 {t_run * 1e6:.1f}; schedule 1 "
            + ", ".join(f"{k} streams {t * 1e6:.1f}" for k, t in t_streams.items()) + " us/step")
    times = {"schedule0": t_queue * 1e6, "schedule3": t_run * 1e6 if single_launch else None,
             **{f"schedule1_streams{k}": t * 1e6 for k, t in t_streams.items()}}
    if t_streams[k_best] < min(t_queue, t_run):
        return {"schedule": 1, "nstreams": k_best, "shots": [list(x) for x in shots],
                "us_per_step": times}
    apply(props, classes)
    return {"schedule": 3 if t_run < t_queue else 0, "nstreams": 1,
            "classes": {k: list(v) for k, v in classes.items()}, "us_per_step": times}


ONE_LAUNCH_CHUNKS = (32, 64, 0)  # z-chunk planes (0: the whole grid depth)


def tune_one_launch(props, srcs, stream, nsteps: int = 30, log=None) -> tuple:
    """The fastest common (variant, z-chunk planes) for running the whole
    batch as one cooperative launch (schedule 3: every shot must use the
    same kernel to share the launch), timed with schedule 3 itself; leaves
    the Propagators configured with it.  Call it after any multi-stream
    replays the process still wants to time: see tune_batch."""
    best = None
    for name in VARIANTS:
        for zc in ONE_LAUNCH_CHUNKS:
            for p in props:
                p.configure(name, zc if zc else p.nz)
            t = time_batch(props, srcs, nsteps, stream, schedule=3)
            if log:
                log(f"tune one launch: {name} zc {zc or 'nz'}: {t * 1e6:.1f} us/step")
            if best is None or t < best[0]:
                best = (t, name, zc)
    _, name, zc = best
    for p in props:
        p.configure(name, zc if zc else p.nz)
    return name, zc


def tune_classes(props, srcs, stream, nsteps: int = 30, use_cache: bool = True, log=None) -> dict:
    """Choose (variant, chunks) per size class for schedule 0; returns
    {class: (variant, chunks)} and configures the Propagators with it."""
    classes = sorted({size_class(p.nx) for p in props},
                     key=lambda c: -sum(p.points for p in props if size_class(p.nx) == c))
    dtype = props[0].dtype
    cache = load_cache() if use_cache else {}
    known = set(wave.variants())
    choice = {c: tuple(cache[_key(dtype, c)]) for c in classes
              if _key(dtype, c) in cache and cache[_key(dtype, c)][0] in known}
    todo = [c for c in classes if c not in choice]
    for c in todo:
        choice[c] = DEFAULT
    if todo:
        apply(props, choice)
        best = time_batch(props, srcs, nsteps, stream)
        for c in todo:
            for name in VARIANTS:
                for parts in CHUNK_FRACTIONS:
                    cand = dict(choice)
                    cand[c] = (name, parts)
                    if cand[c] == choice[c]:
                        continue
                    apply(props, cand)
                    t = time_batch(props, srcs, nsteps, stream)
                    if log:
                        log(f"tune {c}: {name} /{parts}: {t * 1e6:.1f} us/step")
                    if t < best:
                        best, choice = t, cand
            cache[_key(dtype, c)] = list(choice[c])
        if use_cache:
            save_cache(cache)
    apply(props, choice)
    return choice
