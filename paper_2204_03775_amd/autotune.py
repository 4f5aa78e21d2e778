"""Tile and z-chunk selection per size class, measured on the GPU.

Shots are grouped into size classes by the x extent of their grid (the
axis tiles are widest along, so it decides how many lanes of the last tile
idle).  For a batch, every class gets a kernel variant and a z-chunk
fraction; candidates are timed on the batch itself, one class at a time
(coordinate descent from a common start), because a configuration that is
best for a shot running alone (many z-chunks to fill the GPU) is not best
when 32 shots share the GPU (chunks re-read 8 planes each).

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


def time_batch(props, srcs, nsteps: int, stream) -> float:
    """Seconds per step of one batched run (eager launches, after a short
    warm-up); fields are reset before and after."""
    b = wave.Batch(props, stream=stream, use_graph=False)
    try:
        for p in props:
            p.reset()
        b.run(3, srcs)
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


def tune_batch(props, srcs, stream, nsteps: int = 30, use_cache: bool = True, log=None) -> dict:
    """Choose (variant, chunks) per size class for this batch; returns
    {class: (variant, chunks)} and configures the Propagators with it."""
    classes = sorted({size_class(p.nx) for p in props},
                     key=lambda c: -sum(p.points for p in props if size_class(p.nx) == c))
    dtype = props[0].dtype
    cache = load_cache() if use_cache else {}
    choice = {c: tuple(cache[_key(dtype, c)]) for c in classes if _key(dtype, c) in cache}
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
