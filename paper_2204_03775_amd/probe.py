"""Measured HBM bandwidth of plain streaming kernels (libwave_probe.so).

``python -m paper_2204_03775_amd.probe [elements]`` prints one JSON line with
the copy (1 read + 1 write) and read3-write1 (the propagator's per-update
access mix) bandwidth in GB/s, for arrays of ``elements`` floats each
(default: one 512^3 field in the propagator's padded layout).
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwave_probe.so")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.probe_copy.argtypes = [vp, vp, i64, vp]
    lib.probe_copy.restype = ctypes.c_int
    lib.probe_read3_write1.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.probe_read3_write1.restype = ctypes.c_int
    lib.probe_adjoint_mix.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp]
    lib.probe_adjoint_mix.restype = ctypes.c_int
    return lib


def measure(n: int, repeats: int = 20, with_adjoint_mix: bool = False) -> dict:
    lib = _load()
    n -= n % 4
    bufs = [torch.rand(n, device="cuda") for _ in range(4)]
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream
    ptr = [b.data_ptr() for b in bufs]

    def launched(rc):
        if rc != 0:
            raise RuntimeError(f"probe launch failed (code {rc})")

    def timed(fn, bytes_per_call):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(repeats):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / repeats
        return bytes_per_call / sec / 1e9, sec

    def copy():
        launched(lib.probe_copy(ptr[0], ptr[1], n, s))

    def r3w1():
        launched(lib.probe_read3_write1(ptr[0], ptr[1], ptr[2], ptr[3], n, s))

    copy_gbs, copy_s = timed(copy, 8 * n)
    r3w1_gbs, r3w1_s = timed(r3w1, 16 * n)
    # verify the arithmetic once so the timing is of real work
    ref = bufs[0] + bufs[1] + bufs[2]
    if not (torch.allclose(bufs[3], ref) and torch.equal(bufs[1], bufs[0])):
        raise RuntimeError("probe kernels computed a wrong result")
    out = {"elements": n, "copy_gbs": round(copy_gbs, 1), "copy_us": round(copy_s * 1e6, 2),
           "read3_write1_gbs": round(r3w1_gbs, 1), "read3_write1_us": round(r3w1_s * 1e6, 2)}
    if with_adjoint_mix:
        o = torch.empty(n, device="cuda")
        g = torch.zeros(n, dtype=torch.float64, device="cuda")

        def adjmix():
            launched(lib.probe_adjoint_mix(ptr[0], ptr[1], ptr[2], ptr[3], g.data_ptr(), o.data_ptr(), n, s))

        adj_gbs, adj_s = timed(adjmix, 36 * n)
        ref = ((bufs[0] + bufs[1]) + bufs[2]) + bufs[3]
        if not (torch.equal(o, ref) and torch.allclose(g, (repeats + 1) * ref.double())):
            raise RuntimeError("adjoint-mix probe computed a wrong result")
        out.update(adjoint_mix_gbs=round(adj_gbs, 1), adjoint_mix_us=round(adj_s * 1e6, 2))
        del o, g
    return out


if __name__ == "__main__":
    if len(sys.argv) > 1:
        n = int(sys.argv[1])
    else:
        sys.path.insert(0, os.path.dirname(_HERE))
        from paper_2204_03775_amd import wave

        n = wave.wave_layout(512, 512, 512).elems
    print(json.dumps(measure(n, with_adjoint_mix=True)), flush=True)
