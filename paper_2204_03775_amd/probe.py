"""Measured HBM bandwidth of plain streaming kernels (libwave_probe.so).

``python -m paper_2204_03775_amd.probe [elements]`` prints one JSON line with
the copy (1 read + 1 write) and read3-write1 (the propagator's per-update
access mix) bandwidth in GB/s, for arrays of ``elements`` floats each
(default: one 512^3 field in the propagator's padded layout);
``python -m paper_2204_03775_amd.probe step-stream NX NY NZ ZC`` the step's
access pattern on that grid and z-chunk (``measure_step_stream``).
``measure_sync`` gives the cost of synchronising work-groups inside one
launch, against that of a launch; ``measure_step_stream`` the bandwidth of
the step's own access pattern (tiles, z-chunks, in-place write) without its
arithmetic, with every launch marching up and with alternating directions,
``measure_step_stream16`` the same for the 16-bit storage forms and
``measure_adjoint_stream`` for the fused adjoint step.
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
    ci = ctypes.c_int
    lib.probe_sync.argtypes = [vp, ci, ci, ci, ctypes.c_double, vp]
    lib.probe_sync.restype = ci
    lib.probe_empty.argtypes = [ci, vp]
    lib.probe_empty.restype = ci
    lib.probe_step_stream.argtypes = [vp, vp, vp, ci, ci, ci, i64, i64, ci, ci, vp]
    lib.probe_step_stream.restype = ci
    lib.probe_step_stream16.argtypes = [vp, vp, vp, vp, ci, ci, ci, i64, i64, ci, ci, ci, ci, vp]
    lib.probe_step_stream16.restype = ci
    lib.probe_adjoint_stream.argtypes = [vp, vp, vp, vp, vp, ci, ci, ci, i64, i64, ci, ci, ci, vp]
    lib.probe_adjoint_stream.restype = ci
    return lib


def measure_step_stream(nx: int = 512, ny: int = 512, nz: int = 512, zc: int = 256, launches: int = 20) -> dict:
    """GB/s (16 bytes per interior cell) of the step's access pattern without
    its arithmetic: a sequence of launches that swap the two wave fields, as
    the propagator's run does, all marching z upwards, and alternating
    direction launch by launch (what the library's tiled launches do).  Three
    fields in the library's FP32 padded layout, 256 x 8 tiles, z-chunks of
    zc planes."""
    lib = _load()
    x0 = 32
    pitch = -(-(x0 + nx + 4) // 32) * 32
    elems = pitch * (ny + 8) * (nz + 8)
    f = [torch.rand(elems, device="cuda") for _ in range(3)]
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream

    def launch(a, b, down):
        rc = lib.probe_step_stream(a.data_ptr(), b.data_ptr(), f[2].data_ptr(), nx, ny, nz, pitch, x0, zc,
                                   int(down), s)
        if rc != 0:
            raise RuntimeError(f"probe_step_stream failed (code {rc})")

    # one launch checked against its definition: b = a (four planes on) + b + k
    view = lambda t: t.view(nz + 8, ny + 8, pitch)[:, 4:4 + ny, x0:x0 + nx]
    b0 = view(f[1]).clone()
    launch(f[0], f[1], False)
    torch.cuda.synchronize()
    ref = view(f[0])[8:8 + nz] + b0[4:4 + nz] + view(f[2])[4:4 + nz]
    if not torch.equal(view(f[1])[4:4 + nz], ref):
        raise RuntimeError("step-stream probe computed a wrong result")
    del b0, ref
    out = {"nx": nx, "ny": ny, "nz": nz, "zchunk": zc, "launches": launches}
    for name, alternate in (("ascending", False), ("alternating", True)):
        def seq(count):
            a, b = f[0], f[1]
            for i in range(count):
                launch(a, b, alternate and (i & 1))
                a, b = b, a
        seq(4)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        seq(launches)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / launches
        out[f"{name}_gbs"] = round(16.0 * nx * ny * nz / sec / 1e9, 1)
        out[f"{name}_us"] = round(sec * 1e6, 2)
    del f
    return out


def measure_step_stream16(nx: int, ny: int, nz: int, zc: int, ty: int, ry: int, uv: bool,
                          launches: int = 20) -> dict:
    """The same for a 16-bit storage form: GB/s at 8 bytes per interior
    cell (two levels) or 10 (u and step change), of launches that swap the
    level buffers, all marching up and alternating direction.  Tiles of 128
    cells x ty * ry rows (32 x ty threads), z-chunks of zc planes, as the
    form's step kernel tiles the grid."""
    lib = _load()
    x0 = 64  # 128-byte aligned interior rows
    pitch = -(-(x0 + nx + 4) // 64) * 64
    elems = pitch * (ny + 8) * (nz + 8)
    nf = 4 if uv else 3
    f = [torch.randint(-32768, 32767, (elems,), dtype=torch.int16, device="cuda") for _ in range(nf)]
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream

    def launch(u, p, o, down):
        rc = lib.probe_step_stream16(u.data_ptr(), p.data_ptr(), o.data_ptr() if o is not None else None,
                                     f[2].data_ptr(), nx, ny, nz, pitch, x0, zc, ty, ry, int(down), s)
        if rc != 0:
            raise RuntimeError(f"probe_step_stream16 failed (code {rc})")

    # one launch checked against its definition, every cell of the written fields
    view = lambda t: t.view(nz + 8, ny + 8, pitch)
    inner = lambda t, dz=0: view(t)[4 + dz:4 + dz + nz, 4:4 + ny, x0:x0 + nx]
    ahead = inner(f[0], 4)
    if uv:
        want_o, want_d = f[3].clone(), f[1].clone()
        inner(want_o).copy_(ahead ^ inner(f[2]))
        inner(want_d).copy_(inner(f[1]) ^ ahead)
        launch(f[0], f[1], f[3], False)
        torch.cuda.synchronize()
        ok = torch.equal(f[3], want_o) and torch.equal(f[1], want_d)
        del want_o, want_d
    else:
        want = f[1].clone()
        inner(want).copy_(ahead ^ inner(f[1]) ^ inner(f[2]))
        launch(f[0], f[1], None, False)
        torch.cuda.synchronize()
        ok = torch.equal(f[1], want)
        del want
    del ahead
    if not ok:
        raise RuntimeError("16-bit step-stream probe computed a wrong result")
    bpp = 10 if uv else 8
    out = {"form": "u and step change" if uv else "two levels", "bytes_per_point": bpp, "nx": nx, "ny": ny,
           "nz": nz, "zchunk": zc, "tile": f"t128x{ty * ry}_r{ry}", "launches": launches}
    for name, alternate in (("ascending", False), ("alternating", True)):
        def seq(count):
            a, b = f[0], (f[3] if uv else f[1])
            for i in range(count):
                if uv:
                    launch(a, f[1], b, alternate and (i & 1))
                else:
                    launch(a, b, None, alternate and (i & 1))
                a, b = b, a
        seq(4)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        seq(launches)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / launches
        out[f"{name}_gbs"] = round(bpp * nx * ny * nz / sec / 1e9, 1)
        out[f"{name}_us"] = round(sec * 1e6, 2)
    del f
    return out


def measure_adjoint_stream(nx: int, ny: int, nz: int, zc: int, ty: int = 16, launches: int = 20) -> dict:
    """The fused adjoint step's access pattern without its arithmetic: GB/s
    at 36 bytes per interior cell, launches swapping the two wave fields,
    all marching up and alternating direction; tiles of 128 cells x ty rows
    and z-chunks of zc planes, as the adjoint kernel tiles the grid."""
    lib = _load()
    x0 = 32
    pitch = -(-(x0 + nx + 4) // 32) * 32
    elems = pitch * (ny + 8) * (nz + 8)
    f = [torch.randint(-2 ** 31, 2 ** 31 - 1, (elems,), dtype=torch.int32, device="cuda") for _ in range(4)]
    g = torch.randint(-2 ** 31, 2 ** 31 - 1, (2 * elems,), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream

    def launch(c, p, down):
        rc = lib.probe_adjoint_stream(c.data_ptr(), f[2].data_ptr(), p.data_ptr(), f[3].data_ptr(), g.data_ptr(),
                                      nx, ny, nz, pitch, x0, zc, ty, int(down), s)
        if rc != 0:
            raise RuntimeError(f"probe_adjoint_stream failed (code {rc})")

    # one launch checked against its definition over the whole fields
    view = lambda t, w=1: t.view(nz + 8, ny + 8, w * pitch)
    inner = lambda t, dz=0: view(t)[4 + dz:4 + dz + nz, 4:4 + ny, x0:x0 + nx]
    c4, a4 = inner(f[0], 4), inner(f[2], 4)
    want_p, want_g = f[1].clone(), g.clone()
    inner(want_p).copy_(c4 ^ a4 ^ inner(f[1]) ^ inner(f[3]))
    gi = view(want_g, 2)[4:4 + nz, 4:4 + ny, 2 * x0:2 * (x0 + nx)].reshape(nz, ny, nx // 4, 8)
    gi[..., :4] ^= c4.reshape(nz, ny, nx // 4, 4)
    gi[..., 4:] ^= a4.reshape(nz, ny, nx // 4, 4)
    launch(f[0], f[1], False)
    torch.cuda.synchronize()
    ok = torch.equal(f[1], want_p) and torch.equal(g, want_g)
    del want_p, want_g, gi, c4, a4
    if not ok:
        raise RuntimeError("adjoint-stream probe computed a wrong result")
    out = {"bytes_per_point": 36, "nx": nx, "ny": ny, "nz": nz, "zchunk": zc, "tile": f"t128x{ty}_r1",
           "launches": launches}
    for name, alternate in (("ascending", False), ("alternating", True)):
        def seq(count):
            a, b = f[0], f[1]
            for i in range(count):
                launch(a, b, alternate and (i & 1))
                a, b = b, a
        seq(4)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        seq(launches)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / launches
        out[f"{name}_gbs"] = round(36 * nx * ny * nz / sec / 1e9, 1)
        out[f"{name}_us"] = round(sec * 1e6, 2)
    del f, g
    return out


def measure_sync(nsteps: int = 2000) -> dict:
    """Microseconds per step of synchronising all work-groups of one
    cooperative launch (a grid barrier, or waits for two ring neighbours),
    at one and two 256-thread work-groups per CU, against the cost of an
    empty launch of as many work-groups."""
    lib = _load()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    out = {"steps": nsteps}
    for per in (1, 2):
        blocks = per * cus
        words = torch.zeros(4 + blocks, dtype=torch.int32, device="cuda")
        for ring, name in ((0, "grid_barrier"), (1, "neighbour_flags")):
            words.zero_()
            torch.cuda.synchronize()

            def run():
                rc = lib.probe_sync(words.data_ptr(), blocks, nsteps, ring, 10.0, s)
                if rc != 0:
                    raise RuntimeError(f"probe_sync failed (code {rc})")

            us = timed(run, 1) / nsteps
            if int(words[2].item()):
                raise RuntimeError("probe_sync: a wait gave up")
            out[f"{name}_us_{per}wg_per_cu"] = round(us, 3)

        def empty():
            if lib.probe_empty(blocks, s) != 0:
                raise RuntimeError("probe_empty failed")

        empty()
        out[f"empty_launch_us_{per}wg_per_cu"] = round(timed(empty, nsteps), 3)
    return out


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
    if len(sys.argv) == 6 and sys.argv[1] == "step-stream":
        # python -m paper_2204_03775_amd.probe step-stream NX NY NZ ZC
        nx, ny, nz, zc = (int(v) for v in sys.argv[2:])
        print(json.dumps(measure_step_stream(nx, ny, nz, zc, launches=6)), flush=True)
        sys.exit(0)
    if len(sys.argv) > 1:
        n = int(sys.argv[1])
    else:
        sys.path.insert(0, os.path.dirname(_HERE))
        from paper_2204_03775_amd import wave

        n = wave.wave_layout(512, 512, 512).elems
    print(json.dumps(measure(n, with_adjoint_mix=True)), flush=True)
