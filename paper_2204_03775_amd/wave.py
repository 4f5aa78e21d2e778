"""ctypes binding of libwave.so (C ABI in include/wave.h).

Argument marshalling only: every step of the propagator runs in the HIP
kernels of libwave.so.  PyTorch supplies device memory and streams.  The
functions carry the C names; ``Propagator`` bundles the allocation of the
padded fields and the context for convenience.

The library must be built (``__graft_entry__.build()``); importing this
module raises ``ImportError`` if it is missing, so nothing can silently fall
back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime libwave.so resolves against (same soname)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwave.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "wave.h")

WAVE_OK = 0
WAVE_EINVAL = -1
WAVE_EUNSTABLE = -2
WAVE_ESTATE = -3
WAVE_ENOMEM = -4
WAVE_EHIP = -5
WAVE_F32 = 0
WAVE_F16 = 1
WAVE_BF16 = 2
WAVE_F16_UV = 3
WAVE_BF16_UV = 4
DTYPES = {"f32": WAVE_F32, "f16": WAVE_F16, "bf16": WAVE_BF16, "f16uv": WAVE_F16_UV,
          "bf16uv": WAVE_BF16_UV}
_TORCH_DTYPE = {WAVE_F32: torch.float32, WAVE_F16: torch.float16, WAVE_BF16: torch.bfloat16,
                WAVE_F16_UV: torch.float16, WAVE_BF16_UV: torch.bfloat16}

GHOST = 4


class WaveError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


class wave_layout_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("pitch_x", "rows", "planes", "x_offset", "plane", "elems", "bytes")]


class wave_params_t(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("sponge_width", ctypes.c_int32), ("sponge_alpha", ctypes.c_double),
                ("dtype", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    ci = ctypes.c_int
    sig = {
        "wave_layout": ([i32, i32, i32, i32, ctypes.POINTER(wave_layout_t)], ci),
        "wave_init": ([ctypes.POINTER(vp), ctypes.POINTER(wave_params_t), vp, vp, vp,
                       ctypes.POINTER(i32), ctypes.POINTER(i32), i32, vp], ci),
        "wave_record": ([vp, vp, i32], ci),
        "wave_step": ([vp, f32], ci),
        "wave_run": ([vp, i32, vp], ci),
        "wave_fields": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64)], ci),
        "wave_export": ([vp, i32, vp], ci),
        "wave_reset": ([vp], ci),
        "wave_set_stream": ([vp, vp], ci),
        "wave_configure": ([vp, i32, i32], ci),
        "wave_variant_count": ([], i32),
        "wave_variant_name": ([i32], ctypes.c_char_p),
        "wave_config": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], ci),
        "wave_sync": ([vp], ci),
        "wave_destroy": ([vp], ci),
        "wave_forward_checkpointed": ([vp, i32, vp, i32], ci),
        "wave_adjoint": ([vp, vp, vp, i32], ci),
        "wave_adjoint_velocity": ([vp, vp, vp, ctypes.c_double, i32, vp, i32], ci),
        "wave_velocity_to_k": ([vp, i64, ctypes.c_double, vp, vp], ci),
        "wave_set_adjoint_fusion": ([vp, i32], ci),
        "wave_set_graph": ([vp, i32], ci),
        "wave_check": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], ci),
        "wave_check_noalloc": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], ci),
        "wave_grad_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                            ctypes.POINTER(i64)], ci),
        "wave_misfit": ([vp, vp, i64, vp, vp, vp], ci),
        "wave_batch_create": ([ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, i32], ci),
        "wave_batch_run": ([vp, i32, ctypes.POINTER(vp)], ci),
        "wave_batch_set_schedule": ([vp, i32, i32], ci),
        "wave_batch_set_wait_limit": ([vp, i32], ci),
        "wave_batch_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)], ci),
        "wave_batch_sync": ([vp], ci),
        "wave_batch_destroy": ([vp], ci),
        "wave_batch_last_error": ([vp], ctypes.c_char_p),
        "wave_strerror": ([ci], ctypes.c_char_p),
        "wave_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc: int, ctx=None):
    if rc != WAVE_OK:
        msg = _lib.wave_strerror(rc).decode()
        if ctx:
            detail = _lib.wave_last_error(ctx).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise WaveError(rc, msg)


# --- the C functions, one for one -------------------------------------------

def wave_layout(nx: int, ny: int, nz: int, dtype: int = WAVE_F32) -> wave_layout_t:
    out = wave_layout_t()
    _check(_lib.wave_layout(nx, ny, nz, dtype, ctypes.byref(out)))
    return out


def _zyx_array(pts):
    import numpy as np

    a = np.ascontiguousarray(np.asarray(pts, dtype=np.int32).reshape(-1, 3))
    return a, (ctypes.c_int32 * a.size)(*a.ravel().tolist())


def wave_init(params: wave_params_t, k_ptr: int, cur_ptr: int, prev_ptr: int, src=None,
              rec=None, stream: int | None = None):
    ctx = ctypes.c_void_p()
    src_buf = (ctypes.c_int32 * 3)(*[int(v) for v in src]) if src is not None else None
    nrec = 0
    rec_buf = None
    if rec is not None:
        arr, rec_buf = _zyx_array(rec)
        nrec = arr.shape[0]
        if nrec == 0:
            rec_buf = None
    rc = _lib.wave_init(ctypes.byref(ctx), ctypes.byref(params), k_ptr, cur_ptr, prev_ptr,
                        src_buf, rec_buf, nrec, stream)
    _check(rc)
    return ctx


def wave_record(ctx, traces_ptr, nt_capacity: int):
    _check(_lib.wave_record(ctx, traces_ptr, nt_capacity), ctx)


def wave_step(ctx, src_value: float):
    _check(_lib.wave_step(ctx, src_value), ctx)


def wave_run(ctx, nsteps: int, src_ptr=None):
    _check(_lib.wave_run(ctx, nsteps, src_ptr), ctx)


def wave_fields(ctx):
    cur, prev, step = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
    _check(_lib.wave_fields(ctx, ctypes.byref(cur), ctypes.byref(prev), ctypes.byref(step)), ctx)
    return cur.value, prev.value, step.value


def wave_export(ctx, which: int, dst_ptr: int):
    _check(_lib.wave_export(ctx, which, dst_ptr), ctx)


def wave_reset(ctx):
    _check(_lib.wave_reset(ctx), ctx)


def wave_set_stream(ctx, stream):
    _check(_lib.wave_set_stream(ctx, stream), ctx)


def wave_configure(ctx, variant: int = 0, zchunk: int = 0):
    _check(_lib.wave_configure(ctx, variant, zchunk), ctx)


def wave_variant_count() -> int:
    return _lib.wave_variant_count()


def wave_variant_name(v: int):
    r = _lib.wave_variant_name(v)
    return r.decode() if r is not None else None


def wave_config(ctx):
    v, zc, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.wave_config(ctx, ctypes.byref(v), ctypes.byref(zc), ctypes.byref(wg)), ctx)
    return v.value, zc.value, wg.value


def wave_sync(ctx):
    _check(_lib.wave_sync(ctx), ctx)


def wave_destroy(ctx):
    _check(_lib.wave_destroy(ctx))


def wave_forward_checkpointed(ctx, nt: int, src_ptr=None, every: int = 0):
    _check(_lib.wave_forward_checkpointed(ctx, nt, src_ptr, every), ctx)


def wave_adjoint(ctx, trace_grad_ptr, grad_ptr, accumulate: bool = False):
    _check(_lib.wave_adjoint(ctx, trace_grad_ptr, grad_ptr, int(bool(accumulate))), ctx)


def wave_adjoint_velocity(ctx, trace_grad_ptr, v_ptr, dt: float, source_scales_with_k: bool,
                          grad_v_ptr, accumulate: bool = False):
    _check(_lib.wave_adjoint_velocity(ctx, trace_grad_ptr, v_ptr, float(dt), int(bool(source_scales_with_k)),
                                      grad_v_ptr, int(bool(accumulate))), ctx)


def wave_velocity_to_k(v_ptr, n: int, dt: float, k_ptr, stream):
    _check(_lib.wave_velocity_to_k(v_ptr, int(n), float(dt), k_ptr, stream))


def wave_check(ctx):
    f, t = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.wave_check(ctx, ctypes.byref(f), ctypes.byref(t)), ctx)
    return f.value, t.value


def wave_check_noalloc(ctx):
    f, t = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.wave_check_noalloc(ctx, ctypes.byref(f), ctypes.byref(t)), ctx)
    return f.value, t.value


def wave_set_graph(ctx, on: bool):
    _check(_lib.wave_set_graph(ctx, int(bool(on))), ctx)


def wave_set_adjoint_fusion(ctx, on: bool):
    _check(_lib.wave_set_adjoint_fusion(ctx, int(bool(on))), ctx)


def wave_grad_info(ctx):
    nt, every, seg, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.wave_grad_info(ctx, ctypes.byref(nt), ctypes.byref(every), ctypes.byref(seg),
                               ctypes.byref(nb)), ctx)
    return nt.value, every.value, seg.value, nb.value


def wave_misfit(traces_ptr, observed_ptr, n: int, residual_ptr, misfit_ptr, stream):
    _check(_lib.wave_misfit(traces_ptr, observed_ptr, n, residual_ptr, misfit_ptr, stream))


def wave_strerror(code: int) -> str:
    return _lib.wave_strerror(code).decode()


def wave_last_error(ctx) -> str:
    return _lib.wave_last_error(ctx).decode()


def _bcheck(rc: int, b=None):
    if rc != WAVE_OK:
        msg = _lib.wave_strerror(rc).decode()
        if b:
            detail = _lib.wave_batch_last_error(b).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise WaveError(rc, msg)


def wave_batch_create(ctxs, stream, use_graph: bool = True):
    b = ctypes.c_void_p()
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    _bcheck(_lib.wave_batch_create(ctypes.byref(b), arr, len(ctxs), stream, int(bool(use_graph))))
    return b


def wave_batch_run(b, nsteps: int, src_ptrs=None):
    arr = None
    if src_ptrs is not None:
        arr = (ctypes.c_void_p * len(src_ptrs))(*[p or None for p in src_ptrs])
    _bcheck(_lib.wave_batch_run(b, nsteps, arr), b)


def wave_batch_set_schedule(b, schedule: int, nstreams: int = 1):
    _bcheck(_lib.wave_batch_set_schedule(b, int(schedule), int(nstreams)), b)


def wave_batch_set_wait_limit(b, polls: int):
    _bcheck(_lib.wave_batch_set_wait_limit(b, int(polls)), b)


def wave_batch_info(b):
    g, wg, pts = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    _bcheck(_lib.wave_batch_info(b, ctypes.byref(g), ctypes.byref(wg), ctypes.byref(pts)), b)
    return g.value, wg.value, pts.value


def wave_batch_sync(b):
    _bcheck(_lib.wave_batch_sync(b), b)


def wave_batch_destroy(b):
    _bcheck(_lib.wave_batch_destroy(b))


def _indexed(device) -> torch.device:
    """``device`` with its index made explicit ("cuda" -> "cuda:<current>")."""
    d = torch.device(device)
    return torch.device(d.type, torch.cuda.current_device()) if d.type == "cuda" and d.index is None else d


def _device_f32(t, n: int, what: str, device) -> int:
    """Pointer of a contiguous FP32 tensor on ``device`` holding at least
    ``n`` values.  The library trusts the caller for the length of arrays
    it reads, so a short one is refused here (explicitly, not by assert)."""
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{what}: a contiguous FP32 device tensor is required")
    if device is not None and t.device != _indexed(device):
        raise ValueError(f"{what}: on {t.device}, the fields are on {device}")
    if t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} values, {n} needed")
    return t.data_ptr()


def variants() -> dict:
    return {wave_variant_name(i): i for i in range(wave_variant_count())}


# --- convenience wrapper ----------------------------------------------------

class Propagator:
    """Fields in the library's padded layout (torch tensors on the current
    device) plus a context.  ``k`` is a dense [nz][ny][nx] array (numpy or
    torch) of V^2 dt^2, rounded to FP32 once.  ``dtype`` selects the field
    storage: "f32"; "f16" / "bf16" (two 16-bit time levels, FP32
    arithmetic); "f16uv" / "bf16uv" (16-bit u^n and step change d^n, the
    latter held by the library).  ``u_cur`` / ``u_prev`` (dense, FP32
    storage only) give the state to start from, e.g. to resume a run."""

    def __init__(self, nx, ny, nz, h, k, *, src=None, rec=None, sponge_width=0,
                 sponge_alpha=0.0, stream=None, device=None, dtype="f32", u_cur=None,
                 u_prev=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.h = tuple(float(v) for v in h)
        self.device = _indexed(device if device is not None else "cuda")
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.layout = wave_layout(self.nx, self.ny, self.nz, self.dtype)
        self.layout32 = wave_layout(self.nx, self.ny, self.nz, WAVE_F32)
        n = self.layout.elems
        tdt = _TORCH_DTYPE[self.dtype]
        # FP32 k in the FP32 layout; with 16-bit storage the library encodes
        # its own copy at init and this one is released afterwards
        self.k = torch.zeros(self.layout32.elems, dtype=torch.float32, device=self.device)
        self.buf = [torch.zeros(n, dtype=tdt, device=self.device),
                    torch.zeros(n, dtype=tdt, device=self.device)]
        self.interior(self.k).copy_(torch.as_tensor(k).to(device=self.device, dtype=torch.float32))
        if u_cur is not None or u_prev is not None:
            # a state to resume from (the library starts 16-bit fields from zero)
            if self.dtype != WAVE_F32:
                raise ValueError("initial fields are supported for FP32 storage only")
            for b, u in zip(self.buf, (u_cur, u_prev)):
                if u is not None:
                    self.interior(b).copy_(torch.as_tensor(u).to(device=self.device, dtype=torch.float32))
        self.src = tuple(int(v) for v in src) if src is not None else None
        self.rec = rec
        self.nrec = 0 if rec is None else len(rec)
        p = wave_params_t(self.nx, self.ny, self.nz, self.h[0], self.h[1], self.h[2],
                          int(sponge_width), float(sponge_alpha), self.dtype)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = wave_init(p, self.k.data_ptr(), self.buf[0].data_ptr(), self.buf[1].data_ptr(),
                             self.src, rec, self.stream.cuda_stream)
        if self.dtype != WAVE_F32:
            self.k = None
        self.traces = None

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz

    # layout helpers (views, no copies)
    def _layout_of(self, buf):
        return self.layout32 if buf.dtype == torch.float32 else self.layout

    def padded(self, buf):
        L = self._layout_of(buf)
        return buf.view(L.planes, L.rows, L.pitch_x)

    def interior(self, buf):
        L = self._layout_of(buf)
        x0 = L.x_offset
        return self.padded(buf)[GHOST:GHOST + self.nz, GHOST:GHOST + self.ny, x0:x0 + self.nx]

    def export(self, which: int = 0):
        """u^n (which=0) or u^{n-1} (which=1) decoded to FP32, as a dense
        [nz][ny][nx] tensor (device)."""
        out = torch.zeros(self.layout32.elems, dtype=torch.float32, device=self.device)
        wave_export(self.ctx, int(which), out.data_ptr())
        return self.interior(out)

    def _by_ptr(self, ptr):
        for b in self.buf:
            if b.data_ptr() == ptr:
                return b
        raise RuntimeError("library reported an unknown field pointer")

    def fields(self):
        """(u^n, u^{n-1}, n): padded tensors in their current roles."""
        cur, prev, step = wave_fields(self.ctx)
        return self._by_ptr(cur), self._by_ptr(prev), step

    def record(self, nt_capacity: int):
        self.traces = torch.zeros((nt_capacity, max(self.nrec, 1)), dtype=torch.float32,
                                  device=self.device)
        wave_record(self.ctx, self.traces.data_ptr(), nt_capacity)
        return self.traces

    def step(self, src_value: float = 0.0):
        wave_step(self.ctx, float(src_value))

    def run(self, nsteps: int, src=None):
        """``src``: device FP32 tensor with >= nsteps values, or None."""
        ptr = None if src is None else _device_f32(src, int(nsteps), "src", self.device)
        wave_run(self.ctx, int(nsteps), ptr)

    def forward_checkpointed(self, nt: int, src=None, every: int = 0):
        """``run`` that also keeps what ``adjoint`` needs (checkpoints every
        ``every`` steps; 0 lets the library choose)."""
        ptr = None if src is None else _device_f32(src, int(nt), "src", self.device)
        wave_forward_checkpointed(self.ctx, int(nt), ptr, int(every))

    def adjoint(self, trace_grad=None, grad=None, accumulate: bool = False):
        """dJ/dk (FP64 [nz][ny][nx] device tensor) of the last checkpointed
        run, for ``trace_grad`` = dJ/d traces ([nt][nrec] FP32 device)."""
        ptr = None
        if self.nrec > 0:
            if trace_grad is None:
                raise ValueError("trace_grad is required when the shot has receivers")
            nt = wave_grad_info(self.ctx)[0]  # 0 without a run: the library reports it
            ptr = _device_f32(trace_grad, nt * self.nrec, "trace_grad", self.device)
            if nt and tuple(trace_grad.shape) != (nt, self.nrec):
                raise ValueError(f"trace_grad: shape {tuple(trace_grad.shape)}, expected {(nt, self.nrec)}")
        if grad is None:
            grad = torch.zeros((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
            accumulate = False
        if not (grad.dtype == torch.float64 and grad.is_cuda and grad.is_contiguous()
                and grad.device == self.device and tuple(grad.shape) == (self.nz, self.ny, self.nx)):
            raise ValueError(f"grad: a contiguous FP64 [{self.nz}][{self.ny}][{self.nx}] tensor on "
                             f"{self.device} is required")
        wave_adjoint(self.ctx, ptr, grad.data_ptr(), accumulate)
        return grad

    def adjoint_velocity(self, trace_grad, v, dt: float, source_scales_with_v: bool = False, grad=None,
                         accumulate: bool = False):
        """dJ/dv (FP64 [nz][ny][nx] device tensor) of the last checkpointed
        run, for a context whose k was made from ``v`` (dense FP32 device)
        as (v dt)^2; ``source_scales_with_v``: the source values were made
        with the velocity at the source cell (see wave_adjoint_velocity)."""
        ptr = None
        if self.nrec > 0:
            if trace_grad is None:
                raise ValueError("trace_grad is required when the shot has receivers")
            nt = wave_grad_info(self.ctx)[0]
            ptr = _device_f32(trace_grad, nt * self.nrec, "trace_grad", self.device)
        vptr = _device_f32(v, self.points, "v", self.device)
        if grad is None:
            grad = torch.zeros((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
            accumulate = False
        if not (grad.dtype == torch.float64 and grad.is_cuda and grad.is_contiguous()
                and grad.device == self.device and tuple(grad.shape) == (self.nz, self.ny, self.nx)):
            raise ValueError(f"grad: a contiguous FP64 [{self.nz}][{self.ny}][{self.nx}] tensor on "
                             f"{self.device} is required")
        wave_adjoint_velocity(self.ctx, ptr, vptr, dt, source_scales_with_v, grad.data_ptr(), accumulate)
        return grad

    def grad_info(self):
        """(steps, segment length, segments, checkpoint bytes) of the last
        checkpointed run."""
        return wave_grad_info(self.ctx)

    def check(self):
        """(non-finite values in u^n, non-finite trace values so far)."""
        return wave_check(self.ctx)

    def use_graph(self, on: bool = True):
        """Replay repeated runs from a captured HIP graph (needs a
        non-default stream)."""
        wave_set_graph(self.ctx, on)

    def configure(self, variant=0, zchunk=0):
        if isinstance(variant, str):
            variant = variants()[variant]
        wave_configure(self.ctx, variant, zchunk)

    def config(self):
        return wave_config(self.ctx)

    def reset(self, zero_fields: bool = True):
        wave_reset(self.ctx)
        if zero_fields:
            for b in self.buf:
                b.zero_()
            if self.traces is not None:
                self.traces.zero_()

    def sync(self):
        wave_sync(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            wave_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several Propagators advanced together by one launch per step (per
    group of shots sharing a kernel), optionally replayed from a HIP graph.
    ``stream`` must be a non-default torch stream when ``use_graph``."""

    def __init__(self, props, stream=None, use_graph: bool = True):
        self.props = list(props)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.props[0].device)
        self.handle = wave_batch_create([p.ctx for p in self.props], self.stream.cuda_stream, use_graph)

    def set_schedule(self, schedule: int, nstreams: int = 1):
        """0: one persistent launch per step and kernel group; 1: every
        shot with its own kernel on ``nstreams`` streams; 2: switched off
        (the library refuses it); 3: one cooperative launch per kernel
        group for the whole run, a grid barrier between steps."""
        wave_batch_set_schedule(self.handle, schedule, nstreams)
        self.schedule, self.nstreams = int(schedule), int(nstreams)

    def set_wait_limit(self, polls: int):
        """Schedule 2: polls before a dependency wait gives up (negative:
        every wait after the first step gives up, to test that path)."""
        wave_batch_set_wait_limit(self.handle, polls)

    def info(self):
        """(launch groups, work-groups per step, interior points per step)"""
        return wave_batch_info(self.handle)

    def run(self, nsteps: int, srcs=None):
        """``srcs``: one device FP32 tensor (or None) per shot."""
        ptrs = None
        if srcs is not None:
            ptrs = []
            for t in srcs:
                if t is None:
                    ptrs.append(None)
                else:
                    ptrs.append(_device_f32(t, int(nsteps), "srcs", self.props[0].device))
        # order against work on the caller's current stream both ways
        # (field resets before, reads after)
        cur = torch.cuda.current_stream(self.props[0].device)
        self.stream.wait_stream(cur)
        wave_batch_run(self.handle, int(nsteps), ptrs)
        cur.wait_stream(self.stream)

    def sync(self):
        wave_batch_sync(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            wave_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def misfit(traces, observed, stream=None):
    """(0.5 sum (traces - observed)^2 as an FP64 device scalar, FP32
    residual traces - observed), both computed by the library."""
    if traces.shape != observed.shape:
        raise ValueError(f"traces {tuple(traces.shape)} and observed {tuple(observed.shape)} differ")
    _device_f32(traces, traces.numel(), "traces", None)
    _device_f32(observed, traces.numel(), "observed", traces.device)
    stream = stream if stream is not None else torch.cuda.current_stream(traces.device)
    out = torch.empty((), dtype=torch.float64, device=traces.device)
    res = torch.empty_like(traces)
    wave_misfit(traces.data_ptr(), observed.data_ptr(), traces.numel(), res.data_ptr(),
                out.data_ptr(), stream.cuda_stream)
    return out, res


class Survey:
    """Everything of a shot except the model: grid spacing, time step,
    steps, source position and values, receivers, sponge, checkpoint
    interval (0: library's choice).  ``source_scales_with_v``: the source
    values were made with the velocity at the source cell (Eq. 2's
    dt^2 V^2 f^n, as the workload generators make them), so the gradient
    includes their dependence on it; otherwise they are held fixed."""

    def __init__(self, h, dt, nt, src, src_values, rec, sponge_width=0, sponge_alpha=0.0,
                 every=0, source_scales_with_v=False):
        self.h = tuple(float(v) for v in h)
        self.dt = float(dt)
        self.nt = int(nt)
        self.src = tuple(int(v) for v in src) if src is not None else None
        self.src_values = src_values
        self.rec = rec
        self.sponge_width = int(sponge_width)
        self.sponge_alpha = float(sponge_alpha)
        self.every = int(every)
        self.source_scales_with_v = bool(source_scales_with_v)


class _TracesOfVelocity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, survey):
        nz, ny, nx = v.shape
        vv = v.detach().to(torch.float32).contiguous()
        k = torch.empty_like(vv)
        stream = torch.cuda.current_stream(vv.device)
        wave_velocity_to_k(vv.data_ptr(), vv.numel(), survey.dt, k.data_ptr(), stream.cuda_stream)
        prop = Propagator(nx, ny, nz, survey.h, k, src=survey.src, rec=survey.rec,
                          sponge_width=survey.sponge_width, sponge_alpha=survey.sponge_alpha,
                          device=v.device)
        prop.record(survey.nt)
        src = survey.src_values
        if src is not None:
            src = torch.as_tensor(src, dtype=torch.float32).to(v.device).contiguous()
        prop.forward_checkpointed(survey.nt, src, survey.every)
        ctx.prop = prop
        ctx.survey = survey
        ctx.v = vv
        ctx.v_dtype = v.dtype
        return prop.traces[:, :prop.nrec].clone()

    @staticmethod
    def backward(ctx, g):
        prop, survey = ctx.prop, ctx.survey
        g = g.to(torch.float32).contiguous()
        grad_v = prop.adjoint_velocity(g if prop.nrec else None, ctx.v, survey.dt, survey.source_scales_with_v)
        prop.close()
        ctx.prop = None
        return grad_v.to(ctx.v_dtype), None


def traces_of_velocity(v, survey: Survey):
    """Receiver traces [nt][nrec] of the shot ``survey`` in the velocity
    model ``v`` (dense [nz][ny][nx] device tensor), differentiable with
    respect to ``v`` through the library's adjoint run (k = (v dt)^2)."""
    return _TracesOfVelocity.apply(v, survey)
